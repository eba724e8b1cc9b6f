"""The HBM probe kernel (pcg_stream_probe) through the C ABI: every access
mix the bench times writes out_k = sum_i in_i * 2^-(i+k) exactly (power-of-two
coefficients, so the sums are exact in the order written and the check is
bitwise), on ragged sizes and with few workgroups (several strips each)."""
import numpy as np
import pytest

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")
if not torch.cuda.is_available():
    pytest.skip("no GPU", allow_module_level=True)

import paper_1302_7193_amd as pcg  # noqa: E402
import synth_inputs as si  # noqa: E402


@pytest.mark.parametrize("nr,nw", [(1, 1), (2, 2), (4, 3), (3, 1)])
@pytest.mark.parametrize("nt", [0, 1, 2, 3])
@pytest.mark.parametrize("blocks", [0, 3])
def test_probe_writes_its_linear_map(nr, nw, nt, blocks):
    n = 2 * 12345                       # FP64 values: 12345 16-byte elements
    ins = [si.uniform_pm1(900 + i, n) for i in range(nr)]
    reads = [torch.from_numpy(v).cuda() for v in ins]
    writes = [torch.full((n,), float("nan"), dtype=torch.float64, device="cuda") for _ in range(nw)]
    pcg.pcg_stream_probe(reads, writes, nontemporal=nt, blocks=blocks)
    torch.cuda.synchronize()
    for k, w in enumerate(writes):
        want = np.zeros(n)
        for i, v in enumerate(ins):
            want = want + np.ldexp(1.0, -(i + k)) * v
        np.testing.assert_array_equal(w.cpu().numpy(), want)
