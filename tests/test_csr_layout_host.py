"""The closed-form CSR row offsets used by the device-side assembly of the
matrix-explicit comparator equal the row pointers of the oracle's assembled
matrix (same cell order, same neighbour sets).  Host only: the header is
compiled with g++."""
import os
import subprocess

import numpy as np
import pytest

import oracle

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))

PROG = r'''
#include <cstdio>
#include "csr_layout.h"
int main(int argc, char** argv) {
    long nx = atol(argv[1]), ny = atol(argv[2]), nz = atol(argv[3]);
    int px = atoi(argv[4]), py = atoi(argv[5]);
    for (long i = 0; i < nx; ++i) for (long j = 0; j < ny; ++j) for (long k = 0; k < nz; ++k)
        printf("%ld\n", (long)pcg::csr::row_offset(nx, ny, nz, px, py, i, j, k));
    printf("%ld\n", (long)pcg::csr::total_nnz(nx, ny, nz, px, py));
    return 0;
}
'''


@pytest.fixture(scope="module")
def exe(tmp_path_factory):
    d = tmp_path_factory.mktemp("csr")
    src = d / "rows.cpp"
    src.write_text("#include <cstdlib>\n" + PROG)
    out = d / "rows"
    subprocess.check_call(["g++", "-std=c++17", "-O1",
                           "-I" + os.path.join(ROOT, "paper_1302_7193_amd", "csrc"),
                           str(src), "-o", str(out)])
    return str(out)


@pytest.mark.parametrize("shape", [(5, 4, 6, 0, 0), (3, 3, 7, 1, 1), (6, 5, 1, 0, 1),
                                   (1, 1, 9, 0, 0), (1, 7, 4, 0, 0), (4, 1, 3, 1, 0),
                                   (2, 2, 2, 0, 0), (8, 3, 2, 1, 0)])
def test_closed_form_row_offsets_equal_oracle_row_pointers(exe, shape):
    nx, ny, nz, px, py = shape
    got = np.array(subprocess.check_output([exe] + [str(v) for v in shape]).split(), dtype=np.int64)
    g = oracle.Grid(nx, ny, nz, 1.0 / nx, 1.0 / ny, 1.0, 1.05, 1.0, 10.0, bool(px), bool(py))
    A = oracle.assemble(g)
    np.testing.assert_array_equal(got, A.row_ptr)
