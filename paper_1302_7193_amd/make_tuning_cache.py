"""Regenerate the launch-shape tuning cache on the GPU at hand.

Runs pcg_autotune for the workload shapes the benchmark and the tests use
(the 512x512x128 periodic FP64 workload, plain and on a stretched grid; the
64x64x32 latency case; 1024x1024x128 in both precisions; 64 batched
256x256x64 right-hand sides; square grids 64..512 x 32..128 in both
precisions) and writes the table with pcg_tuning_cache_save.

    python -m paper_1302_7193_amd.make_tuning_cache OUT.txt

Start it with PCG_TUNING_CACHE set to an empty string so that no cached entry
is loaded and every shape is timed afresh.  Copy OUT.txt over
paper_1302_7193_amd/tuning_cache.txt to make it the default.
"""
from __future__ import annotations

import argparse
import time

import paper_1302_7193_amd as pcg
import synth_inputs as si

F64, F32 = pcg.PCG_F64, pcg.PCG_F32


def jobs():
    """((nx, ny, nz, anisotropy, bc), dtype, nrhs, stretched) to tune."""
    out = [((512, 512, 128, 1e5, 1), F64, 1, False),
           ((64, 64, 32, 1e5, 1), F64, 1, False),
           ((1024, 1024, 128, 1e4, 1), F64, 1, False),
           ((1024, 1024, 128, 1e4, 1), F32, 1, False),
           ((256, 256, 64, 1e3, 1), F32, 64, False),
           ((256, 256, 64, 1e3, 1), F64, 64, False)]
    for n in (64, 128, 256, 512):
        for nz in (32, 64, 128):
            for dt in (F64, F32):
                out.append(((n, n, nz, 1e3, 0), dt, 1, False))
    out.append(((512, 512, 128, 1e5, 1), F64, 1, True))
    return out


def main():
    ap = argparse.ArgumentParser(description=__doc__.split("\n")[0])
    ap.add_argument("out", help="file to write the tuning table to")
    args = ap.parse_args()
    for (nx, ny, nz, g2, bc), dt, nrhs, stretched in jobs():
        d = pcg.pcg_desc_from_ratio(nx, ny, nz, 1.05, g2, bc)
        if stretched:
            p = pcg.Problem(d, si.widths_sine(nx, 0.5), si.widths_sine(ny, 0.25))
        else:
            p = pcg.Problem(d)
        t0 = time.time()
        t = pcg.pcg_autotune(p, dt, nrhs)
        print(nx, ny, nz, "f64" if dt == F64 else "f32", nrhs,
              "stretched" if stretched else "uniform", t.as_dict(),
              "%.1fs" % (time.time() - t0), flush=True)
        del p
    pcg.pcg_tuning_cache_save(args.out)
    print(open(args.out).read())


if __name__ == "__main__":
    main()
