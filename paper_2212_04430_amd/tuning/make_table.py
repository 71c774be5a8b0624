"""Regenerate the stencil tuning table for the GPU this runs on.

    python -m paper_2212_04430_amd.tuning.make_table OUT [--dims 16 16 16 32] [--batch 432]

For each storage precision, fs_autotune times every stencil configuration
(rhs block, work-group size, variant, residency cap) on a synthetic gauge
field of the given extent, and appends the fastest one to OUT:
* FP32, FP16 and BF16 at the batch size of a batched estimate;
* FP64 at one system, the configuration of the plain single-system path.
Existing lines for the same key are reused, not re-timed, so start from an
empty file to re-tune.
"""

import argparse
import os
import sys

HERE = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, os.path.dirname(os.path.dirname(HERE)))

import synth  # noqa: E402
from paper_2212_04430_amd import _lib as L  # noqa: E402


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("out")
    ap.add_argument("--dims", type=int, nargs=4, default=[16, 16, 16, 32])
    ap.add_argument("--batch", type=int, default=432)
    ap.add_argument("--eps", type=float, default=0.2)
    a = ap.parse_args()
    ctx = L.fs_create(tuple(a.dims), 0, 0)
    try:
        L.fs_upload_gauge(ctx, synth.gauge_field(tuple(a.dims), eps=a.eps, seed=0))
        for prec, n_sys in (("f32", a.batch), ("f16", a.batch), ("bf16", a.batch), ("f64", 1)):
            nr, wg = L.fs_autotune(ctx, prec, n_sys, a.out)
            print(f"{prec} n_sys={n_sys}: rhs_block={nr} wg={wg}", flush=True)
    finally:
        L.fs_destroy(ctx)


if __name__ == "__main__":
    main()
