"""Run single kernels of the path in the benchmark's launch shape, for profilers.

    python -m paper_1903_06986_amd.kernel_probe --kernel hop32 --nrhs 8 --reps 20

kernels: hop32 / hop64 (both parities of the stencil, internal even/odd
layout), schur32 / schur64 (the even/odd operator in FP32 / FP64), schur16 (the even/odd
operator reading FP16 per-site-scaled input, LEX in/out), copy (a plain
device copy of a 256 MiB buffer, the reference for scaling memory
counters).  --tile 0/1 switches the link-tiled stencil off/on.  The
lattice is the 24^3 x 32 workload's (links exp(i 0.2 H), seed 1003).
Prints the per-launch algorithmic bytes the library's timer assigns.
"""
import argparse
import os
import sys

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--kernel", default="hop32", choices=["hop32", "hop64", "schur32", "schur64", "schur16", "copy"])
    ap.add_argument("--tile", type=int, default=1)
    ap.add_argument("--order", type=int, default=0)
    ap.add_argument("--nb", type=int, default=0, help="lane-grouped right-hand sides (0: default)")
    ap.add_argument("--tblock", type=int, default=-1, help="plane-blocked tile order: timeslices per block (-1 auto, 0 index order)")
    ap.add_argument("--tsites", type=int, default=32, help="sites per tile (FP32: 16, 32 or 64; FP64: 16 or 32)")
    ap.add_argument("--rgroup", type=int, default=0, help="right-hand sides per group of the tiled stencil")
    ap.add_argument("--nrhs", type=int, default=8)
    ap.add_argument("--reps", type=int, default=20)
    ap.add_argument("--dims", default="24x24x24x32")
    a = ap.parse_args()
    import torch
    if a.kernel == "copy":
        src = torch.empty(256 << 20, dtype=torch.uint8, device="cuda").fill_(1)
        dst = torch.empty_like(src)
        for _ in range(a.reps):
            dst.copy_(src)
        torch.cuda.synchronize()
        print("copy: %d launches of %d bytes read + %d written" % (a.reps, src.numel(), src.numel()))
        return
    from paper_1903_06986_amd import Context
    from synth import random_su3_links
    dims = tuple(int(x) for x in a.dims.split("x"))
    U = random_su3_links(dims, 0.2, 1003)
    ctx = Context(dims, U, 0.13)
    ctx.tune(hop_tile64=a.tile, hop_tile32=a.tile, hop_order=a.order, hop_tblock64=a.tblock,
             hop_tblock32=a.tblock, hop_tsites32=a.tsites, hop_rgroup=a.rgroup,
             hop_tsites64=min(a.tsites, 32))
    if a.nb:
        ctx.tune(hop_nb64=a.nb, hop_nb32=a.nb)
    Vh = dims[0] * dims[1] * dims[2] * dims[3] // 2
    if a.kernel == "schur16":
        x = torch.randn((a.nrhs,) + ctx.shape, dtype=torch.complex128, device="cuda")
        y = torch.empty_like(x)
        ctx.timer(True)
        for _ in range(a.reps):
            ctx.wilson_apply("schur", x, prec="f16", out=y)
        kt = ctx.timer_read()
        ms, by, n = kt["hop32"]
        print("%s nrhs=%d tile=%d: %d stencil launches, %.1f us each, %.0f algorithmic bytes per launch, "
              "%.1f GB/s (order %d nb %d tblock %d tsites %d rgroup %d)" % (a.kernel, a.nrhs, a.tile, n, ms * 1e3 / n,
                                                    by / n, by / (ms * 1e-3) / 1e9, a.order, a.nb, a.tblock,
                                                    a.tsites, a.rgroup))
        return
    prec = "f64" if a.kernel in ("hop64", "schur64") else "f32"
    dt = torch.complex128 if prec == "f64" else torch.complex64
    op = "schur" if a.kernel.startswith("schur") else "hop"
    shape = (a.nrhs, 2, 12, Vh)  # even/odd layout; the Schur operator reads the even half
    x = torch.randn(shape, dtype=dt, device="cuda")
    y = torch.empty_like(x)
    ctx.timer(True)
    for _ in range(a.reps):
        ctx.wilson_apply(op, x, prec=prec, layout="eo", out=y)
    kt = ctx.timer_read()
    k = "hop64" if prec == "f64" else "hop32"
    ms, by, n = kt[k]
    print("%s nrhs=%d tile=%d order=%d nb=%d tblock=%d tsites=%d rgroup=%d: %d launches, %.1f us each, %.0f "
          "algorithmic bytes per launch, %.1f GB/s" % (a.kernel, a.nrhs, a.tile, a.order, a.nb, a.tblock, a.tsites,
                                                      a.rgroup, n, ms * 1e3 / n, by / n, by / (ms * 1e-3) / 1e9))


if __name__ == "__main__":
    main()
