"""GPU parity: Z(4) noise, even/odd packing and the Wilson operators.

Noise codes and the even/odd permutation are integer work and must match
the oracle bit for bit; FP64 operators agree to rounding (1e-13 relative
to the largest component), FP32 ones to 5e-6.  Lattices cover neighbour
aliasing (2^4), a ragged last block (6x4x2x8: V/2 = 192 sites), several
blocks (4^4 with 3 right-hand sides) and the 16^3 x 32 production shape.
"""
import numpy as np
import pytest

from tests.gpu_common import require_gpu, context, to_gpu, to_host, say, rel_err
from oracle import noise as ON
from oracle import wilson as W
from oracle import lattice as L

pytestmark = pytest.mark.gpu

DIMS = [(2, 2, 2, 2), (6, 4, 2, 8), (4, 4, 4, 4)]


@pytest.mark.parametrize("dims", DIMS + [(16, 16, 16, 32)])
def test_noise_bit_exact(dims):
    require_gpu()
    ctx, _ = context(dims, 0.3, 5, 0.12)
    for seed, first, n in ((2001, 0, 3), (0xDEADBEEFCAFEF00D, (1 << 33) + 7, 2)):
        say("noise", dims, seed, first)
        eta, codes = ctx.noise_z4(seed, first, n, codes=True)
        ref = ON.z4_codes(seed, dims, first, n)
        assert np.array_equal(to_host(codes), ref)
        assert np.array_equal(to_host(eta), ON.z4_noise(seed, dims, first, n))


@pytest.mark.parametrize("dims", DIMS)
def test_pack_matches_checkerboard_tables(dims):
    require_gpu()
    ctx, _ = context(dims, 0.3, 5, 0.12)
    rng = np.random.default_rng(1)
    shape = (2,) + ctx.shape
    x = rng.standard_normal(shape) + 1j * rng.standard_normal(shape)
    say("pack", dims)
    eo = to_host(ctx.pack_eo(to_gpu(x)))            # (nrhs, 2, 12, V/2)
    e, o = L.to_eo(dims, x)                          # (nrhs, V/2, 4, 3)
    assert np.array_equal(eo[:, 0], e.reshape(2, -1, 12).transpose(0, 2, 1))
    assert np.array_equal(eo[:, 1], o.reshape(2, -1, 12).transpose(0, 2, 1))
    back = to_host(ctx.unpack_eo(to_gpu(eo)))
    assert np.array_equal(back, x)


def _oracle_op(op, U, kappa, x, dims):
    if op == "M":
        return W.apply_M(U, kappa, x)
    if op == "Mdag":
        return W.apply_Mdag(U, kappa, x)
    if op == "MG5":
        return W.apply_Mprime(U, kappa, x)
    if op == "hop":
        return W.hop(U, x)
    if op == "schur":
        return W.apply_Mhat(U, kappa, x, dims)
    raise ValueError(op)


@pytest.mark.parametrize("dims", DIMS)
@pytest.mark.parametrize("op", ["M", "Mdag", "MG5", "hop", "schur"])
def test_operator_parity_fp64(dims, op):
    require_gpu()
    kappa = 0.13
    ctx, U = context(dims, 0.3, 7, kappa)
    rng = np.random.default_rng(3)
    shape = (3,) + ctx.shape
    x = rng.standard_normal(shape) + 1j * rng.standard_normal(shape)
    say("op", op, dims, "f64")
    y = to_host(ctx.wilson_apply(op, to_gpu(x)))
    ref = _oracle_op(op, U, kappa, x, dims)
    assert rel_err(y, ref) < 1e-13


@pytest.mark.parametrize("op", ["M", "hop", "schur", "MG5"])
def test_operator_parity_fp32(op):
    require_gpu()
    dims, kappa = (6, 4, 2, 8), 0.13
    ctx, U = context(dims, 0.3, 7, kappa)
    rng = np.random.default_rng(4)
    x = rng.standard_normal((2,) + ctx.shape) + 1j * rng.standard_normal((2,) + ctx.shape)
    say("op", op, dims, "f32")
    y = to_host(ctx.wilson_apply(op, to_gpu(x), prec="f32"))
    assert rel_err(y, _oracle_op(op, U, kappa, x, dims)) < 5e-6


def test_eo_layout_matches_lex():
    require_gpu()
    dims, kappa = (4, 4, 4, 4), 0.125
    ctx, U = context(dims, 0.3, 9, kappa)
    rng = np.random.default_rng(5)
    x = rng.standard_normal((2,) + ctx.shape) + 1j * rng.standard_normal((2,) + ctx.shape)
    say("eo layout", dims)
    xg = to_gpu(x)
    eo = ctx.pack_eo(xg)
    y_eo = ctx.wilson_apply("M", eo, layout="eo")
    assert rel_err(to_host(ctx.unpack_eo(y_eo)), to_host(ctx.wilson_apply("M", xg))) < 1e-15


def test_full_size_operator_16x32():
    require_gpu()
    dims, kappa = (16, 16, 16, 32), 0.125
    ctx, U = context(dims, 0.25, 1002, kappa)
    eta = ON.z4_noise(11, dims, 0, 1)
    say("op M full size", dims)
    y = to_host(ctx.wilson_apply("M", to_gpu(eta)))
    assert rel_err(y, W.apply_M(U, kappa, eta)) < 1e-13
    say("op schur full size", dims)
    y = to_host(ctx.wilson_apply("schur", to_gpu(eta)))
    assert rel_err(y, W.apply_Mhat(U, kappa, eta, dims)) < 1e-13


# tile shapes and orders of the link-tiled stencil: (timeslices per plane
# block, sites per tile (FP64: at most 32), right-hand sides per group);
# 0 timeslices = tiles of consecutive sites in index order, 0 right-hand
# sides = one group.  Launches with fewer right-hand sides than a tile's
# pass (256 / sites) take the next larger tile.
# The fourth entry: right-hand sides per group swept in turn within each
# block of timeslices (plane order only; 0 = off).
TILE_SHAPES = [(0, 64, 0, 0), (1, 64, 0, 0), (3, 64, 0, 0), (64, 64, 0, 0), (0, 32, 0, 0), (2, 32, 0, 0),
               (-1, 32, 0, 0), (-1, 32, 4, 0), (2, 64, 4, 0), (0, 32, 8, 0), (0, 16, 0, 0), (-1, 16, 0, 0),
               (2, 16, 0, 0), (-1, 16, 16, 0), (1, 16, 4, 0), (-1, 32, 0, 4), (2, 16, 0, 8), (1, 32, 0, 3),
               (3, 64, 4, 2), (0, 32, 0, 4), (-1, 32, 0, -1), (2, 16, 4, -1)]


@pytest.mark.parametrize("dims", [(2, 2, 2, 4), (6, 6, 2, 4), (6, 4, 2, 8), (8, 6, 2, 6)])
@pytest.mark.parametrize("prec,nrhs", [("f64", 9), ("f64", 17), ("f32", 5), ("f32", 9), ("f32", 17), ("f16", 5),
                                       ("f16", 8), ("f16", 16), ("bf16", 8), ("bf16", 16)])
def test_link_tiled_stencil(dims, prec, nrhs):
    """Launches with many right-hand sides take the link-tiled stencil
    (links staged in LDS per tile of sites): same operator as the oracle,
    and equal to the lane-grouped form up to rounding (the same sums in the
    same order; the compiler may fuse multiply-adds differently in the two
    kernels, so a few units in the last place) for every tile shape and
    order.  A wrong site, link or right-hand side would differ at O(1).
    Lattices give one partial tile (V/2 = 16), ragged tiles (V/2 = 144),
    whole tiles (V/2 = 192) and planes of 24 sites (ragged in every plane)
    with a partial last block of timeslices."""
    require_gpu()
    kappa = 0.13
    ctx, U = context(dims, 0.3, 7, kappa)
    rng = np.random.default_rng(6)
    x = rng.standard_normal((nrhs,) + ctx.shape) + 1j * rng.standard_normal((nrhs,) + ctx.shape)
    ops = ["schur"] if prec in ("f16", "bf16") else ["M", "Mdag", "MG5", "hop", "schur"]
    for op in ops:
        ctx.tune(hop_tile64=0, hop_tile32=0)
        y0 = to_host(ctx.wilson_apply(op, to_gpu(x), prec=prec))
        tol = {"f64": 1e-13, "f32": 5e-6, "f16": 2e-3, "bf16": 1.6e-2}[prec]
        assert rel_err(y0, _oracle_op(op, U, kappa, x, dims)) < tol, op
        for tb, ts, rg, rn in TILE_SHAPES:
            say("tiled stencil", op, prec, dims, nrhs, "tblock", tb, "tsites", ts, "rgroup", rg, "rnest", rn)
            ctx.tune(hop_tile64=1, hop_tile32=1, hop_tblock64=tb, hop_tblock32=tb, hop_tsites32=ts, hop_rgroup=rg,
                     hop_tsites64=min(ts, 32), hop_rnest=rn)
            y = to_host(ctx.wilson_apply(op, to_gpu(x), prec=prec))
            d = rel_err(y, y0)
            assert d < {"f64": 1e-14, "f32": 1e-6, "f16": 1e-6, "bf16": 1e-6}[prec], (op, tb, ts, rg, rn, d)
            assert rel_err(y, _oracle_op(op, U, kappa, x, dims)) < tol, (op, tb, ts, rg, rn)
    ctx.tune(hop_tile64=1, hop_tile32=1, hop_tblock64=-1, hop_tblock32=-1, hop_tsites32=32, hop_rgroup=0,
             hop_tsites64=32, hop_rnest=-1)
