"""HIP path vs the FP64 CPU oracle, element by element, through the C ABI.

Tolerances, derived from the arithmetic of one hop (a sum of ~100 products
of O(1) numbers per output), each applied both to the max-abs difference over
the field relative to max |oracle| and per 5d site relative to that site's own
max |oracle| (tests/parity.py):
  FP64: 1e-12     (unit roundoff 1.1e-16 times the ~1e2 terms, with margin)
  FP32: 2e-5      (unit roundoff 6e-8 times ~1e2 terms, with margin)
  FP16 storage:   4e-3 of the site norm per stored value (binary16 unit roundoff
                  4.9e-4 on spinor and link storage, a few roundings deep)
Besides Gaussian fields, the hop blocks and D_pre are checked on graded
fields whose 5d site norms span six decades.
"""
import sys

import numpy as np
import pytest

from parity import check, graded

pytestmark = pytest.mark.gpu

TOL = {0: 1e-12, 1: 2e-5, 2: 4e-3}


def _flush(msg):
    print(msg, flush=True)
    sys.stdout.flush()


@pytest.fixture(scope="module")
def torch_cuda():
    import torch
    assert torch.cuda.is_available(), "GPU tests need an MI355X"
    return torch


def _params(dims, Ls, M5=1.8, mf=0.05, b5=1.5, c5=0.5):
    from oracle import Params
    return Params(tuple(dims), Ls, M5, mf, b5, c5)


def _setup(torch, p, seed=3, eps=0.5):
    from paper_1206_5214_amd import inputs, mobius
    rng = np.random.default_rng(seed)
    U = inputs.random_links(p.dims, eps, rng)
    psi = inputs.gaussian_spinor(p.dims, p.Ls, rng)
    op = mobius.Operator(p.dims, p.Ls, p.M5, p.mf, p.b5, p.c5, torch.from_numpy(U).cuda())
    return U, psi, op


CASES = [
    # dims, Ls, b5, c5, mf : several tiles, ragged tails, Ls not dividing 64
    ((4, 4, 4, 4), 8, 1.0, 0.0, 0.01),        # Shamir
    ((4, 4, 4, 4), 8, 1.5, 0.5, 0.05),
    ((6, 4, 2, 4), 12, 1.75, 0.75, 0.005),    # Vh = 96: ragged last block for Ls = 12
    ((2, 2, 2, 2), 5, 1.5, 0.5, 1.0),         # Pauli-Villars mass, tiny lattice, Ls = 5
    ((4, 2, 6, 2), 16, 1.2, 0.3, 0.2),
    ((4, 4, 2, 2), 33, 1.5, 0.5, 0.1),        # one site per wavefront
    ((2, 4, 2, 4), 2, 2.0, 1.0, 0.0),         # Ls = 2, mf = 0
]


@pytest.mark.parametrize("case", CASES, ids=[f"{c[0]}-Ls{c[1]}-b{c[2]}-c{c[3]}" for c in CASES])
@pytest.mark.parametrize("prec", [0, 1, 2], ids=["f64", "f32", "f16"])
def test_hop_blocks_vs_oracle(torch_cuda, orc, case, prec):
    torch = torch_cuda
    dims, Ls, b5, c5, mf = case
    p = _params(dims, Ls, b5=b5, c5=c5, mf=mf)
    _flush(f"hop parity {case} prec={prec}")
    U, psi, op = _setup(torch, p)
    canon = torch.from_numpy(psi).cuda()
    even, odd = op.pack(canon, prec)
    zero = op.new_field(prec)
    halves = {0: even, 1: odd}
    for dag in (False, True):
        for outp in (0, 1):
            out = op.dslash(halves[1 - outp], outp, prec, dag=dag)
            got = op.unpack(out if outp == 0 else zero, zero if outp == 0 else out, prec).cpu().numpy()
            want = orc.hop(p, U, psi, outp, dag=dag)
            check(got, want, TOL[prec], (case, prec, dag, outp))
    op.close()


@pytest.mark.parametrize("case", CASES[:4], ids=[f"{c[0]}-Ls{c[1]}" for c in CASES[:4]])
@pytest.mark.parametrize("prec", [0, 1, 2], ids=["f64", "f32", "f16"])
def test_m5_and_m5inv_vs_oracle(torch_cuda, orc, case, prec):
    from paper_1206_5214_amd import mobius
    torch = torch_cuda
    dims, Ls, b5, c5, mf = case
    p = _params(dims, Ls, b5=b5, c5=c5, mf=mf)
    _flush(f"m5 parity {case} prec={prec}")
    U, psi, op = _setup(torch, p)
    canon = torch.from_numpy(psi).cuda()
    even, odd = op.pack(canon, prec)
    for dag in (False, True):
        me = op.dslash(even, 0, prec, op=mobius.OP_M5, dag=dag)
        mo = op.dslash(odd, 1, prec, op=mobius.OP_M5, dag=dag)
        got = op.unpack(me, mo, prec).cpu().numpy()
        check(got, orc.m5(p, U, psi, dag=dag), TOL[prec], ("m5", dag))
        ie = op.m5inv(even, prec, dag=dag)
        io = op.m5inv(odd, prec, dag=dag)
        got = op.unpack(ie, io, prec).cpu().numpy()
        check(got, orc.m5inv(p, psi, dag=dag), TOL[prec], ("m5inv", dag))
    op.close()


@pytest.mark.parametrize("case", CASES[:5], ids=[f"{c[0]}-Ls{c[1]}" for c in CASES[:5]])
@pytest.mark.parametrize("prec", [0, 1, 2], ids=["f64", "f32", "f16"])
def test_schur_vs_oracle(torch_cuda, orc, case, prec):
    from paper_1206_5214_amd import mobius
    from oracle import restrict
    torch = torch_cuda
    dims, Ls, b5, c5, mf = case
    p = _params(dims, Ls, b5=b5, c5=c5, mf=mf)
    _flush(f"schur parity {case} prec={prec}")
    U, psi, op = _setup(torch, p)
    psi_o = restrict(p, psi, 1)
    even, odd = op.pack(torch.from_numpy(psi_o).cuda(), prec)
    zero = op.new_field(prec)
    for dag in (False, True):
        out = op.dslash(odd, 1, prec, op=mobius.OP_SCHUR, dag=dag)
        got = op.unpack(zero, out, prec).cpu().numpy()
        want = orc.schur(p, U, psi_o, dag=dag)
        tol = TOL[prec] * (3 if prec == 2 else 1)
        check(got, want, tol, ("schur", dag))
    op.close()


@pytest.mark.parametrize("case", CASES[:5], ids=[f"{c[0]}-Ls{c[1]}" for c in CASES[:5]])
@pytest.mark.parametrize("prec", [0, 1, 2], ids=["f64", "f32", "f16"])
def test_full_operator_vs_oracle(torch_cuda, orc, case, prec):
    """MOBIUS_OP_FULL: the unpreconditioned D_DW(m) and D_DW(m)^+ on both packed
    halves against the oracle's whole-lattice D_DW, one and two right-hand sides."""
    from paper_1206_5214_amd import mobius
    torch = torch_cuda
    dims, Ls, b5, c5, mf = case
    p = _params(dims, Ls, b5=b5, c5=c5, mf=mf)
    _flush(f"full operator parity {case} prec={prec}")
    U, psi, op = _setup(torch, p)
    psi2 = np.stack([psi, graded(psi, np.random.default_rng(5))])
    for nrhs, field in ((1, psi), (2, psi2)):
        x = op.pack_full(torch.from_numpy(np.ascontiguousarray(field)).cuda(), prec, nrhs)
        for dag in (False, True):
            out = op.dslash(x, 0, prec, op=mobius.OP_FULL, dag=dag, nrhs=nrhs)
            got = op.unpack_full(out, prec, nrhs).cpu().numpy()
            want = np.stack([orc.dw(p, U, f, dag=dag) for f in (field if nrhs > 1 else [field])])
            check(got.reshape(want.shape), want, TOL[prec], ("full", nrhs, dag))
    # in and out overlap by one half: rejected before anything is launched
    x = op.pack_full(torch.from_numpy(psi).cuda(), prec)
    fb = op.field_bytes(prec)
    assert mobius.lib().mobius_dslash(op._h, prec, mobius.OP_FULL, 0, mobius._ptr(x),
                                      mobius._ptr(x[fb:]), 1, None) == -22
    op.close()


@pytest.mark.parametrize("case", [CASES[1], CASES[2], CASES[4]], ids=["4^4-Ls8", "6x4x2x4-Ls12", "4x2x6x2-Ls16"])
@pytest.mark.parametrize("prec", [0, 1, 2], ids=["f64", "f32", "f16"])
def test_graded_field_vs_oracle(torch_cuda, orc, case, prec):
    """Hop blocks (D and D^+, both parities) and D_pre (and D_pre^+) on a field
    whose 5d site norms span six decades, per site against the oracle."""
    from paper_1206_5214_amd import mobius
    from oracle import restrict
    torch = torch_cuda
    dims, Ls, b5, c5, mf = case
    p = _params(dims, Ls, b5=b5, c5=c5, mf=mf)
    _flush(f"graded-field parity {case} prec={prec}")
    U, psi, op = _setup(torch, p)
    psi = graded(psi, np.random.default_rng(77))
    even, odd = op.pack(torch.from_numpy(psi).cuda(), prec)
    zero = op.new_field(prec)
    halves = {0: even, 1: odd}
    for dag in (False, True):
        for outp in (0, 1):
            out = op.dslash(halves[1 - outp], outp, prec, dag=dag)
            got = op.unpack(out if outp == 0 else zero, zero if outp == 0 else out, prec).cpu().numpy()
            check(got, orc.hop(p, U, psi, outp, dag=dag), TOL[prec], ("graded hop", dag, outp))
    psi_o = restrict(p, psi, 1)
    _, odd = op.pack(torch.from_numpy(psi_o).cuda(), prec)
    for dag in (False, True):
        out = op.dslash(odd, 1, prec, op=mobius.OP_SCHUR, dag=dag)
        got = op.unpack(zero, out, prec).cpu().numpy()
        check(got, orc.schur(p, U, psi_o, dag=dag), TOL[prec] * (3 if prec == 2 else 1),
              ("graded schur", dag))
    op.close()


def test_pack_roundtrip_and_adjoint_on_gpu(torch_cuda):
    """Pack/unpack is exact in FP64; <x, D y> = <D^+ x, y> for the GPU hop blocks."""
    torch = torch_cuda
    p = _params((4, 4, 2, 6), 12, b5=1.75, c5=0.75, mf=0.005)
    U, psi, op = _setup(torch, p)
    canon = torch.from_numpy(psi).cuda()
    e, o = op.pack(canon, 0)
    back = op.unpack(e, o, 0)
    assert torch.equal(back, canon)
    rng = np.random.default_rng(8)
    from paper_1206_5214_amd import inputs
    x = torch.from_numpy(inputs.gaussian_spinor(p.dims, p.Ls, rng)).cuda()
    xe, xo = op.pack(x, 0)
    zero = op.new_field(0)
    # block D_{e,o}: odd -> even, its adjoint (D^+)_{o,e}: even -> odd
    Dy = op.unpack(op.dslash(o, 0, 0), zero, 0)
    Ddx = op.unpack(zero, op.dslash(xe, 1, 0, dag=True), 0)
    lhs = torch.vdot(x.flatten(), Dy.flatten()).item()
    rhs = torch.vdot(Ddx.flatten(), canon.flatten()).item()
    assert abs(lhs - rhs) < 1e-12 * abs(lhs)
    op.close()


def test_f16_pack_tiny_sites(torch_cuda):
    """FP16 storage of a field whose 5d sites span 1 .. 1e-45 in magnitude (as
    the front of a Krylov vector grown from a point source does): sites whose
    largest component is below the smallest normal FP32 number are stored as
    zero, every other site to binary16 precision relative to its own norm, and
    nothing decodes to inf or NaN."""
    torch = torch_cuda
    p = _params((4, 4, 2, 6), 8)
    U, psi, op = _setup(torch, p)
    rng = np.random.default_rng(11)
    scale = 10.0 ** -rng.uniform(0, 45, size=psi.shape[:-2])
    x = psi * scale[..., None, None]
    canon = torch.from_numpy(x).cuda()
    e, o = op.pack(canon, 2)
    back = op.unpack(e, o, 2).cpu().numpy()
    assert np.all(np.isfinite(back))
    xf = x.astype(np.complex64).astype(np.complex128)  # the pack rounds to FP32 first
    site_max = np.max(np.maximum(np.abs(xf.real), np.abs(xf.imag)), axis=(-2, -1))
    tiny = site_max < np.finfo(np.float32).tiny
    assert np.count_nonzero(tiny) > 0 and np.count_nonzero(~tiny) > 0
    assert np.all(back[tiny] == 0)
    err = np.max(np.abs(back - xf), axis=(-2, -1))
    assert np.all(err[~tiny] <= 2.0 ** -10 * site_max[~tiny])
    op.close()


def test_repeatable_bitwise(torch_cuda):
    """Two applications give bit-identical results (no atomics, fixed reduction order)."""
    from paper_1206_5214_amd import mobius
    torch = torch_cuda
    p = _params((4, 4, 4, 4), 8)
    U, psi, op = _setup(torch, p)
    e, o = op.pack(torch.from_numpy(psi).cuda(), 0)
    a = op.dslash(o, 1, 0, op=mobius.OP_SCHUR)
    b = op.dslash(o, 1, 0, op=mobius.OP_SCHUR)
    assert torch.equal(a, b)
    op.close()


def test_argument_errors(torch_cuda):
    from paper_1206_5214_amd import mobius
    torch = torch_cuda
    p = _params((4, 4, 4, 4), 8)
    U, psi, op = _setup(torch, p)
    f = op.new_field(0)
    with pytest.raises(mobius.MobiusError):
        op.dslash(f, 0, 0, out=f)                     # aliasing
    with pytest.raises(mobius.MobiusError):
        op.dslash(f, 0, 0, op=mobius.OP_SCHUR)        # SCHUR needs odd output
    with pytest.raises(mobius.MobiusError):
        op.dslash(f, 2, 0)                            # bad parity
    with pytest.raises(mobius.MobiusError):
        op.dslash(f, 0, 7, out=op.new_field(0))       # bad precision
    op.close()


BRICKS = [(2, 2, 2), (2, 4, 2), (4, 2, 6), (6, 2, 4), (4, 3, 5)]  # last: partial bricks


@pytest.mark.parametrize("brick", BRICKS, ids=[f"brick{b}" for b in BRICKS])
def test_site_orders_vs_oracle(torch_cuda, orc, brick, monkeypatch):
    """Every bricked site order (including bricks that do not divide the lattice)
    gives the same operator: hop, Schur and a solve against the oracle."""
    from paper_1206_5214_amd import mobius
    from oracle import restrict
    torch = torch_cuda
    monkeypatch.setenv("MOBIUS_BRICK", ",".join(map(str, brick)))
    p = _params((8, 6, 10, 4), 6, b5=1.5, c5=0.5, mf=0.02)
    _flush(f"site order brick={brick}")
    U, psi, op = _setup(torch, p)
    canon = torch.from_numpy(psi).cuda()
    for prec in (0, 2):
        even, odd = op.pack(canon, prec)
        assert torch.equal(op.unpack(even, odd, 0), canon) if prec == 0 else True
        zero = op.new_field(prec)
        got = op.unpack(op.dslash(odd, 0, prec), zero, prec).cpu().numpy()
        check(got, orc.hop(p, U, psi, 0), TOL[prec], ("hop", brick, prec))
        got = op.unpack(zero, op.dslash(even, 1, prec, dag=True), prec).cpu().numpy()
        check(got, orc.hop(p, U, psi, 1, dag=True), TOL[prec], ("hop dag", brick, prec))
    psi_o = restrict(p, psi, 1)
    e, o = op.pack(torch.from_numpy(psi_o).cuda(), 0)
    got = op.unpack(op.new_field(0), op.dslash(o, 1, 0, op=mobius.OP_SCHUR), 0).cpu().numpy()
    check(got, orc.schur(p, U, psi_o), TOL[0], ("schur", brick))
    sol, info, rc = op.solve(canon, tol=1e-10)
    assert rc == mobius.OK
    res = np.linalg.norm(orc.dw(p, U, sol.cpu().numpy()) - psi) / np.linalg.norm(psi)
    assert res <= 1e-10
    op.close()
