"""Per-slice coefficients b5(s), c5(s) of the general Moebius operator
(Sec. 2.1) on the GPU against the FP64 CPU oracle: hop blocks, I, I^-1,
D_pre and the whole D_DW with their adjoints in every storage precision
(tolerances as tests/test_gpu_parity.py, global and per 5d site), solves in
every inner precision, the force and the 4d propagator."""
import sys

import numpy as np
import pytest

from parity import check

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


def _coeffs(Ls, seed, sym=False):
    rng = np.random.default_rng(seed)
    b = rng.uniform(1.0, 2.0, Ls)
    c = rng.uniform(0.0, 0.8, Ls)
    if sym:
        b, c = 0.5 * (b + b[::-1]), 0.5 * (c + c[::-1])
    return tuple(b), tuple(c)


def _setup(torch, dims, Ls, mf, seed, sym=False, eps=0.5):
    from oracle import Params
    from paper_1206_5214_amd import inputs, mobius
    b5s, c5s = _coeffs(Ls, seed, sym)
    p = Params(tuple(dims), Ls, 1.8, mf, 1.5, 0.5, 0.0, b5s, c5s)
    rng = np.random.default_rng(seed + 100)
    U = inputs.random_links(dims, eps, rng)
    psi = inputs.gaussian_spinor(dims, Ls, rng)
    op = mobius.Operator(dims, Ls, 1.8, mf, 1.5, 0.5, torch.from_numpy(U).cuda(), b5s=b5s, c5s=c5s)
    return p, U, psi, op


CASES = [((4, 4, 4, 4), 8, 0.02), ((6, 4, 2, 4), 12, 0.005), ((4, 2, 2, 2), 5, 0.3), ((2, 4, 2, 4), 16, 1.0)]


@pytest.mark.parametrize("case", CASES, ids=[f"{c[0]}-Ls{c[1]}" for c in CASES])
@pytest.mark.parametrize("prec", [0, 1, 2], ids=["f64", "f32", "f16"])
def test_sdep_operator_blocks(torch_cuda, orc, case, prec):
    from oracle import restrict
    from paper_1206_5214_amd import mobius
    torch = torch_cuda
    dims, Ls, mf = case
    _flush(f"s-dependent blocks {case} prec={prec}")
    p, U, psi, op = _setup(torch, dims, Ls, mf, seed=Ls)
    canon = torch.from_numpy(psi).cuda()
    even, odd = op.pack(canon, prec)
    zero = op.new_field(prec)
    halves = {0: even, 1: odd}
    for dag in (False, True):
        for outp in (0, 1):
            out = op.dslash(halves[1 - outp], outp, prec, dag=dag)
            got = op.unpack(out if outp == 0 else zero, zero if outp == 0 else out, prec).cpu().numpy()
            check(got, orc.hop(p, U, psi, outp, dag=dag), TOL[prec], ("hop", dag, outp))
        me = op.dslash(even, 0, prec, op=mobius.OP_M5, dag=dag)
        mo = op.dslash(odd, 1, prec, op=mobius.OP_M5, dag=dag)
        check(op.unpack(me, mo, prec).cpu().numpy(), orc.m5(p, U, psi, dag=dag), TOL[prec], ("m5", dag))
        ie, io = op.m5inv(even, prec, dag=dag), op.m5inv(odd, prec, dag=dag)
        check(op.unpack(ie, io, prec).cpu().numpy(), orc.m5inv(p, psi, dag=dag), TOL[prec], ("m5inv", dag))
        full = op.dslash(op.pack_full(canon, prec), 0, prec, op=mobius.OP_FULL, dag=dag)
        check(op.unpack_full(full, prec).cpu().numpy(), orc.dw(p, U, psi, dag=dag), TOL[prec], ("full", dag))
    psi_o = restrict(p, psi, 1)
    _, o = op.pack(torch.from_numpy(psi_o).cuda(), prec)
    for dag in (False, True):
        out = op.dslash(o, 1, prec, op=mobius.OP_SCHUR, dag=dag)
        check(op.unpack(zero, out, prec).cpu().numpy(), orc.schur(p, U, psi_o, dag=dag),
              TOL[prec] * (3 if prec == 2 else 1), ("schur", dag))
    op.close()


@pytest.mark.parametrize("inner", [0, 1, 2], ids=["f64", "mixed_f32", "mixed_f16"])
def test_sdep_solve(torch_cuda, orc, inner):
    from paper_1206_5214_amd import mobius
    torch = torch_cuda
    _flush(f"s-dependent solve inner={inner}")
    p, U, psi, op = _setup(torch, (4, 4, 4, 8), 8, 0.01, seed=21, sym=True)
    eta = psi
    sol, info, rc = op.solve(torch.from_numpy(eta).cuda(), tol=1e-10, maxiter=20000, inner_prec=inner)
    assert rc == mobius.OK, info
    got = sol.cpu().numpy()
    res = float(np.linalg.norm(orc.dw(p, U, got) - eta) / np.linalg.norm(eta))
    want, oinfo = orc.solve(p, U, eta, tol=1e-13, maxiter=20000)
    err = float(np.linalg.norm(got - want) / np.linalg.norm(want))
    _flush(f"  iters {info[0].iters}, true resid {res:.2e}, error vs oracle {err:.2e}, kappa {info[0].kappa:.1f}")
    assert oinfo.converged and res <= 1e-10 and err <= 1e-8
    op.close()


def test_sdep_force_and_propagator(torch_cuda, orc):
    from oracle import restrict
    from paper_1206_5214_amd import mobius
    torch = torch_cuda
    _flush("s-dependent force and 4d propagator")
    p, U, psi, op = _setup(torch, (4, 4, 2, 4), 6, 0.05, seed=31, sym=True)
    phi = restrict(p, psi, 1)
    S, G, gphi, info, rc = op.force(torch.from_numpy(phi).cuda(), tol=1e-13)
    assert rc == mobius.OK
    S_o, X_o, G_o, oinfo = orc.force(p, U, phi, tol=1e-13)
    assert abs(S - S_o) <= 1e-10 * abs(S_o)
    err = float((G.cpu().numpy() - G_o).__abs__().max() / np.abs(G_o).max())
    _flush(f"  force: S {S:.10e} (oracle {S_o:.10e}), gradient error {err:.1e}")
    assert err <= 1e-9
    b4 = psi[0]
    q, infos, rc = op.propagator4d(torch.from_numpy(np.ascontiguousarray(b4)).cuda(), tol=1e-12)
    assert rc == mobius.OK
    q_o, oinf = orc.propagator4d(p, U, b4, tol=1e-13)
    err = float(np.linalg.norm(q.cpu().numpy() - q_o) / np.linalg.norm(q_o))
    _flush(f"  4d propagator error vs oracle {err:.1e}")
    assert err <= 1e-8
    op.close()


def test_sdep_argument_errors(torch_cuda):
    from paper_1206_5214_amd import inputs, mobius
    torch = torch_cuda
    dims, Ls = (4, 4, 4, 4), 6
    U = torch.from_numpy(inputs.unit_links(dims)).cuda()
    with pytest.raises(mobius.MobiusError):   # wrong length
        mobius.Operator(dims, Ls, 1.8, 0.01, 1.5, 0.5, U, b5s=(1.5,) * (Ls - 1))
    with pytest.raises(mobius.MobiusError):   # M+(s) = b5(s) (4 - M5) + 1 = 0 on one slice
        mobius.Operator(dims, Ls, 1.8, 0.01, 1.5, 0.5, U, b5s=(1.5,) * (Ls - 1) + (-1.0 / 2.2,))
    with pytest.raises(mobius.MobiusError):   # not finite
        mobius.Operator(dims, Ls, 1.8, 0.01, 1.5, 0.5, U, c5s=(0.5,) * (Ls - 1) + (float("nan"),))
