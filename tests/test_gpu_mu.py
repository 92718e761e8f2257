"""Chemical potential (time-like hops e^{+mu} forward, e^{-mu} backward; the
adjoint with the opposite factors) on the GPU against the FP64 CPU oracle:
hop blocks and D_pre with their adjoints in every storage precision, the
solve, the 4d propagator, and both forces (pseudofermion and wall)."""
import sys

import numpy as np
import pytest

from parity import check

pytestmark = pytest.mark.gpu

TOL = {0: 1e-12, 1: 2e-5, 2: 4e-3}  # as the operator parity tests


def _flush(msg):
    print(msg, flush=True)
    sys.stdout.flush()


@pytest.fixture(scope="module")
def torch_cuda():
    import torch
    assert torch.cuda.is_available(), "GPU tests need an MI355X"
    return torch


def _rel(a, b):
    return float(np.linalg.norm((a - b).ravel()) / np.linalg.norm(b.ravel()))


def _setup(torch, dims, Ls, mu, seed=31):
    from oracle import Params
    from paper_1206_5214_amd import inputs, mobius
    p = Params(tuple(dims), Ls, 1.8, 0.05, 1.5, 0.5, mu)
    rng = np.random.default_rng(seed)
    U = inputs.random_links(dims, 0.5, rng)
    psi = inputs.gaussian_spinor(dims, Ls, rng)
    op = mobius.Operator(dims, Ls, 1.8, 0.05, 1.5, 0.5, torch.from_numpy(U).cuda(), mu=mu)
    return p, U, psi, op


@pytest.mark.parametrize("mu", [0.3, -0.5])
@pytest.mark.parametrize("prec", [0, 1, 2], ids=["f64", "f32", "f16"])
def test_hop_and_schur_with_mu(torch_cuda, orc, mu, prec):
    from oracle import restrict
    from paper_1206_5214_amd import mobius
    torch = torch_cuda
    dims, Ls = (4, 4, 2, 6), 8
    _flush(f"mu={mu} hop/schur parity prec={prec}")
    p, U, psi, op = _setup(torch, dims, Ls, mu)
    even, odd = op.pack(torch.from_numpy(psi).cuda(), prec)
    zero = op.new_field(prec)
    halves = {0: even, 1: odd}
    for dag in (False, True):
        for outp in (0, 1):
            out = op.dslash(halves[1 - outp], outp, prec, dag=dag)
            got = op.unpack(out if outp == 0 else zero, zero if outp == 0 else out, prec).cpu().numpy()
            check(got, orc.hop(p, U, psi, outp, dag=dag), TOL[prec], ("hop", dag, outp))
    psi_o = restrict(p, psi, 1)
    e, o = op.pack(torch.from_numpy(psi_o).cuda(), prec)
    for dag in (False, True):
        got = op.unpack(zero, op.dslash(o, 1, prec, op=mobius.OP_SCHUR, dag=dag), prec).cpu().numpy()
        check(got, orc.schur(p, U, psi_o, dag=dag), TOL[prec] * (3 if prec == 2 else 1),
              ("schur", dag))
    op.close()


@pytest.mark.parametrize("inner", [0, 2], ids=["f64", "mixed_f16"])
def test_solve_with_mu(torch_cuda, orc, inner):
    from paper_1206_5214_amd import mobius
    torch = torch_cuda
    dims, Ls = (4, 4, 4, 4), 8
    p, U, psi, op = _setup(torch, dims, Ls, 0.4, seed=32)
    _flush(f"mu=0.4 solve inner={inner}")
    eta = psi
    sol, info, rc = op.solve(torch.from_numpy(eta).cuda(), tol=1e-10, maxiter=50000, inner_prec=inner)
    assert rc == mobius.OK, info
    got = sol.cpu().numpy()
    res = _rel(orc.dw(p, U, got), eta)
    want, oi = orc.solve(p, U, eta, tol=1e-13, maxiter=50000)
    assert oi.converged
    err = _rel(got, want)
    _flush(f"  iters {info[0].iters} resid {res:.2e} err {err:.2e}")
    assert res <= 1e-10
    assert err <= 1e-8
    op.close()


def test_propagator4d_with_mu(torch_cuda, orc):
    from paper_1206_5214_amd import mobius
    torch = torch_cuda
    dims, Ls = (4, 4, 4, 4), 6
    p, U, _, op = _setup(torch, dims, Ls, 0.25, seed=33)
    rng = np.random.default_rng(34)
    shape4 = (dims[3], dims[2], dims[1], dims[0], 4, 3)
    b = rng.normal(size=shape4) + 1j * rng.normal(size=shape4)
    q, info, rc = op.propagator4d(torch.from_numpy(b).cuda(), tol=1e-11, maxiter=50000)
    assert rc == mobius.OK, info
    want, oi = orc.propagator4d(p, U, b, tol=1e-13)
    err = _rel(q.cpu().numpy(), want)
    _flush(f"  mu=0.25 propagator err {err:.2e}")
    assert err <= 1e-8
    op.close()


@pytest.mark.parametrize("mu", [0.3, -0.25])
def test_forces_with_mu_vs_oracle(torch_cuda, orc, mu):
    """The pseudofermion force and the wall-pseudofermion force with a chemical
    potential: actions and link gradients against the oracle's (whose
    derivative is pinned against central differences at mu != 0)."""
    from oracle import Params
    from paper_1206_5214_amd import inputs, mobius
    torch = torch_cuda
    dims, Ls, mf = (4, 4, 2, 4), 6, 0.2
    _flush(f"forces with mu={mu}")
    p = Params(dims, Ls, 1.8, mf, 1.5, 0.5, mu)
    rng = np.random.default_rng(61)
    U = inputs.random_links(dims, 0.5, rng)
    phi = inputs.gaussian_spinor(dims, Ls, rng)
    op = mobius.Operator(dims, Ls, 1.8, mf, 1.5, 0.5, torch.from_numpy(U).cuda(), mu=mu)
    S_o, X_o, G_o, info_o = orc.force(p, U, orc.restrict(p, phi, 1), tol=1e-14)
    assert info_o.converged
    S, G, gphi, info, rc = op.force(torch.from_numpy(phi).cuda(), tol=1e-12)
    assert rc == mobius.OK, info
    err = np.abs(G.cpu().numpy() - G_o).max() / np.abs(G_o).max()
    _flush(f"  force: S {S:.12e} oracle {S_o:.12e}, gradient error {err:.1e}")
    assert abs(S - S_o) <= 1e-10 * abs(S_o) and err <= 1e-9
    assert _rel(gphi.cpu().numpy(), 2 * X_o) <= 1e-10
    phi4 = rng.normal(size=p.shape4()) + 1j * rng.normal(size=p.shape4())
    Sw, Gw, infow, rc = op.force_wall(torch.from_numpy(phi4).cuda(), tol=1e-13)
    assert rc == mobius.OK, infow
    Sw_o, Gw_o, _ = orc.force_wall(p, U, phi4, tol=1e-14)
    errw = np.abs(Gw.cpu().numpy() - Gw_o).max() / np.abs(Gw_o).max()
    _flush(f"  wall force: S {Sw:.12e} oracle {Sw_o:.12e}, gradient error {errw:.1e}")
    assert abs(Sw - Sw_o) <= 1e-10 * abs(Sw_o) and errw <= 1e-9
    op.close()
