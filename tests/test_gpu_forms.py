"""Operator variants on the same data, on the GPU against the FP64 CPU oracle:
the right-preconditioned Schur operator D_R = 1 - D_oe I^-1 D_eo I^-1, the
Schur complement S = I - D_oe I^-1 D_eo itself, and their adjoints, the hop
and Schur blocks of the left form D^ = D-^-1 D_DW D- of Sec. 2.1, red/black
solves that iterate on each, the adjoint system
D_DW^+ psi = eta, and the 4d-HMC action with the pseudofermion on the wall
(Sec. 2.4) with its two-inversion link gradient."""
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


def _setup(torch, dims, Ls, mf=0.02, b5=1.5, c5=0.5, seed=7, eps=0.5):
    from oracle import Params
    from paper_1206_5214_amd import inputs, mobius
    p = Params(tuple(dims), Ls, 1.8, mf, b5, c5)
    rng = np.random.default_rng(seed)
    U = inputs.random_links(dims, eps, rng)
    psi = inputs.gaussian_spinor(dims, Ls, rng)
    op = mobius.Operator(dims, Ls, 1.8, mf, b5, c5, torch.from_numpy(U).cuda())
    return p, U, psi, op


CASES = [((4, 4, 4, 4), 8), ((6, 4, 2, 4), 12), ((4, 2, 2, 2), 5)]


@pytest.mark.parametrize("case", CASES, ids=[f"{c[0]}-Ls{c[1]}" for c in CASES])
@pytest.mark.parametrize("prec", [0, 1, 2], ids=["f64", "f32", "f16"])
def test_schur_right_vs_oracle(torch_cuda, orc, case, prec):
    from oracle import restrict
    from paper_1206_5214_amd import mobius
    torch = torch_cuda
    dims, Ls = case
    _flush(f"right Schur operator {case} prec={prec}")
    p, U, psi, op = _setup(torch, dims, Ls)
    psi_o = restrict(p, psi, 1)
    _, odd = op.pack(torch.from_numpy(psi_o).cuda(), prec)
    zero = op.new_field(prec)
    for dag in (False, True):
        out = op.dslash(odd, 1, prec, op=mobius.OP_SCHUR_RIGHT, dag=dag)
        got = op.unpack(zero, out, prec).cpu().numpy()
        check(got, orc.schur_right(p, U, psi_o, dag=dag), TOL[prec] * (3 if prec == 2 else 1),
              ("schur right", dag))
    op.close()


@pytest.mark.parametrize("case", CASES, ids=[f"{c[0]}-Ls{c[1]}" for c in CASES])
@pytest.mark.parametrize("prec", [0, 1, 2], ids=["f64", "f32", "f16"])
def test_schur_complement_vs_oracle(torch_cuda, orc, case, prec):
    from oracle import restrict
    from paper_1206_5214_amd import mobius
    torch = torch_cuda
    dims, Ls = case
    _flush(f"Schur complement {case} prec={prec}")
    p, U, psi, op = _setup(torch, dims, Ls)
    psi_o = restrict(p, psi, 1)
    _, odd = op.pack(torch.from_numpy(psi_o).cuda(), prec)
    zero = op.new_field(prec)
    for dag in (False, True):
        out = op.dslash(odd, 1, prec, op=mobius.OP_SCHUR_COMPLEMENT, dag=dag)
        got = op.unpack(zero, out, prec).cpu().numpy()
        check(got, orc.schur_complement(p, U, psi_o, dag=dag), TOL[prec] * (3 if prec == 2 else 1),
              ("schur complement", dag))
    op.close()


@pytest.mark.parametrize("case", CASES, ids=[f"{c[0]}-Ls{c[1]}" for c in CASES])
@pytest.mark.parametrize("prec", [0, 1, 2], ids=["f64", "f32", "f16"])
def test_left_form_blocks_vs_oracle(torch_cuda, orc, case, prec):
    """OP_HOP_LEFT (-1/2 B H, both output parities) and OP_SCHUR_LEFT, each with
    its adjoint, against the oracle's left form D^ = B D_W + 1 - C5."""
    from oracle import restrict
    from paper_1206_5214_amd import mobius
    torch = torch_cuda
    dims, Ls = case
    _flush(f"left-form blocks {case} prec={prec}")
    p, U, psi, op = _setup(torch, dims, Ls)
    even, odd = op.pack(torch.from_numpy(psi).cuda(), prec)
    halves = {0: even, 1: odd}
    zero = op.new_field(prec)
    for outp in (0, 1):
        for dag in (False, True):
            out = op.dslash(halves[1 - outp], outp, prec, op=mobius.OP_HOP_LEFT, dag=dag)
            got = op.unpack(out if outp == 0 else zero, zero if outp == 0 else out, prec).cpu().numpy()
            check(got, orc.hop_left(p, U, psi, outp, dag=dag), TOL[prec], ("hop left", outp, dag))
    psi_o = restrict(p, psi, 1)
    for dag in (False, True):
        out = op.dslash(odd, 1, prec, op=mobius.OP_SCHUR_LEFT, dag=dag)
        got = op.unpack(zero, out, prec).cpu().numpy()
        check(got, orc.schur_left(p, U, psi_o, dag=dag), TOL[prec] * (3 if prec == 2 else 1),
              ("schur left", dag))
    op.close()


def test_left_form_rejects_per_slice_coefficients(torch_cuda):
    """The left-form blocks and solve need constant b5, c5 (B and I commute only then)."""
    from paper_1206_5214_amd import inputs, mobius
    torch = torch_cuda
    dims, Ls = (4, 4, 4, 4), 6
    U = inputs.random_links(dims, 0.5, np.random.default_rng(3))
    op = mobius.Operator(dims, Ls, 1.8, 0.02, 1.5, 0.5, torch.from_numpy(U).cuda(),
                         b5s=np.linspace(1.2, 1.8, Ls), c5s=np.full(Ls, 0.5))
    x = op.new_field(0)
    with pytest.raises(mobius.MobiusError, match="constant b5, c5"):
        op.dslash(x, 1, 0, op=mobius.OP_SCHUR_LEFT)
    src = torch.from_numpy(inputs.gaussian_spinor(dims, Ls, np.random.default_rng(4))).cuda()
    with pytest.raises(mobius.MobiusError, match="constant b5, c5"):
        op.solve(src, form=2)
    op.close()


@pytest.mark.parametrize("form", [2, 3], ids=["left_form_Dhat", "schur_complement"])
@pytest.mark.parametrize("inner", [0, 1, 2], ids=["f64", "mixed_f32", "mixed_f16"])
def test_form_solve(torch_cuda, orc, inner, form):
    """form=2 iterates on B D_pre B^-1 and maps back with B^-1; form=3 on the
    Schur complement S = I D_pre: the solution of D_DW psi = eta to the
    oracle's (two right-hand sides)."""
    from paper_1206_5214_amd import inputs, mobius
    torch = torch_cuda
    dims, Ls = (4, 4, 4, 8), 12
    _flush(f"solve form {form}, inner={inner}")
    p, U, psi, op = _setup(torch, dims, Ls, mf=0.01, b5=1.75, c5=0.75, seed=9, eps=0.5)
    eta = np.stack([psi, inputs.gaussian_spinor(dims, Ls, np.random.default_rng(11))])
    sol, info, rc = op.solve(torch.from_numpy(eta).cuda(), tol=1e-10, maxiter=20000, inner_prec=inner,
                             form=form)
    assert rc == mobius.OK, info
    got = sol.cpu().numpy()
    for r in range(2):
        res = float(np.linalg.norm(orc.dw(p, U, got[r]) - eta[r]) / np.linalg.norm(eta[r]))
        want, oinfo = orc.solve(p, U, eta[r], tol=1e-13, maxiter=20000)
        err = float(np.linalg.norm(got[r] - want) / np.linalg.norm(want))
        _flush(f"  rhs {r}: iters {info[r].iters}, resid {res:.2e} (solver {info[r].true_resid:.2e}), "
               f"error {err:.2e}, kappa {info[r].kappa:.1f}")
        assert oinfo.converged and res <= 1e-10 and err <= 1e-8
        assert abs(res - info[r].true_resid) <= 1e-11 + 0.05 * res
    op.close()


@pytest.mark.parametrize("inner", [0, 1, 2], ids=["f64", "mixed_f32", "mixed_f16"])
def test_right_form_and_adjoint_solves(torch_cuda, orc, inner):
    """form=1 reaches the left form's solution; mobius_cg_solve_dag solves
    D_DW^+ psi = eta (true residual recomputed with the oracle's D_DW^+, and
    the oracle's own adjoint-system solve), two right-hand sides each."""
    from paper_1206_5214_amd import mobius
    torch = torch_cuda
    dims, Ls = (4, 4, 4, 8), 12
    _flush(f"right form and adjoint system, inner={inner}")
    p, U, psi, op = _setup(torch, dims, Ls, mf=0.01, b5=1.75, c5=0.75, seed=9, eps=0.5)
    rng = np.random.default_rng(10)
    from paper_1206_5214_amd import inputs
    eta = np.stack([psi, inputs.gaussian_spinor(dims, Ls, rng)])
    src = torch.from_numpy(eta).cuda()
    for dagger, form in ((False, 1), (True, 0)):
        sol, info, rc = op.solve(src, tol=1e-10, maxiter=20000, inner_prec=inner, form=form, dagger=dagger)
        assert rc == mobius.OK, info
        got = sol.cpu().numpy()
        for r in range(2):
            res = float(np.linalg.norm(orc.dw(p, U, got[r], dag=dagger) - eta[r]) / np.linalg.norm(eta[r]))
            want, oinfo = orc.solve_form(p, U, eta[r], 2 if dagger else 0, tol=1e-13, maxiter=20000)
            err = float(np.linalg.norm(got[r] - want) / np.linalg.norm(want))
            _flush(f"  dagger {dagger} form {form} rhs {r}: iters {info[r].iters}, resid {res:.2e} "
                   f"(solver {info[r].true_resid:.2e}), error {err:.2e}, kappa {info[r].kappa:.1f}")
            assert oinfo.converged and res <= 1e-10 and err <= 1e-8
            assert abs(res - info[r].true_resid) <= 1e-11 + 0.05 * res
    op.close()


def test_force_wall_vs_oracle(torch_cuda, orc):
    """The two-inversion force of the wall pseudofermion action against the
    oracle's action and gradient, and the action against phi^+ (D_ov^+ D_ov)^-1 phi
    evaluated through the oracle's 4d propagator: with D_ov^+ = g5 D_ov g5 it is
    |D_ov^-1 g5 phi|^2."""
    from paper_1206_5214_amd import mobius
    torch = torch_cuda
    dims, Ls = (4, 4, 2, 4), 6
    _flush("wall pseudofermion force")
    p, U, psi, op = _setup(torch, dims, Ls, mf=0.05, seed=12)
    rng = np.random.default_rng(13)
    phi = rng.normal(size=p.shape4()) + 1j * rng.normal(size=p.shape4())
    S, G, info, rc = op.force_wall(torch.from_numpy(phi).cuda(), tol=1e-13)
    assert rc == mobius.OK, info
    S_o, G_o, oinfo = orc.force_wall(p, U, phi, tol=1e-14)
    err = float(np.abs(G.cpu().numpy() - G_o).max() / np.abs(G_o).max())
    g5phi = phi * np.array([1, 1, -1, -1])[:, None]
    q, _ = orc.propagator4d(p, U, g5phi, tol=1e-14)
    S_ov = float(np.vdot(q, q).real)
    _flush(f"  S {S:.12e} oracle {S_o:.12e} |D_ov^-1 phi|^2 {S_ov:.12e}; gradient error {err:.1e}; "
           f"iters {info.iters}")
    assert abs(S - S_o) <= 1e-10 * abs(S_o) and abs(S - S_ov) <= 1e-9 * abs(S_ov)
    assert err <= 1e-9
    S2, G2, info2, rc = op.force_wall(torch.from_numpy(phi).cuda(), tol=1e-13, link_grad=False)
    assert rc == mobius.OK and G2 is None and S2 == S
    op.close()
