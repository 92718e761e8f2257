"""Pseudofermion force on the GPU (mobius_force and its torch.autograd
binding) against the FP64 CPU oracle and against central finite differences.

S = phi_o^+ (D_pre^+ D_pre)^-1 phi_o;  dS/dU (every link entry as an
independent complex number, gradient dS/dRe U + i dS/dIm U) and dS/dphi = 2X.
"""
import sys

import numpy as np
import pytest

pytestmark = pytest.mark.gpu


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


FORCE_CASES = [  # dims, Ls, b5, c5, mf, eps, seed
    ((4, 4, 4, 4), 8, 1.0, 0.0, 0.05, 0.5, 1),
    ((4, 4, 4, 4), 8, 1.5, 0.5, 0.01, 0.5, 2),
    ((6, 4, 2, 4), 12, 1.75, 0.75, 0.05, 0.6, 3),
    ((4, 2, 2, 6), 5, 1.5, 0.5, 0.1, 0.5, 4),
]


@pytest.mark.parametrize("case", FORCE_CASES, ids=lambda c: f"{c[0]}-Ls{c[1]}-b{c[2]}-c{c[3]}")
def test_force_vs_oracle(torch_cuda, orc, case):
    from oracle import Params
    from paper_1206_5214_amd import inputs, mobius
    torch = torch_cuda
    dims, Ls, b5, c5, mf, eps, seed = case
    _flush(f"force {dims} Ls={Ls} b5={b5} c5={c5}")
    p = Params(dims, Ls, 1.8, mf, b5, c5)
    rng = np.random.default_rng(seed)
    U = inputs.random_links(dims, eps, rng)
    phi = inputs.gaussian_spinor(dims, Ls, rng)  # even sites must be ignored
    S_o, X_o, G_o, info_o = orc.force(p, U, orc.restrict(p, phi, 1), tol=1e-14)
    assert info_o.converged
    op = mobius.Operator(dims, Ls, 1.8, mf, b5, c5, torch.from_numpy(U).cuda())
    S, G, gphi, info, rc = op.force(torch.from_numpy(phi).cuda(), tol=1e-12)
    assert rc == mobius.OK, info
    G, gphi = G.cpu().numpy(), gphi.cpu().numpy()
    _flush(f"  S {S:.12e} oracle {S_o:.12e}  iters {info.iters}")
    assert abs(S - S_o) <= 1e-10 * abs(S_o)
    assert _rel(gphi, 2 * X_o) <= 1e-10
    err = np.abs(G - G_o).max() / np.abs(G_o).max()
    _flush(f"  max |G - G_oracle| / max |G| = {err:.2e}")
    assert err <= 1e-9
    op.close()


def _apply_normal(torch, op, x_canon):
    """D_pre^+ D_pre on the odd half of a canonical field (GPU, FP64), canonical out."""
    from paper_1206_5214_amd import mobius
    e, o = op.pack(x_canon, mobius.F64)
    t = op.dslash(o, 1, mobius.F64, op=mobius.OP_SCHUR)
    q = op.dslash(t, 1, mobius.F64, op=mobius.OP_SCHUR, dag=True)
    return op.unpack(torch.zeros_like(e), q, mobius.F64)


def test_force_finite_differences_8x8x8x16(torch_cuda):
    """20 random links of the 8^3 x 16, Ls = 8 workload: the GPU gradient along a
    random complex direction E at each link against (S(U+hE) - S(U-hE)) / 2h,
    h = 1e-5, with the difference formed as <X+, (A- - A+) X-> (A = D_pre^+ D_pre,
    X+- its solutions at U +- hE) so that no cancellation limits the check."""
    from paper_1206_5214_amd import inputs, mobius
    torch = torch_cuda
    w = inputs.WORKLOADS["force_8x8x8x16_ls8"]
    U, _ = inputs.workload_fields(w, with_source=False)
    rng = np.random.default_rng(w.seed + 100)
    phi = torch.from_numpy(inputs.gaussian_spinor(w.dims, w.Ls, rng)).cuda()
    Ud = torch.from_numpy(U).cuda()
    args = (w.dims, w.Ls, w.M5, w.mf, w.b5, w.c5)
    op = mobius.Operator(*args, Ud)
    S, G, gphi, info, rc = op.force(phi, tol=1e-13, maxiter=50000)
    assert rc == mobius.OK, info
    _flush(f"force 8^3x16 Ls8: S {S:.10e}, {info.iters} iters, {info.seconds:.3f} s")
    op.close()
    V = int(np.prod(w.dims))
    h = 1e-5
    worst = 0.0
    for k in range(20):
        mu, site = int(rng.integers(4)), int(rng.integers(V))
        E = torch.zeros_like(Ud)
        e = rng.standard_normal((3, 3)) + 1j * rng.standard_normal((3, 3))
        E.view(4, V, 3, 3)[mu, site] = torch.from_numpy(e).cuda()
        opp = mobius.Operator(*args, Ud + h * E)
        opm = mobius.Operator(*args, Ud - h * E)
        _, _, gp, ip, rcp = opp.force(phi, tol=1e-13, maxiter=50000)
        _, _, gm, im, rcm = opm.force(phi, tol=1e-13, maxiter=50000)
        assert rcp == mobius.OK and rcm == mobius.OK
        Xp, Xm = gp / 2, gm / 2
        diff = _apply_normal(torch, opm, Xm) - _apply_normal(torch, opp, Xm)
        dS = torch.vdot(Xp.flatten(), diff.flatten()).real.item() / (2 * h)
        want = (torch.conj(G.view(4, V, 3, 3)[mu, site]) * E.view(4, V, 3, 3)[mu, site]).sum().real.item()
        rel = abs(dS - want) / max(abs(want), 1e-30)
        worst = max(worst, rel)
        _flush(f"  link ({mu},{site}): FD {dS:.10e} kernel {want:.10e} rel {rel:.1e}")
        assert rel <= 1e-6
        opp.close()
        opm.close()
    _flush(f"  worst relative difference {worst:.1e}")


def test_autograd_action(torch_cuda):
    """S.backward() through MobiusAction gives the library's gradients, scaled by
    the incoming gradient, for links and phi."""
    from paper_1206_5214_amd import autograd, inputs, mobius
    torch = torch_cuda
    dims, Ls = (4, 4, 4, 4), 8
    rng = np.random.default_rng(5)
    U = torch.from_numpy(inputs.random_links(dims, 0.5, rng)).cuda()
    phi = torch.from_numpy(inputs.gaussian_spinor(dims, Ls, rng)).cuda()
    Ul = U.clone().requires_grad_(True)
    ph = phi.clone().requires_grad_(True)
    S = autograd.action(Ul, ph, dims, Ls, 1.8, 0.05, 1.5, 0.5, tol=1e-12)
    (3.0 * S).backward()
    op = mobius.Operator(dims, Ls, 1.8, 0.05, 1.5, 0.5, U)
    S2, G, gphi, info, rc = op.force(phi, tol=1e-12)
    op.close()
    assert abs(S.item() - S2) <= 1e-12 * abs(S2)
    assert torch.allclose(Ul.grad, 3.0 * G, rtol=0, atol=1e-12 * G.abs().max().item())
    assert torch.allclose(ph.grad, 3.0 * gphi, rtol=0, atol=1e-12 * gphi.abs().max().item())
    # phi only: the links need no gradient, so the link-derivative pass is
    # skipped (an existing operator on the same links is reused)
    op = mobius.Operator(dims, Ls, 1.8, 0.05, 1.5, 0.5, U)
    ph2 = phi.clone().requires_grad_(True)
    S3 = autograd.action(U, ph2, dims, Ls, 1.8, 0.05, 1.5, 0.5, op=op)
    S3.backward()
    assert torch.allclose(ph2.grad, gphi, rtol=0, atol=1e-10 * gphi.abs().max().item())
    assert abs(S3.item() - S2) <= 1e-10 * abs(S2)
    S4, G4, gphi4, info4, rc = op.force(phi, tol=1e-12, link_grad=False)
    assert rc == mobius.OK and G4 is None
    assert S4 == S2 and torch.equal(gphi4, gphi)
    assert info4.dirac_apps == info.dirac_apps - 3
    op.close()


@pytest.mark.parametrize("inner", [1, 2], ids=["mixed_f32", "mixed_f16"])
def test_force_mixed_inner_solve(torch_cuda, inner):
    """A low-precision inner operator with FP64 reliable updates reaches the same
    force (the normal-equations residual is recomputed in FP64)."""
    from paper_1206_5214_amd import inputs, mobius
    torch = torch_cuda
    dims, Ls = (4, 4, 4, 8), 8
    rng = np.random.default_rng(6)
    U = torch.from_numpy(inputs.random_links(dims, 0.5, rng)).cuda()
    phi = torch.from_numpy(inputs.gaussian_spinor(dims, Ls, rng)).cuda()
    op = mobius.Operator(dims, Ls, 1.8, 0.01, 1.5, 0.5, U)
    S64, G64, p64, i64, rc = op.force(phi, tol=1e-12)
    assert rc == mobius.OK
    S, G, gp, info, rc = op.force(phi, tol=1e-12, inner_prec=inner)
    assert rc == mobius.OK, info
    _flush(f"  inner {inner}: iters {info.iters} ({i64.iters} FP64), reliable {info.reliable_updates}")
    assert abs(S - S64) <= 1e-10 * abs(S64)
    assert ((G - G64).abs().max() / G64.abs().max()).item() <= 1e-9
    op.close()


def test_force_rejects_bad_arguments(torch_cuda):
    from paper_1206_5214_amd import inputs, mobius
    torch = torch_cuda
    dims, Ls = (4, 4, 4, 4), 8
    op = mobius.Operator(dims, Ls, 1.8, 0.05, 1.5, 0.5, torch.from_numpy(inputs.unit_links(dims)).cuda())
    phi = torch.zeros(op.canon_shape(), dtype=torch.complex128, device="cuda")
    S, G, gphi, info, rc = op.force(phi)
    assert rc == mobius.OK and S == 0.0 and info.iters == 0
    assert torch.count_nonzero(G).item() == 0 and torch.count_nonzero(gphi).item() == 0
    with pytest.raises(mobius.MobiusError):
        op.force(phi[:2].contiguous())
    op.close()


def test_force_lie_vs_oracle(torch_cuda, orc):
    """F = TA(U G^+) per link on the GPU (mobius_force_lie) against the oracle's
    projection, for the force of the 4^4, Ls=8 lattice and for random G."""
    from paper_1206_5214_amd import inputs, mobius
    torch = torch_cuda
    dims, Ls = (4, 4, 4, 4), 8
    rng = np.random.default_rng(51)
    U = inputs.random_links(dims, 0.5, rng)
    op = mobius.Operator(dims, Ls, 1.8, 0.05, 1.5, 0.5, torch.from_numpy(U).cuda())
    G = rng.normal(size=U.shape) + 1j * rng.normal(size=U.shape)
    F = op.force_lie(torch.from_numpy(U).cuda(), torch.from_numpy(G).cuda()).cpu().numpy()
    want = orc.force_lie(U, G)
    err = float(np.abs(F - want).max() / np.abs(want).max())
    assert err < 1e-14, err
    import ctypes
    u = torch.from_numpy(U).cuda()
    assert mobius.lib().mobius_force_lie(op._h, mobius._ptr(u), mobius._ptr(u), mobius._ptr(u),
                                         None) == -22  # output aliases an input
    op.close()


@pytest.mark.parametrize("check", [0, 5], ids=["check8", "check5"])
def test_force_deferred_x_update(torch_cuda, monkeypatch, check):
    """The force's normal-equations CG with the x update deferred to the end of
    each chunk (FP16 inner operator) against the update in every iteration
    (MOBIUS_DEFER_X=0): same action and gradient to the solve's accuracy."""
    from paper_1206_5214_amd import inputs, mobius
    torch = torch_cuda
    dims, Ls = (4, 4, 4, 8), 8
    rng = np.random.default_rng(7)
    U = torch.from_numpy(inputs.random_links(dims, 0.5, rng)).cuda()
    phi = torch.from_numpy(inputs.gaussian_spinor(dims, Ls, rng)).cuda()
    op = mobius.Operator(dims, Ls, 1.8, 0.02, 1.5, 0.5, U)
    res = {}
    for d in ("1", "0"):
        monkeypatch.setenv("MOBIUS_DEFER_X", d)
        S, G, gp, info, rc = op.force(phi, tol=1e-12, inner_prec=mobius.F16, check_every=check)
        assert rc == mobius.OK, info
        res[d] = (S, G, info)
    S1, G1, i1 = res["1"]
    S0, G0, i0 = res["0"]
    dg = ((G1 - G0).abs().max() / G0.abs().max()).item()
    _flush(f"  check {check}: iters {i1.iters} / {i0.iters}, action diff {abs(S1 - S0) / abs(S0):.1e}, "
           f"gradient diff {dg:.1e}")
    assert abs(S1 - S0) <= 1e-10 * abs(S0) and dg <= 1e-9
    op.close()
