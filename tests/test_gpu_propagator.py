"""4d overlap propagator through the 5d solve (mobius_propagator4d) against the
FP64 CPU oracle: q = [P^+ D_DW(m)^-1 D_DW(1) P b]_1 = D_ov(m)^-1 b (Sec. 2.2).

The oracle's own route (oracle.propagator4d) is pinned by the free-field
closed form and by a dense D_ov on a small interacting lattice
(tests/pins.py); here the GPU result must match it to 1e-8 with random links,
and the closed form directly in the free field.
"""
import sys

import numpy as np
import pytest

pytestmark = pytest.mark.gpu

TOL = 1e-10
ERR = 1e-8


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


@pytest.mark.parametrize("inner", [0, 1, 2], ids=["f64", "mixed_f32", "mixed_f16"])
def test_propagator4d_vs_oracle(torch_cuda, orc, inner):
    """Two Gaussian 4d sources in one call on 4^4, Ls=8 (Moebius b5=1.5, c5=0.5)."""
    from oracle import Params
    from paper_1206_5214_amd import inputs, mobius
    torch = torch_cuda
    dims, Ls = (4, 4, 4, 4), 8
    _flush(f"propagator4d {dims} Ls={Ls} inner={inner}")
    rng = np.random.default_rng(21)
    U = inputs.random_links(dims, 0.5, rng)
    shape4 = (dims[3], dims[2], dims[1], dims[0], 4, 3)
    b = rng.normal(size=(2,) + shape4) + 1j * rng.normal(size=(2,) + shape4)
    p = Params(dims, Ls, 1.8, 0.01, 1.5, 0.5)
    op = mobius.Operator(dims, Ls, 1.8, 0.01, 1.5, 0.5, torch.from_numpy(U).cuda())
    q, info, rc = op.propagator4d(torch.from_numpy(b).cuda(), tol=TOL, maxiter=50000, inner_prec=inner)
    assert rc == mobius.OK, info
    q = q.cpu().numpy()
    want, oinfo = orc.propagator4d(p, U, b, tol=1e-13)
    assert all(i.converged for i in oinfo)
    for r in range(2):
        err = _rel(q[r], want[r])
        _flush(f"  rhs {r}: iters {info[r].iters} 5d resid {info[r].true_resid:.2e} err {err:.2e}")
        assert info[r].true_resid <= TOL
        assert err <= ERR, err
    op.close()


def test_propagator4d_free_field(torch_cuda):
    """Unit links: a plane wave e^{ipx} u comes back as e^{ipx} D_ov(p)^-1 u."""
    sys.path.insert(0, __file__.rsplit("/", 1)[0])
    import freefield as ff
    from paper_1206_5214_amd import inputs, mobius
    torch = torch_cuda
    dims, Ls, M5, mf, b5, c5 = (4, 4, 4, 8), 8, 1.8, 0.02, 1.5, 0.5
    U = inputs.unit_links(dims)
    op = mobius.Operator(dims, Ls, M5, mf, b5, c5, torch.from_numpy(U).cuda())
    rng = np.random.default_rng(22)
    for mom in [np.zeros(4)] + ff.momenta(dims, rng, 2):
        wave = ff.plane_wave(dims, mom)
        u = rng.normal(size=(4, 3)) + 1j * rng.normal(size=(4, 3))
        b = np.ascontiguousarray(wave[..., None, None] * u)
        q, info, rc = op.propagator4d(torch.from_numpy(b).cuda(), tol=1e-12, maxiter=50000)
        assert rc == mobius.OK, info
        want = wave[..., None, None] * (np.linalg.inv(ff.overlap_symbol(mom, M5, b5, c5, Ls, mf)) @ u)
        err = _rel(q.cpu().numpy(), want)
        _flush(f"  p = {np.round(mom, 3)}: iters {info[0].iters} err {err:.2e}")
        assert err <= 1e-9, err
    op.close()


def test_propagator4d_rejects_bad_arguments(torch_cuda):
    import ctypes
    from paper_1206_5214_amd import inputs, mobius
    torch = torch_cuda
    dims, Ls = (4, 4, 4, 4), 4
    op = mobius.Operator(dims, Ls, 1.8, 0.1, 1.0, 0.0, torch.from_numpy(inputs.unit_links(dims)).cuda())
    b = torch.zeros((4, 4, 4, 4, 4, 3), dtype=torch.complex128, device="cuda")
    with pytest.raises(mobius.MobiusError):
        op.propagator4d(b[..., :2, :].contiguous())              # wrong shape
    with pytest.raises(mobius.MobiusError):
        op.propagator4d(b.to(torch.complex64))                    # wrong dtype
    opts = mobius._SolveOpts(1e-10, 100, 0, 0.0, 1, 0)
    infos = (mobius._SolveInfo * 1)()
    L = mobius.lib()
    assert L.mobius_propagator4d(op._h, mobius._ptr(b), mobius._ptr(b), ctypes.byref(opts), infos,
                                 None) == -22  # source and solution alias (MOBIUS_EINVAL)
    assert L.mobius_propagator4d(op._h, None, mobius._ptr(b), ctypes.byref(opts), infos,
                                 None) == -22
    op.close()


@pytest.mark.parametrize("inner", [0, 2], ids=["f64", "mixed_f16"])
def test_bulk5d_vs_oracle(torch_cuda, orc, inner):
    """Overlap to bulk reconstruction (mobius_bulk5d, Sec. 2.3): from the
    overlap solution psi = D_ov^-1 b, the 5d field Psi = P^+ D(m)^-1 D(1) P B
    with one Pauli-Villars solve, against the oracle's route and against the
    5d equation D(m) P Psi = D(1) P B recomputed with the oracle's D_DW; two
    right-hand sides in one call."""
    from oracle import Params
    from paper_1206_5214_amd import inputs, mobius
    torch = torch_cuda
    dims, Ls = (4, 4, 4, 4), 8
    p = Params(dims, Ls, 1.8, 0.02, 1.5, 0.5)
    rng = np.random.default_rng(61)
    U = inputs.random_links(dims, 0.4, rng)
    b = rng.normal(size=(2,) + p.shape4()) + 1j * rng.normal(size=(2,) + p.shape4())
    psi, _ = orc.propagator4d(p, U, b, tol=1e-13)
    op = mobius.Operator(dims, Ls, 1.8, 0.02, 1.5, 0.5, torch.from_numpy(U).cuda())
    Psi, infos, rc = op.bulk5d(torch.from_numpy(psi).cuda(), tol=1e-12, inner_prec=inner)
    assert rc == mobius.OK, infos
    got = Psi.cpu().numpy()
    want, _, _ = orc.bulk5d(p, U, psi, tol=1e-13)
    p1 = Params(dims, Ls, 1.8, 1.0, 1.5, 0.5)
    for r in range(2):
        err = float(np.linalg.norm(got[r] - want[r]) / np.linalg.norm(want[r]))
        X = got[r].copy()                                  # X = P Psi
        X[:, ..., :2, :] = np.roll(got[r], -1, axis=0)[:, ..., :2, :]
        B = np.zeros(p.shape5(), complex)                  # P B
        B[0, ..., 2:, :] = b[r][..., 2:, :]
        B[-1, ..., :2, :] = b[r][..., :2, :]
        lhs, rhs = orc.dw(p, U, X), orc.dw(p1, U, B)
        res = float(np.linalg.norm(lhs - rhs) / np.linalg.norm(rhs))
        _flush(f"  rhs {r}: PV iters {infos[r].iters}, error vs oracle {err:.2e}, 5d residual {res:.2e}")
        assert err <= 1e-9 and res <= 1e-9
    op.close()
