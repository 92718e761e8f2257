"""Multi-RHS and uneven-batch solves on the GPU (mobius_cg_solve with nrhs > 1,
mobius_batch_solve) against the FP64 CPU oracle.

Every system must reach the full-system true residual 1e-10, recomputed here
with the oracle's own D_DW, and (where the oracle can solve the system in
seconds) match the oracle's solution to 1e-8.
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


def _check_system(orc, p, U, eta, psi, info, solve_oracle=True):
    res = _rel(orc.dw(p, U, psi), eta)
    assert res <= TOL, (res, info)
    assert abs(res - info.true_resid) <= 1e-11 + 0.05 * res, (res, info)
    if solve_oracle:
        psi_o, oi = orc.solve(p, U, eta, tol=1e-13, maxiter=50000)
        assert oi.converged
        err = _rel(psi, psi_o)
        assert err <= ERR, err
        return res, err
    return res, None


@pytest.mark.parametrize("inner", [0, 1, 2], ids=["f64", "mixed_f32", "mixed_f16"])
def test_point_sources_multi_rhs_vs_oracle(torch_cuda, orc, inner):
    """12 spin-colour point sources in one solve (links read once per 4d site
    for all 12 right-hand sides)."""
    from oracle import Params
    from paper_1206_5214_amd import inputs, mobius
    torch = torch_cuda
    dims, Ls = (4, 4, 4, 8), 8
    _flush(f"multi-rhs 12 point sources {dims} Ls={Ls} inner={inner}")
    p = Params(dims, Ls, 1.8, 0.01, 1.5, 0.5)
    U = inputs.random_links(dims, 0.5, np.random.default_rng(7))
    eta = inputs.wall_point_sources(dims, Ls)
    op = mobius.Operator(dims, Ls, 1.8, 0.01, 1.5, 0.5, torch.from_numpy(U).cuda())
    sol, info, rc = op.solve(torch.from_numpy(eta).cuda(), tol=TOL, maxiter=20000, inner_prec=inner)
    assert rc == mobius.OK, info
    assert len(info) == 12
    psi = sol.cpu().numpy()
    for a in range(12):
        res, err = _check_system(orc, p, U, eta[a], psi[a], info[a])
        _flush(f"  rhs {a}: iters {info[a].iters} resid {res:.2e} err {err:.2e}")
    # one right-hand side alone gives the same solution (to the tolerance)
    s1, i1, rc1 = op.solve(torch.from_numpy(np.ascontiguousarray(eta[5])).cuda(), tol=TOL,
                           maxiter=20000, inner_prec=inner)
    assert rc1 == mobius.OK
    assert _rel(s1.cpu().numpy(), psi[5]) <= 2 * ERR
    op.close()


UNEVEN = [  # dims, Ls, b5, c5, mf, eps, seed
    ((4, 4, 4, 4), 8, 1.5, 0.5, 0.01, 0.5, 1),
    ((6, 6, 4, 4), 8, 1.5, 0.5, 0.01, 0.5, 2),
    ((8, 4, 4, 4), 12, 1.75, 0.75, 0.005, 0.6, 3),
]


@pytest.mark.parametrize("inner", [0, 1, 2], ids=["f64", "mixed_f32", "mixed_f16"])
@pytest.mark.parametrize("nrhs", [1, 2])
def test_uneven_batch_vs_oracle(torch_cuda, orc, inner, nrhs):
    """Lattices of different volume and Ls in one lockstep solve (one persistent
    hop launch over all lattices per operator application)."""
    from oracle import Params
    from paper_1206_5214_amd import inputs, mobius
    torch = torch_cuda
    _flush(f"uneven batch nrhs={nrhs} inner={inner}")
    ops, srcs, host = [], [], []
    for dims, Ls, b5, c5, mf, eps, seed in UNEVEN:
        rng = np.random.default_rng(seed)
        U = inputs.random_links(dims, eps, rng)
        eta = inputs.gaussian_spinor(dims, Ls, rng, nrhs if nrhs > 1 else None)
        ops.append(mobius.Operator(dims, Ls, 1.8, mf, b5, c5, torch.from_numpy(U).cuda()))
        srcs.append(torch.from_numpy(eta).cuda())
        host.append((Params(dims, Ls, 1.8, mf, b5, c5), U, eta))
    sols, infos, rc = mobius.batch_solve(ops, srcs, tol=TOL, maxiter=20000, inner_prec=inner)
    assert rc == mobius.OK, infos
    for j, (p, U, eta) in enumerate(host):
        psi = sols[j].cpu().numpy()
        for r in range(nrhs):
            e = eta if nrhs == 1 else eta[r]
            x = psi if nrhs == 1 else psi[r]
            res, err = _check_system(orc, p, U, e, x, infos[j][r])
            _flush(f"  lattice {j} rhs {r}: iters {infos[j][r].iters} resid {res:.2e} err {err:.2e}")
    for op in ops:
        op.close()


def test_graph_replay_matches_eager(torch_cuda, monkeypatch):
    """Iteration chunks captured in a hipGraph give bit-identical results to the
    same launches issued one by one."""
    from paper_1206_5214_amd import inputs, mobius
    torch = torch_cuda
    outs = []
    for graph in ("1", "0", "1"):
        monkeypatch.setenv("MOBIUS_GRAPH", graph)
        ops, srcs = [], []
        for dims, Ls, b5, c5, mf, eps, seed in UNEVEN[:2]:
            rng = np.random.default_rng(seed)
            U = inputs.random_links(dims, eps, rng)
            eta = inputs.gaussian_spinor(dims, Ls, rng, 2)
            ops.append(mobius.Operator(dims, Ls, 1.8, mf, b5, c5, torch.from_numpy(U).cuda()))
            srcs.append(torch.from_numpy(eta).cuda())
        sols, infos, rc = mobius.batch_solve(ops, srcs, tol=TOL, maxiter=20000,
                                             inner_prec=mobius.F32, check_every=4)
        assert rc == mobius.OK
        outs.append(([s.cpu() for s in sols], [[i.iters for i in g] for g in infos]))
        _flush(f"  graph={graph}: iters {outs[-1][1]}")
        for op in ops:
            op.close()
    for k in (1, 2):
        assert outs[k][1] == outs[0][1]
        for a, b in zip(outs[k][0], outs[0][0]):
            assert torch.equal(a, b)


def test_batch_solve_rejects_bad_arguments(torch_cuda):
    from paper_1206_5214_amd import inputs, mobius
    torch = torch_cuda
    dims, Ls = (4, 4, 4, 4), 8
    U = torch.from_numpy(inputs.unit_links(dims)).cuda()
    op = mobius.Operator(dims, Ls, 1.8, 0.01, 1.5, 0.5, U)
    src = torch.zeros(op.canon_shape(), dtype=torch.complex128, device="cuda")
    with pytest.raises(mobius.MobiusError):
        mobius.batch_solve([op, op], [src, src.clone()])
    with pytest.raises(mobius.MobiusError):
        mobius.batch_solve([op], [])
    op.close()


def test_uneven_batch_full_size(torch_cuda, orc):
    """The 8^4 + 12^4 + 16^4, Ls = 8 batch at full size, FP32 operator with FP64
    reliable updates: every system's true residual recomputed by the oracle."""
    from oracle import Params
    from paper_1206_5214_amd import inputs, mobius
    torch = torch_cuda
    ops, srcs, host = [], [], []
    for w in inputs.UNEVEN_BATCH:
        U, eta = inputs.workload_fields(w)
        ops.append(mobius.Operator(w.dims, w.Ls, w.M5, w.mf, w.b5, w.c5, torch.from_numpy(U).cuda()))
        srcs.append(torch.from_numpy(eta).cuda())
        host.append((Params(w.dims, w.Ls, w.M5, w.mf, w.b5, w.c5), U, eta))
    _flush("uneven batch 8^4 12^4 16^4 Ls=8 FP32")
    sols, infos, rc = mobius.batch_solve(ops, srcs, tol=TOL, maxiter=20000, inner_prec=mobius.F32)
    assert rc == mobius.OK, infos
    for j, (p, U, eta) in enumerate(host):
        psi = sols[j].cpu().numpy()
        res, _ = _check_system(orc, p, U, eta, psi, infos[j][0], solve_oracle=False)
        _flush(f"  lattice {p.dims}: iters {infos[j][0].iters} resid {res:.2e} "
               f"{infos[j][0].seconds:.3f} s")
    for op in ops:
        op.close()


def test_point_sources_full_size_sampled(torch_cuda, orc):
    """12 point sources on 16^3 x 32, Ls = 16 in one FP32-operator solve; the
    oracle recomputes the true residual of three sampled right-hand sides."""
    from oracle import Params
    from paper_1206_5214_amd import inputs, mobius
    torch = torch_cuda
    w = inputs.MULTI_RHS
    U, _ = inputs.workload_fields(w, with_source=False)
    op = mobius.Operator(w.dims, w.Ls, w.M5, w.mf, w.b5, w.c5, torch.from_numpy(U).cuda())
    src = torch.from_numpy(inputs.wall_point_sources(w.dims, w.Ls)).cuda()
    _flush("multi-rhs 16^3x32 Ls=16, 12 point sources, FP32")
    sol, info, rc = op.solve(src, tol=TOL, maxiter=50000, inner_prec=mobius.F32)
    assert rc == mobius.OK, info
    p = Params(w.dims, w.Ls, w.M5, w.mf, w.b5, w.c5)
    for a in (0, 5, 11):
        eta = src[a].cpu().numpy()
        psi = sol[a].cpu().numpy()
        res, _ = _check_system(orc, p, U, eta, psi, info[a], solve_oracle=False)
        _flush(f"  rhs {a}: iters {info[a].iters} resid {res:.2e}")
    op.close()


@pytest.mark.parametrize("inner", [1, 2], ids=["mixed_f32", "mixed_f16"])
def test_multi_rhs_12x12x12x12_ls16(torch_cuda, orc, inner):
    """Several right-hand sides on a lattice large enough that many workgroups
    share each CU (the case whose FP16 outputs were corrupted while the
    per-system norms were fused into the multi-RHS hop kernel)."""
    from oracle import Params
    from paper_1206_5214_amd import inputs, mobius
    torch = torch_cuda
    dims, Ls = (12, 12, 12, 12), 16
    rng = np.random.default_rng(0)
    U = inputs.random_links(dims, 0.5, rng)
    eta = inputs.gaussian_spinor(dims, Ls, rng, 3)
    op = mobius.Operator(dims, Ls, 1.8, 0.01, 1.5, 0.5, torch.from_numpy(U).cuda())
    _flush(f"multi-rhs 12^4 Ls16 nrhs 3 inner {inner}")
    sol, info, rc = op.solve(torch.from_numpy(eta).cuda(), tol=TOL, maxiter=50000, inner_prec=inner)
    assert rc == mobius.OK, info
    p = Params(dims, Ls, 1.8, 0.01, 1.5, 0.5)
    psi = sol.cpu().numpy()
    for r in range(3):
        res, _ = _check_system(orc, p, U, eta[r], psi[r], info[r], solve_oracle=False)
        _flush(f"  rhs {r}: iters {info[r].iters} resid {res:.2e}")
    op.close()


@pytest.mark.parametrize("inner", [1, 2], ids=["mixed_f32", "mixed_f16"])
def test_batch_systems_match_single_solves(torch_cuda, orc, inner):
    """In a batch every system takes its reliable updates at its own threshold
    (the others sit the update out), so each system runs exactly the
    iterations of its solo solve and reaches the same solution: a batch of
    three sources of very different character (Gaussian, point, scaled
    Gaussian) against three single solves."""
    from oracle import Params
    from paper_1206_5214_amd import inputs, mobius
    torch = torch_cuda
    dims, Ls = (8, 8, 8, 8), 8
    _flush(f"batch vs single solves {dims} Ls={Ls} inner={inner}")
    rng = np.random.default_rng(11)
    U = inputs.random_links(dims, 0.5, rng)
    gauss = inputs.gaussian_spinor(dims, Ls, rng, 2)
    point = inputs.wall_point_sources(dims, Ls)[5]
    eta = np.stack([gauss[0], point, 1e3 * gauss[1]])
    op = mobius.Operator(dims, Ls, 1.8, 0.01, 1.5, 0.5, torch.from_numpy(U).cuda())
    sol_b, info_b, rc = op.solve(torch.from_numpy(eta).cuda(), tol=TOL, maxiter=50000, inner_prec=inner)
    assert rc == mobius.OK, info_b
    psi_b = sol_b.cpu().numpy()
    p = Params(dims, Ls, 1.8, 0.01, 1.5, 0.5)
    for r in range(3):
        sol_1, info_1, rc1 = op.solve(torch.from_numpy(eta[r]).cuda(), tol=TOL, maxiter=50000,
                                      inner_prec=inner)
        assert rc1 == mobius.OK, info_1
        _flush(f"  rhs {r}: batch {info_b[r].iters} it / {info_b[r].reliable_updates} ru, "
               f"single {info_1[0].iters} it / {info_1[0].reliable_updates} ru")
        assert info_b[r].iters == info_1[0].iters
        assert info_b[r].reliable_updates == info_1[0].reliable_updates
        assert _rel(psi_b[r], sol_1.cpu().numpy()) <= 1e-12
        _check_system(orc, p, U, eta[r], psi_b[r], info_b[r], solve_oracle=False)
    op.close()


@pytest.mark.parametrize("inner", [1, 2], ids=["mixed_f32", "mixed_f16"])
def test_uneven_batch_deferred_x_update(torch_cuda, monkeypatch, inner):
    """An uneven batch (one persistent hop launch over several lattices, whose
    per-slot descriptors read the chunk's ring of directions) with the x update
    deferred to the end of each chunk against the update in every iteration:
    both converge to the same solutions to the solve's accuracy, and runs cut by
    maxiter in mid-chunk return the same iterates."""
    from paper_1206_5214_amd import inputs, mobius
    torch = torch_cuda
    _flush(f"uneven batch, deferred x update, inner {inner}")
    ops, srcs = [], []
    for dims, Ls, b5, c5, mf, eps, seed in UNEVEN[:2]:
        rng = np.random.default_rng(seed)
        U = inputs.random_links(dims, eps, rng)
        ops.append(mobius.Operator(dims, Ls, 1.8, mf, b5, c5, torch.from_numpy(U).cuda()))
        srcs.append(torch.from_numpy(inputs.gaussian_spinor(dims, Ls, rng, 2)).cuda())
    out = {}
    for d in ("1", "0"):
        monkeypatch.setenv("MOBIUS_DEFER_X", d)
        sols, infos, rc = mobius.batch_solve(ops, srcs, tol=TOL, maxiter=20000, inner_prec=inner,
                                             check_every=5)
        assert rc == mobius.OK, infos
        cut, cinfos, crc = mobius.batch_solve(ops, srcs, tol=TOL, maxiter=13, inner_prec=inner,
                                              check_every=5)
        assert crc == mobius.NOT_CONVERGED
        out[d] = ([s.cpu() for s in sols], infos, [c.cpu() for c in cut])
        for j, g in enumerate(infos):
            assert all(i.true_resid <= TOL for i in g), g
    for j in range(len(ops)):
        for r in range(2):
            a, b = out["1"][0][j][r], out["0"][0][j][r]
            diff = ((a - b).norm() / b.norm()).item()
            ca, cb = out["1"][2][j][r], out["0"][2][j][r]
            cdiff = ((ca - cb).norm() / cb.norm()).item()
            _flush(f"  lattice {j} rhs {r}: iters {out['1'][1][j][r].iters} / {out['0'][1][j][r].iters}, "
                   f"solutions differ by {diff:.1e}, 13-iteration iterates by {cdiff:.1e}")
            assert diff <= 1e-8 and cdiff <= 1e-5
    for op in ops:
        op.close()
