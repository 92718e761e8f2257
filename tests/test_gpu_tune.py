"""Autotuner of the hop launch parameters (mobius_tune): the chosen parameters
are valid, the operator's results do not change beyond rounding (the
candidates keep the order of the direction sum; only the compiler's choice of
fused multiply-adds may differ between the unrolled variants), and the cache
file is written and re-used."""
import sys

import numpy as np
import pytest

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def torch_cuda():
    import torch
    assert torch.cuda.is_available(), "GPU tests need an MI355X"
    return torch


def _op(torch, dims=(8, 8, 8, 8), Ls=8, seed=3):
    from paper_1206_5214_amd import inputs, mobius
    rng = np.random.default_rng(seed)
    U = torch.from_numpy(inputs.random_links(dims, 0.5, rng)).cuda()
    psi = torch.from_numpy(inputs.gaussian_spinor(dims, Ls, rng)).cuda()
    return mobius.Operator(dims, Ls, 1.8, 0.01, 1.5, 0.5, U), psi


# rounding-level bound on |after - before| / |before| per storage precision
ROUND = {0: 1e-14, 1: 1e-6, 2: 2e-3}


def test_tune_keeps_results(torch_cuda, monkeypatch):
    from paper_1206_5214_amd import mobius
    torch = torch_cuda
    monkeypatch.delenv("MOBIUS_TUNE_CACHE", raising=False)
    op, psi = _op(torch)
    for prec in (mobius.F64, mobius.F32, mobius.F16):
        e, o = op.pack(psi, prec)
        zero = op.new_field(prec)

        def outputs():
            return [op.unpack(op.dslash(o, 0, prec), zero, prec),
                    op.unpack(zero, op.dslash(e, 1, prec, dag=True), prec),
                    op.unpack(zero, op.dslash(o, 1, prec, op=mobius.OP_SCHUR), prec)]
        before = outputs()
        r = op.tune(prec, reps=3)
        print(f"prec {prec}: {r}", flush=True)
        assert r["prec"] == prec and r["prefetch"] in (0, 1, 2)
        assert r["stage_links"] in (0, 1) and r["xcd_remap"] in (0, 1) and r["nt_links"] in (0, 1)
        assert r["mfma"] in (0, 1)
        assert r["hop_us"] > 0
        after = outputs()
        for a, b in zip(before, after):
            rel = (torch.linalg.vector_norm(a - b) / torch.linalg.vector_norm(b)).item()
            assert rel <= ROUND[prec], (prec, rel)
    op.close()


def test_tune_cache(torch_cuda, monkeypatch, tmp_path):
    from paper_1206_5214_amd import mobius
    torch = torch_cuda
    cache = tmp_path / "tune.txt"
    monkeypatch.setenv("MOBIUS_TUNE_CACHE", str(cache))
    op, psi = _op(torch, dims=(8, 8, 4, 8), Ls=12)
    r1 = op.tune(mobius.F32, reps=3)
    text = cache.read_text()
    assert text.count("\n") == 1 and "Ls12" in text and "prec1" in text
    op.close()
    op2, _ = _op(torch, dims=(8, 8, 4, 8), Ls=12, seed=4)
    r2 = op2.tune(mobius.F32, reps=3)
    assert r2 == r1                       # taken from the cache, not re-timed
    assert cache.read_text() == text      # nothing appended
    sol, info, rc = op2.solve(psi, tol=1e-10, inner_prec=mobius.F32)
    assert rc == mobius.OK and info[0].true_resid <= 1e-10
    op2.close()


def test_tune_rejects_bad_precision(torch_cuda):
    from paper_1206_5214_amd import mobius
    torch = torch_cuda
    op, _ = _op(torch, dims=(4, 4, 4, 4))
    with pytest.raises(mobius.MobiusError):
        op.tune(7)
    op.close()


LAUNCH_VARIANTS = ([(pf, st, rm, nt, 0) for pf in (0, 1, 2) for st in (0, 1) for rm in (0, 1) for nt in (0, 1)]
                   + [(2, 1, rm, nt, 1) for rm in (0, 1) for nt in (0, 1)])


@pytest.mark.parametrize("prec", [0, 1, 2], ids=["f64", "f32", "f16"])
def test_every_launch_variant_vs_oracle(torch_cuda, orc, prec):
    """Each of the 28 candidates the tuner may pick (the last four: the FP16
    matrix-core colour multiply, the launch parameters alone elsewhere), set
    explicitly, gives the hop blocks (forward and adjoint, both parities) and
    the Schur operator within the storage precision's tolerance of the FP64
    oracle."""
    from oracle import Params
    from paper_1206_5214_amd import inputs, mobius
    torch = torch_cuda
    tol = {0: 1e-12, 1: 2e-5, 2: 4e-3}[prec]
    dims, Ls = (6, 4, 2, 4), 12
    p = Params(dims, Ls, 1.8, 0.05, 1.75, 0.75)
    rng = np.random.default_rng(21)
    U = inputs.random_links(dims, 0.6, rng)
    psi = inputs.gaussian_spinor(dims, Ls, rng)
    want = [orc.hop(p, U, psi, q, dag=d) for q in (0, 1) for d in (False, True)]
    want_schur = orc.schur(p, U, orc.restrict(p, psi, 1))
    op = mobius.Operator(dims, Ls, 1.8, 0.05, 1.75, 0.75, torch.from_numpy(U).cuda())
    e, o = op.pack(torch.from_numpy(psi).cuda(), prec)
    zero = op.new_field(prec)
    for v in LAUNCH_VARIANTS:
        op.set_tuning(prec, *v)
        got = []
        for q in (0, 1):
            for d in (False, True):
                src = o if q == 0 else e
                out = op.dslash(src, q, prec, dag=d)
                got.append(op.unpack(out, zero, prec) if q == 0 else op.unpack(zero, out, prec))
        for g, w in zip(got, want):
            g = g.cpu().numpy()
            assert np.linalg.norm(g - w) <= tol * np.linalg.norm(w), (v, prec)
        s = op.unpack(zero, op.dslash(o, 1, prec, op=mobius.OP_SCHUR), prec).cpu().numpy()
        assert np.linalg.norm(s - want_schur) <= tol * np.linalg.norm(want_schur), (v, prec)
    with pytest.raises(mobius.MobiusError):
        op.set_tuning(prec, 3, 0, 0, 0)
    with pytest.raises(mobius.MobiusError):
        op.set_tuning(prec, 2, 1, 0, 0, 2)
    op.close()


def test_tune_brick_and_explicit_site_order(torch_cuda, monkeypatch):
    """The layout tuner (mobius_tune_brick) times candidate site-order bricks,
    the automatic one first, and returns one of them; an operator created with
    an explicit brick, including one that does not divide the lattice, gives
    per site exactly the hops of the automatic order in every precision (the
    order only moves sites between workgroups) and solves to the same accuracy."""
    from paper_1206_5214_amd import inputs, mobius
    torch = torch_cuda
    monkeypatch.delenv("MOBIUS_TUNE_CACHE", raising=False)
    dims, Ls = (8, 8, 4, 4), 8
    rng = np.random.default_rng(21)
    U = torch.from_numpy(inputs.random_links(dims, 0.5, rng)).cuda()
    psi = torch.from_numpy(inputs.gaussian_spinor(dims, Ls, rng)).cuda()
    args = (dims, Ls, 1.8, 0.05, 1.5, 0.5)
    brick, us, trials = mobius.tune_brick(*args, U, prec=mobius.F16, reps=2)
    print(f"brick {brick} {us:.1f} us; trials {trials}", flush=True)
    assert 2 <= len(trials) <= 12 and all(t[1] > 0 for t in trials)
    assert brick in [t[0] for t in trials]
    for b, _ in trials[1:]:
        assert all(1 <= b[k] <= dims[k] and dims[k] % b[k] == 0 for k in range(3))
    auto_us = trials[0][1]
    assert (brick == trials[0][0] and us == auto_us) or us < 0.97 * auto_us
    op0 = mobius.Operator(*args, U)
    for b in ((2, 2, 2), (4, 8, 2), (6, 8, 4), brick):
        op1 = mobius.Operator(*args, U, brick=b)
        for prec in (mobius.F64, mobius.F32, mobius.F16):
            outs = []
            for op in (op0, op1):
                e, o = op.pack(psi, prec)
                zero = op.new_field(prec)
                outs.append([op.unpack(op.dslash(o, 0, prec), zero, prec),
                             op.unpack(zero, op.dslash(e, 1, prec, dag=True), prec)])
            for a, c in zip(*outs):
                assert torch.equal(a, c), (b, prec)
        sol, info, rc = op1.solve(psi, tol=1e-10, inner_prec=mobius.F16)
        assert rc == mobius.OK and info[0].true_resid <= 1e-10
        op1.close()
    op0.close()
