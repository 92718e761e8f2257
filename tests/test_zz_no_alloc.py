"""mobius_dslash_noalloc (the allocation-free variant of mobius_dslash /
mobius_dslash_dag) against the allocating entry point, through the C ABI:
identical results for every operator block, two calls in a row with the
second on a smaller input (a smaller lattice, fewer right-hand sides), and a
clear rejection of a call whose SCHUR temporaries exceed the fixed workspace."""
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


def _op(torch, dims, Ls, seed, nrhs):
    from paper_1206_5214_amd import inputs, mobius
    rng = np.random.default_rng(seed)
    U = inputs.random_links(dims, 0.5, rng)
    op = mobius.Operator(dims, Ls, 1.8, 0.02, 1.5, 0.5, torch.from_numpy(U).cuda())
    psi = np.stack([inputs.gaussian_spinor(dims, Ls, rng) for _ in range(nrhs)])
    return op, torch.from_numpy(psi).cuda()


def _compare_all_ops(torch, op, canon, nrhs):
    from paper_1206_5214_amd import mobius
    for prec in (0, 1, 2):
        even, odd = op.pack(canon, prec, nrhs)
        full = op.pack_full(canon, prec, nrhs)
        for dag in (False, True):
            cases = [(mobius.OP_SCHUR, 1, odd), (mobius.OP_HOP, 0, odd), (mobius.OP_HOP, 1, even),
                     (mobius.OP_M5, 1, odd), (mobius.OP_FULL, 0, full), (mobius.OP_SCHUR_RIGHT, 1, odd),
                     (mobius.OP_HOP_LEFT, 0, odd), (mobius.OP_HOP_LEFT, 1, even),
                     (mobius.OP_SCHUR_LEFT, 1, odd), (mobius.OP_SCHUR_COMPLEMENT, 1, odd)]
            for opk, outp, x in cases:
                want = op.dslash(x, outp, prec, op=opk, dag=dag, nrhs=nrhs)
                got = torch.full_like(want, 0xA5)  # stale contents must not matter
                op.dslash_noalloc(x, got, outp, prec, op=opk, dag=dag, nrhs=nrhs)
                torch.cuda.synchronize()
                assert torch.equal(got, want), ("noalloc differs", prec, dag, opk)


def test_noalloc_matches_dslash(torch_cuda):
    torch = torch_cuda
    _flush("noalloc: 4^4 x Ls 8, two right-hand sides")
    op, canon = _op(torch, (4, 4, 4, 4), 8, 3, 2)
    _compare_all_ops(torch, op, canon, 2)
    _flush("noalloc: second call, 2x2x2x4 x Ls 4, one right-hand side")
    op2, canon2 = _op(torch, (2, 2, 2, 4), 4, 4, 1)
    _compare_all_ops(torch, op2, canon2[0].contiguous(), 1)
    op.close()
    op2.close()


def test_noalloc_rejects_oversize(torch_cuda):
    from paper_1206_5214_amd import mobius
    torch = torch_cuda
    op, canon = _op(torch, (4, 4, 4, 4), 8, 5, 1)
    fb = op.field_bytes(mobius.F64)
    nrhs = (64 << 20) // (2 * fb) + 1          # two temporaries per rhs: just over 64 MiB
    x = op.new_field(mobius.F64)
    y = op.new_field(mobius.F64)
    rc = mobius.lib().mobius_dslash_noalloc(op._h, mobius.F64, mobius.OP_SCHUR, 1, 0, mobius._ptr(x),
                                            mobius._ptr(y), nrhs, None)
    assert rc == -22
    assert b"workspace" in mobius.lib().mobius_last_error()
    # within the limit it works (and equals the allocating call)
    want = op.dslash(x, 1, mobius.F64, op=mobius.OP_SCHUR)
    rc = mobius.lib().mobius_dslash_noalloc(op._h, mobius.F64, mobius.OP_SCHUR, 1, 0, mobius._ptr(x),
                                            mobius._ptr(y), 1, mobius._stream())
    assert rc == 0
    torch.cuda.synchronize()
    assert torch.equal(y, want)
    op.close()
