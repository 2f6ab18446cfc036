"""GPU parity of the time-slab decomposition preconditioner (non-overlapping
time decomposition: the exact inverse of each slab's own Galerkin problem)
against the oracle's slab solve: 1e-10 relative in complex128 and 2e-4 in
complex64 on ragged meshes of every dimension and potential kind, and at the
full 2+1D 128^3 packet size (the oracle solves each slab spectrally there);
GMRES with it follows the oracle's GMRES with the same preconditioner step by
step; the batched solver with it reproduces the single-system solves.
"""
import numpy as np
import pytest
import torch

from oracle import oracle as O
from paper_2103_14588_amd import inputs as IN

pytestmark = pytest.mark.gpu

CASES = [
    (IN.Spec(d=1, n=[8, 37], lens=[0.8, 1.3]), 2),
    (IN.Spec(d=1, n=[6, 5], vkind=1, v0=2.0, x0=0.5), 3),
    (IN.Spec(d=1, n=[9, 10], vkind=2, v0=3.0, x0=0.4, lw=0.05), 9),
    (IN.Spec(d=2, n=[6, 17, 9], lens=[1.0, 0.9, 1.1], m=0.7), 2),
    (IN.Spec(d=2, n=[8, 12, 11], vkind=1, v0=2.5, x0=0.5), 4),
    (IN.Spec(d=2, n=[6, 9, 10], vkind=2, v0=1.5, x0=0.4, lw=0.05), 3),
    (IN.Spec(d=3, n=[4, 5, 3, 6]), 2),
    (IN.Spec(d=3, n=[6, 4, 4, 3], vkind=1, v0=1.0, x0=0.3), 3),
]


def ids(c):
    s, k = c
    return "d%d_%s_v%d_k%d" % (s.d, "x".join(map(str, s.n)), s.vkind, k)


@pytest.fixture(scope="module")
def D():
    from paper_2103_14588_amd import dirac_st as D
    assert torch.cuda.is_available()
    return D


def oprob(spec):
    return O.problem(spec.d, spec.n, spec.lens, spec.m, spec.vkind, spec.v0, spec.x0, spec.lw)


def dev(a):
    return torch.from_numpy(np.ascontiguousarray(a)).cuda()


def host(t):
    torch.cuda.synchronize()
    return t.cpu().numpy()


def rand_c(n, seed):
    rng = np.random.default_rng(seed)
    return rng.standard_normal(n) + 1j * rng.standard_normal(n)


@pytest.mark.parametrize("case", CASES, ids=ids)
def test_time_slabs_match_oracle(D, case):
    spec, slabs = case
    op, _ = D.assemble(spec, None)
    p = oprob(spec)
    v = rand_c(op.n, 3)
    want = O.time_slab_solve(p, v, slabs)
    z = host(D.pc_apply(op, dev(v), pc="slabs", slabs=slabs))
    assert np.linalg.norm(z - want) <= 1e-10 * np.linalg.norm(want)
    v32 = v.astype(np.complex64)
    want32 = O.time_slab_solve(p, v32.astype(np.complex128), slabs)
    z32 = host(D.pc_apply(op, dev(v32), pc="slabs", slabs=slabs)).astype(np.complex128)
    assert np.linalg.norm(z32 - want32) <= 2e-4 * np.linalg.norm(want32)


def test_one_slab_is_the_line_preconditioner(D):
    spec = IN.Spec(d=2, n=[6, 12, 11], vkind=1, v0=2.5, x0=0.5)
    op, _ = D.assemble(spec, None)
    v = dev(rand_c(op.n, 4))
    assert torch.equal(D.pc_apply(op, v, pc="slabs", slabs=1), D.pc_apply(op, v, pc="line"))


def test_time_slabs_reject_a_count_that_does_not_divide_n_t(D):
    spec = IN.Spec(d=1, n=[8, 5])
    op, b = D.assemble(spec, None)
    v = dev(rand_c(op.n, 5))
    for bad in (0, 3, 16):
        with pytest.raises(D.DiracError):
            D.pc_apply(op, v, pc="slabs", slabs=bad)
        with pytest.raises(D.DiracError):
            D.gmres(op, v, pc="slabs", slabs=bad, max_it=2)


def test_time_slabs_full_size_packet(D):
    """2+1D 128^3 packet (V = 0), four slabs of 32 time rows: the output equals
    the oracle's spectral solve of every slab problem."""
    wl = IN.packet_2p1(128, 0)
    op, b = D.assemble(wl.spec, dev(wl.psi0))
    p = oprob(wl.spec)
    bh = host(b)
    want = O.time_slab_solve(p, bh, 4)
    z = host(D.pc_apply(op, b, pc="slabs", slabs=4))
    assert np.linalg.norm(z - want) <= 1e-10 * np.linalg.norm(want)
    z32 = host(D.pc_apply(op, b.to(torch.complex64), pc="slabs", slabs=4)).astype(np.complex128)
    assert np.linalg.norm(z32 - want) <= 1e-3 * np.linalg.norm(want)


def test_gmres_with_time_slabs_follows_oracle(D):
    """Klein step 2+1D (ragged 8 x 12 x 10), two slabs: the Arnoldi residual
    estimates of the device GMRES equal those of the oracle's GMRES with the
    oracle's slab solve as preconditioner, step by step."""
    spec = IN.Spec(d=2, n=[8, 12, 10], vkind=1, v0=2.5, x0=0.5)
    psi = IN.gaussian_packet(spec, [0.3, 0.5], [6.0, 1.0], 0.15, IN.positive_energy_spinor([6.0, 1.0], spec.m, 2))
    op, b = D.assemble(spec, dev(psi))
    p = oprob(spec)
    A = O.Matrix(p)
    bo = A.rhs(psi)
    steps = 30
    _, io = A.gmres(bo, restart=15, max_it=steps, rtol=1e-14, pc="fn",
                    pcfn=lambda v: O.time_slab_solve(p, v, 2), history=True)
    x, info = D.gmres(op, b, restart=15, max_it=steps, rtol=1e-14, pc="slabs", slabs=2, history=steps)
    h_or, h = np.array(io["history"]), np.array(info["history"])
    assert len(h) == len(h_or) == steps
    assert np.all(np.abs(h - h_or) <= 1e-7 * h_or + 1e-13), np.c_[h, h_or]


def test_batched_with_time_slabs(D):
    """An uneven batch (every n_t divisible by the slab count): each system's
    result equals its single-system solve with the same options."""
    specs = [IN.Spec(d=2, n=[4, 9, 10], vkind=1, v0=0.4, x0=0.5), IN.Spec(d=2, n=[6, 12, 11], vkind=1, v0=2.9, x0=0.5),
             IN.Spec(d=2, n=[8, 17, 9], vkind=1, v0=1.7, x0=0.5)]
    ops, bs = [], []
    for i, s in enumerate(specs):
        rng = np.random.default_rng(20 + i)
        c, pm = rng.uniform(0.3, 0.7, s.d), rng.uniform(2.0, 6.0, s.d)
        psi = IN.gaussian_packet(s, c, pm, 0.15, IN.positive_energy_spinor(pm, s.m, s.nc))
        op, b = D.assemble(s, dev(psi))
        ops.append(op)
        bs.append(b)
    kw = dict(restart=12, max_it=36, rtol=1e-10, pc="slabs", slabs=2)
    xs, infos, rc = D.fgmres_batched(ops, bs, **kw)
    for op, b, x, inf in zip(ops, bs, xs, infos):
        x1, i1 = D.gmres(op, b, **kw)
        assert inf["iters"] == i1["iters"], (inf, i1)
        assert float(torch.linalg.vector_norm(x - x1) / torch.linalg.vector_norm(x1)) <= 1e-9
