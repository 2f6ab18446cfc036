"""GPU parity of the matrix-free operator (the assembled operator applied as
1D stencils, no stored blocks) against the oracle: the product equals the
oracle's SpMV (1e-13 in complex128, 1e-5 in complex64) on ragged meshes of
every dimension and potential; at the full 2+1D 128^3 and 3+1D 32^4 sizes on
rows sampled across the time ends and the periodic seams, each computed by the
oracle from its own block row; the right-hand side equals the oracle's; GMRES
and BiCGSTAB with matrix_free on an operator without stored arrays land on the
same solution as the stored-block solves.
"""
import numpy as np
import pytest
import torch

from oracle import oracle as O
from paper_2103_14588_amd import inputs as IN

pytestmark = pytest.mark.gpu

CASES = [
    IN.Spec(d=1, n=[7, 37], lens=[0.8, 1.3]),
    IN.Spec(d=1, n=[1, 5]),
    IN.Spec(d=1, n=[2, 3], vkind=1, v0=2.0, x0=0.5),
    IN.Spec(d=1, n=[5, 300], vkind=2, v0=3.0, x0=0.4, lw=0.05),
    IN.Spec(d=2, n=[6, 17, 9], lens=[1.0, 0.9, 1.1], m=0.7),
    IN.Spec(d=2, n=[5, 70, 11], vkind=1, v0=2.5, x0=0.5),
    IN.Spec(d=2, n=[4, 9, 10], vkind=2, v0=1.5, x0=0.4, lw=0.05),
    IN.Spec(d=2, n=[1, 3, 3]),
    IN.Spec(d=3, n=[4, 5, 3, 6]),
    IN.Spec(d=3, n=[3, 4, 4, 3], vkind=1, v0=1.0, x0=0.3),
]


def ids(s):
    return "d%d_%s_v%d" % (s.d, "x".join(map(str, s.n)), s.vkind)


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


@pytest.mark.parametrize("spec", CASES, ids=ids)
def test_spmv_mf_matches_oracle(D, spec):
    A = O.Matrix(oprob(spec))
    x = rand_c(A.N, 11)
    y_or = A.spmv(x)
    y = host(D.spmv_mf(spec, dev(x)))
    assert np.linalg.norm(y - y_or) <= 1e-13 * np.linalg.norm(y_or)
    # complex64: against the FP64 product of the rounded input
    x32 = x.astype(np.complex64)
    y_ref = A.spmv(x32.astype(np.complex128))
    y32 = host(D.spmv_mf(spec, dev(x32))).astype(np.complex128)
    assert np.linalg.norm(y32 - y_ref) <= 1e-5 * np.linalg.norm(y_ref)


@pytest.mark.parametrize("spec", CASES, ids=ids)
def test_rhs_mf_matches_oracle(D, spec):
    A = O.Matrix(oprob(spec))
    psi0 = rand_c(spec.spatial * spec.nc, 12)
    b_or = A.rhs(psi0)
    b = host(D.rhs_mf(spec, dev(psi0)))
    assert np.linalg.norm(b - b_or) <= 1e-13 * np.linalg.norm(b_or)


def sampled_rows(spec, count, seed):
    """Rows at the time ends and the periodic seams of every axis, plus random ones."""
    nt, ns = spec.n[0], spec.n[1:]
    S = spec.spatial
    rng = np.random.default_rng(seed)
    rows = set()
    for tau in (1, 2, nt - 1, nt):
        for corner in range(2 ** spec.d):
            s, stride = 0, 1
            for a in range(spec.d):
                s += (ns[a] - 1 if (corner >> a) & 1 else 0) * stride
                stride *= ns[a]
            rows.add((tau - 1) * S + s)
    rows.update(int(r) for r in rng.integers(0, nt * S, count))
    return sorted(rows)


@pytest.mark.parametrize("spec", [
    IN.Spec(d=2, n=[128, 128, 128]),
    IN.Spec(d=2, n=[128, 128, 128], vkind=1, v0=2.5, x0=0.5),
    IN.Spec(d=3, n=[32, 32, 32, 32]),
], ids=ids)
def test_spmv_mf_full_size_sampled(D, spec):
    """Full-size product, checked on ~1000 rows that the oracle computes one
    by one from the elements containing the row node."""
    p = oprob(spec)
    nc = spec.nc
    N = spec.n[0] * spec.spatial * nc
    gen = torch.Generator(device="cuda").manual_seed(3)
    x = torch.randn(N, dtype=torch.complex128, device="cuda", generator=gen)
    y = host(D.spmv_mf(spec, x))
    xh = host(x).reshape(-1, nc)
    y = y.reshape(-1, nc)
    for r in sampled_rows(spec, 1000, 4):
        cols, blocks = O.row(p, r)
        keep = cols >= 0
        want = np.einsum("kij,kj->i", blocks[keep], xh[cols[keep]])
        assert np.linalg.norm(y[r] - want) <= 1e-13 * max(np.linalg.norm(want), 1e-300), r


@pytest.mark.parametrize("solver", ["gmres", "bicgstab"])
def test_solvers_matrix_free_without_stored_arrays(D, solver):
    """Klein step 2+1D: the solve on an operator with no stored arrays
    (matrix_free) equals the solve with the stored blocks; the spectral and
    line preconditioners need only the problem."""
    spec = IN.Spec(d=2, n=[10, 20, 14], vkind=1, v0=2.5, x0=0.5)
    psi = IN.gaussian_packet(spec, [0.3, 0.5], [6.0, 1.0], 0.15, IN.positive_energy_spinor([6.0, 1.0], spec.m, 2))
    op, b = D.assemble(spec, dev(psi))
    bare = D.problem_operator(spec)
    b_mf = D.rhs_mf(spec, dev(psi))
    assert torch.allclose(b_mf, b, rtol=0, atol=1e-15 * float(b.abs().max()))
    fn = getattr(D, solver)
    # GMRES with the inexact spectral preconditioner (its iterates agree to
    # rounding); BiCGSTAB with the exact line preconditioner (its residual
    # history is too irregular for an iteration count to carry over)
    if solver == "gmres":
        kw = dict(max_it=300, rtol=1e-10, pc="spectral", vbar=1.25, restart=30)
    else:
        kw = dict(max_it=20, rtol=1e-10, pc="line")
    x1, i1 = fn(op, b, **kw)
    x2, i2 = fn(bare, b_mf, matrix_free=True, **kw)
    assert i1["converged"] and i2["converged"]
    assert abs(i1["iters"] - i2["iters"]) <= (1 if solver == "gmres" else 0), (i1, i2)
    A = O.Matrix(oprob(spec))
    x_ref = np.linalg.solve(A.dense(), A.rhs(psi))
    for xx in (x1, x2):
        assert np.linalg.norm(host(xx) - x_ref) <= 1e-8 * np.linalg.norm(x_ref)


def test_matrix_free_fp32_refinement(D):
    """FP32-IR GMRES with the matrix-free operator in both precisions."""
    spec = IN.Spec(d=2, n=[8, 16, 12], vkind=2, v0=2.0, x0=0.5, lw=0.05)
    psi = IN.gaussian_packet(spec, [0.3, 0.5], [5.0, 2.0], 0.15, IN.positive_energy_spinor([5.0, 2.0], spec.m, 2))
    bare = D.problem_operator(spec)
    b = D.rhs_mf(spec, dev(psi))
    x, info = D.gmres(bare, b, restart=30, max_it=400, rtol=1e-10, pc="line", precision=32, inner_rtol=1e-5,
                      matrix_free=True)
    assert info["converged"], info
    A = O.Matrix(oprob(spec))
    x_ref = np.linalg.solve(A.dense(), A.rhs(psi))
    assert np.linalg.norm(host(x) - x_ref) <= 1e-8 * np.linalg.norm(x_ref)


def test_matrix_free_rejections(D):
    spec = IN.Spec(d=2, n=[4, 5, 6])
    bare = D.problem_operator(spec)
    b = torch.ones(bare.n, dtype=torch.complex128, device="cuda")
    with pytest.raises(D.DiracError):  # stored blocks requested, none given
        D.gmres(bare, b, max_it=3, pc="spectral")
    bad = IN.Spec(d=2, n=[4, 2, 6])  # periodic axis below 3 nodes
    with pytest.raises(D.DiracError):
        D.spmv_mf(bad, torch.ones(4 * 12 * 2, dtype=torch.complex128, device="cuda"))
