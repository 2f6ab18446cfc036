"""GPU parity: the HIP path against the CPU oracle, element by element.

Sizes span several workgroup tiles with ragged tails; the full-size checks
sample single rows the oracle computes on its own.  Tolerances:
assembly 1e-14 relative (pattern bit-exact), SpMV complex128 1e-13 normwise,
complex64 2e-6 against FP64 of the rounded inputs, solutions 1e-8 relative.
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
    IN.Spec(d=1, n=[2, 3]),
    IN.Spec(d=2, n=[6, 17, 9], lens=[1.0, 0.9, 1.1], m=0.7),
    IN.Spec(d=2, n=[5, 12, 11], vkind=1, v0=2.5, x0=0.5),
    IN.Spec(d=2, n=[4, 9, 10], vkind=2, v0=1.5, x0=0.4, lw=0.05),
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


def rand_c(n, seed, dtype=np.complex128):
    rng = np.random.default_rng(seed)
    return (rng.standard_normal(n) + 1j * rng.standard_normal(n)).astype(dtype)


def dev(a):
    return torch.from_numpy(np.ascontiguousarray(a)).cuda()


def host(t):
    torch.cuda.synchronize()
    return t.cpu().numpy()


@pytest.mark.parametrize("spec", CASES, ids=ids)
def test_assembly_matches_oracle(D, spec):
    A_or = O.Matrix(oprob(spec))
    rp, col, val = A_or.export()
    psi0 = rand_c(spec.spatial * spec.nc, 7)
    op, b = D.assemble(spec, dev(psi0))
    g_rp, g_ci = host(op.row_ptr), host(op.col_idx)
    assert np.array_equal(g_rp.astype(np.int64), rp)
    assert np.array_equal(g_ci.astype(np.int64), col)
    g_val = host(op.val64).reshape(-1, spec.nc, spec.nc)
    scale = np.abs(val).max()
    assert np.abs(g_val - val).max() <= 1e-14 * scale
    # complex64 copy is the round-to-nearest of the FP64 values
    assert np.array_equal(host(op.val32), host(op.val64).astype(np.complex64))
    # right-hand side b = -D_w21 psi0
    b_or = A_or.rhs(psi0)
    assert np.abs(host(b) - b_or).max() <= 1e-14 * max(np.abs(b_or).max(), 1e-300) * 10
    # node-block Jacobi inverses
    inv_or, bad = A_or.block_jacobi()
    assert op.bsr.singular_blocks == bad
    g_inv = host(op.bjinv64).reshape(-1, spec.nc, spec.nc)
    assert np.abs(g_inv - inv_or).max() <= 1e-12 * np.abs(inv_or).max()


def test_singular_block_guard(D):
    """V = m on every element makes the interior diagonal blocks singular; they
    are replaced by the identity and counted, as in the oracle."""
    spec = IN.Spec(d=2, n=[4, 5, 5], vkind=1, v0=1.0, x0=-1.0)
    op, _ = D.assemble(spec, None)
    inv_or, bad = O.Matrix(oprob(spec)).block_jacobi()
    assert bad == 3 * 25 and op.bsr.singular_blocks == bad
    assert np.allclose(host(op.bjinv64).reshape(-1, 2, 2), inv_or, atol=1e-12)


@pytest.mark.parametrize("spec", CASES, ids=ids)
def test_spmv_matches_oracle(D, spec):
    A_or = O.Matrix(oprob(spec))
    op, _ = D.assemble(spec, None)
    x = rand_c(A_or.N, 11)
    y_or = A_or.spmv(x)
    y = host(D.spmv(op, dev(x)))
    assert np.linalg.norm(y - y_or) <= 1e-13 * np.linalg.norm(y_or)
    # complex64: compare with FP64 arithmetic on the rounded inputs
    x32 = x.astype(np.complex64)
    rp, col, val = A_or.export()
    v32 = val.astype(np.complex64).astype(np.complex128)
    y_ref = np.zeros(A_or.N, np.complex128)
    nc = spec.nc
    xr = x32.astype(np.complex128).reshape(-1, nc)
    for r in range(A_or.nrows):
        s = slice(rp[r], rp[r + 1])
        y_ref[r * nc:(r + 1) * nc] = np.einsum("kij,kj->i", v32[s], xr[col[s]])
    y32 = host(D.spmv(op, dev(x32)))
    assert np.linalg.norm(y32 - y_ref) <= 2e-6 * np.linalg.norm(y_ref)


@pytest.mark.parametrize("spec,vbar", [
    (IN.Spec(d=1, n=[9, 10]), 0.0),
    (IN.Spec(d=2, n=[7, 12, 9], lens=[1.0, 0.8, 1.2]), 0.0),
    (IN.Spec(d=2, n=[6, 10, 8], vkind=1, v0=2.5, x0=0.5), 1.25),
    (IN.Spec(d=3, n=[5, 4, 6, 3]), 0.0),
], ids=lambda v: ids(v) if hasattr(v, "d") else str(v))
def test_preconditioners_match_oracle(D, spec, vbar):
    p = oprob(spec)
    A_or = O.Matrix(p)
    op, _ = D.assemble(spec, None)
    v = rand_c(A_or.N, 5)
    z_or = O.spectral_solve(p, vbar, v)
    z = host(D.pc_apply(op, dev(v), "spectral", vbar))
    assert np.linalg.norm(z - z_or) <= 1e-11 * np.linalg.norm(z_or)
    z32 = host(D.pc_apply(op, dev(v.astype(np.complex64)), "spectral", vbar))
    assert np.linalg.norm(z32 - z_or) <= 2e-3 * np.linalg.norm(z_or)
    inv_or, _ = A_or.block_jacobi()
    zb_or = np.einsum("rij,rj->ri", inv_or, v.reshape(-1, spec.nc)).reshape(-1)
    zb = host(D.pc_apply(op, dev(v), "bj"))
    assert np.linalg.norm(zb - zb_or) <= 1e-13 * np.linalg.norm(zb_or)


@pytest.mark.parametrize("spec", [
    IN.Spec(d=2, n=[6, 11, 9], vkind=1, v0=2.0, x0=0.5),
    # 6992 unknowns: several 1024-element blocks of the small-basis passes
    # and a ragged last block
    IN.Spec(d=2, n=[8, 23, 19], vkind=1, v0=2.0, x0=0.5),
], ids=ids)
def test_gmres_fp64_matches_oracle_iteration_by_iteration(D, spec):
    """Same algorithm (GMRES(m), CGS2, complex Givens, right node-block Jacobi):
    the residual history agrees step by step and the iterate after a fixed
    number of steps matches."""
    A_or = O.Matrix(oprob(spec))
    psi0 = IN.gaussian_packet(spec, [0.3, 0.5], [6.0, 2.0], 0.15, np.array([1, 1]) / np.sqrt(2))
    b_or = A_or.rhs(psi0)
    x_or, info_or = A_or.gmres(b_or, restart=12, max_it=60, rtol=1e-14, pc="bj", history=True)
    op, b = D.assemble(spec, dev(psi0))
    x, info = D.gmres(op, b, restart=12, max_it=60, rtol=1e-14, pc="bj", history=60)
    assert info["iters"] == info_or["iters"] == 60
    h, h_or = np.array(info["history"]), info_or["history"]
    assert np.all(np.abs(h - h_or) <= 1e-9 * h_or[0] + 1e-6 * h_or)
    xg = host(x)
    assert np.linalg.norm(xg - x_or) <= 1e-8 * np.linalg.norm(x_or)
    assert abs(info["relres"] - info_or["relres"]) <= 1e-6 * info_or["relres"]


@pytest.mark.parametrize("precision", [64, 32])
@pytest.mark.parametrize("spec", [
    IN.Spec(d=2, n=[8, 12, 12], vkind=1, v0=2.5, x0=0.5),
    IN.Spec(d=1, n=[16, 24]),
    IN.Spec(d=3, n=[4, 5, 4, 4], vkind=1, v0=1.5, x0=0.5),
], ids=ids)
def test_gmres_solution_matches_exact(D, spec, precision):
    """Converged solves (spectral preconditioner, restart 20) land within 1e-8 of
    the exact discrete solution (dense LU / exact spectral solve in the oracle)."""
    p = oprob(spec)
    A_or = O.Matrix(p)
    rng = np.random.default_rng(2)
    c = rng.uniform(0.3, 0.7, spec.d)
    psi0 = IN.gaussian_packet(spec, c, [4.0] * spec.d, 0.2, np.ones(spec.nc) / np.sqrt(spec.nc))
    b_or = A_or.rhs(psi0)
    vbar = 0.5 * spec.v0 if spec.vkind else 0.0
    if A_or.N <= 4000:
        x_ref = np.linalg.solve(A_or.dense(), b_or)
    else:
        x_ref, inf = A_or.gmres(b_or, restart=40, max_it=4000, rtol=1e-13, pc="spectral", vbar=vbar)
        assert inf["converged"]
    op, b = D.assemble(spec, dev(psi0))
    x, info = D.gmres(op, b, restart=20, max_it=2000, rtol=1e-11, pc="spectral", vbar=vbar,
                      precision=precision, inner_rtol=1e-4 if precision == 32 else 0.0)
    assert info["converged"], info
    xg = host(x)
    assert np.linalg.norm(xg - x_ref) <= 1e-8 * np.linalg.norm(x_ref)
    assert info["relres"] <= 1e-11


@pytest.mark.parametrize("spec", [
    IN.Spec(d=2, n=[6, 17, 9], lens=[1.0, 0.9, 1.1], vkind=1, v0=2.5, x0=0.5),
    IN.Spec(d=1, n=[7, 37], lens=[0.8, 1.3]),
    IN.Spec(d=3, n=[3, 4, 5, 3], vkind=1, v0=1.0, x0=0.4),
], ids=ids)
def test_complex128_only_assembly(D, spec):
    """Assembly without the complex64 copy and the node-block inverses (all a
    complex128 solve with the spectral or line preconditioner reads): the same
    pattern, complex128 blocks and right-hand side as the full assembly, bit
    for bit, also when assembled again into the same arrays; the complex128
    spectral solve on it lands on the exact discrete solution; a complex64
    solve and node-block Jacobi are refused on it."""
    psi0 = rand_c(spec.spatial * spec.nc, 5)
    full, b_full = D.assemble(spec, dev(psi0))
    lean, b = D.assemble(spec, dev(psi0), fp32=False, block_jacobi=False)
    assert lean.val32 is None and lean.bjinv64 is None and lean.bjinv32 is None
    for _ in range(2):
        assert torch.equal(lean.row_ptr, full.row_ptr) and torch.equal(lean.col_idx, full.col_idx)
        assert torch.equal(lean.val64, full.val64) and torch.equal(b, b_full)
        D.assemble_into(lean, dev(psi0), b)
    A_or = O.Matrix(oprob(spec))
    x_ref = np.linalg.solve(A_or.dense(), A_or.rhs(psi0))
    vbar = 0.5 * spec.v0 if spec.vkind else 0.0
    x, info = D.gmres(lean, b, restart=20, max_it=2000, rtol=1e-11, pc="spectral", vbar=vbar)
    assert info["converged"], info
    assert np.linalg.norm(host(x) - x_ref) <= 1e-8 * np.linalg.norm(x_ref)
    with pytest.raises(D.DiracError):
        D.gmres(lean, b, restart=5, max_it=5, pc="spectral", precision=32, inner_rtol=1e-4)
    with pytest.raises(D.DiracError):
        D.gmres(lean, b, restart=5, max_it=5, pc="bj")


def test_gmres_pc_none_and_restart_one(D):
    spec = IN.Spec(d=1, n=[3, 4])
    A_or = O.Matrix(oprob(spec))
    b_or = A_or.rhs(IN.plane_wave(spec, 2 * np.pi))
    x_ref = np.linalg.solve(A_or.dense(), b_or)
    op, b = D.assemble(spec, dev(IN.plane_wave(spec, 2 * np.pi)))
    x, info = D.gmres(op, b, restart=24, max_it=24, rtol=1e-12, pc="none")
    assert info["converged"] and np.linalg.norm(host(x) - x_ref) <= 1e-9 * np.linalg.norm(x_ref)
    x1, info1 = D.gmres(op, b, restart=1, max_it=5, rtol=1e-12, pc="bj")
    assert info1["iters"] == 5 and info1["cycles"] == 5 and not info1["converged"]
    x1o, i1o = A_or.gmres(b_or, restart=1, max_it=5, rtol=1e-12, pc="bj")
    assert np.linalg.norm(host(x1) - x1o) <= 1e-10 * np.linalg.norm(x1o)


def test_gmres_edge_cases(D):
    spec = IN.Spec(d=2, n=[3, 4, 5])
    op, b = D.assemble(spec, dev(rand_c(20 * 2, 3)))
    # zero right-hand side -> x = 0, converged, no iterations
    x, info = D.gmres(op, torch.zeros_like(b), x=torch.ones_like(b), restart=5, max_it=5, pc="bj")
    assert info["converged"] and info["iters"] == 0 and np.abs(host(x)).max() == 0
    # NaN in b -> breakdown error
    bn = b.clone()
    bn[3] = complex(float("nan"), 0.0)
    with pytest.raises(D.DiracError) as e:
        D.gmres(op, bn, restart=5, max_it=5, pc="bj")
    assert e.value.code == D.EBREAKDOWN
    # workspace too small
    import ctypes as C
    o = D.make_opts(restart=5, max_it=5, pc="bj")
    small = torch.empty(4096, dtype=torch.uint8, device="cuda")
    x = torch.zeros_like(b)
    rc = D._lib.dirac_st_gmres(C.byref(op.bsr), C.c_void_p(b.data_ptr()), C.c_void_p(x.data_ptr()),
                               C.byref(o), C.c_void_p(small.data_ptr()), small.numel(), None,
                               C.c_void_p(torch.cuda.current_stream().cuda_stream))
    assert rc == D.ENOSPACE and "workspace" in D.last_error()
    # max_it reached -> NOT_CONVERGED with valid stats
    x, info = D.gmres(op, b, restart=5, max_it=3, rtol=1e-15, pc="bj")
    assert info["rc"] == D.NOT_CONVERGED and info["iters"] == 3 and np.isfinite(info["relres"])


@pytest.mark.parametrize("precision", [64, 32])
def test_gmres_nonzero_initial_guess(D, precision):
    """A nonzero initial guess: started from the solution GMRES stops before
    its first Arnoldi step with x unchanged; started from a random vector it
    lands on the same solution (the first residual is b - A x0, not b)."""
    spec = IN.Spec(d=2, n=[5, 12, 11], vkind=1, v0=2.5, x0=0.5)
    psi0 = rand_c(spec.spatial * spec.nc, 9)
    op, b = D.assemble(spec, dev(psi0))
    A_or = O.Matrix(oprob(spec))
    x_ref = np.linalg.solve(A_or.dense(), A_or.rhs(psi0))
    kw = dict(restart=20, max_it=400, rtol=1e-10, pc="spectral", vbar=1.25, precision=precision,
              inner_rtol=1e-4 if precision == 32 else 0.0)
    x0 = dev(x_ref.copy())
    x, info = D.gmres(op, b, x=x0.clone(), **kw)
    assert info["converged"] and info["iters"] == 0, info
    assert torch.equal(x, x0)
    x, info = D.gmres(op, b, x=dev(rand_c(op.n, 10)), **kw)
    assert info["converged"], info
    assert np.linalg.norm(host(x) - x_ref) <= 1e-8 * np.linalg.norm(x_ref)


# ---------------------------------------------------- full-size, sampled
@pytest.mark.parametrize("wl", ["2p1_128", "3p1_32"])
def test_full_size_sampled_rows(D, wl):
    """Full 2+1D 128^3 and 3+1D 32^4 operators: sampled block rows and sampled
    SpMV outputs against rows the oracle computes one by one."""
    spec = IN.packet_2p1().spec if wl == "2p1_128" else IN.packet_3p1().spec
    p = oprob(spec)
    op, _ = D.assemble(spec, None, fp32=True, block_jacobi=False)
    nc = spec.nc
    rng = np.random.default_rng(0)
    S = spec.spatial
    rows = np.concatenate([rng.integers(0, op.nrows, 40), [0, S - 1, S, op.nrows - S, op.nrows - 1]])
    x = torch.randn(op.n, dtype=torch.complex128, device="cuda")
    y = D.spmv(op, x)
    x32 = x.to(torch.complex64)
    y32 = D.spmv(op, x32)
    rp = op.row_ptr.cpu().numpy()
    for r in rows:
        cols, blocks = O.row(p, int(r))
        keep = cols >= 0
        cols, blocks = cols[keep], blocks[keep]
        a, e = int(rp[r]), int(rp[r + 1])
        assert np.array_equal(op.col_idx[a:e].cpu().numpy(), cols)
        gv = op.val64[a * nc * nc:e * nc * nc].cpu().numpy().reshape(-1, nc, nc)
        assert np.abs(gv - blocks).max() <= 1e-14 * np.abs(blocks).max()
        xs = x.view(-1, nc)[torch.from_numpy(cols).cuda()].cpu().numpy()
        want = np.einsum("kij,kj->i", blocks, xs)
        got = y[r * nc:(r + 1) * nc].cpu().numpy()
        assert np.abs(got - want).max() <= 1e-13 * np.abs(blocks).max() * np.abs(xs).max() * len(cols)
        xs32 = x32.view(-1, nc)[torch.from_numpy(cols).cuda()].cpu().numpy().astype(np.complex128)
        want32 = np.einsum("kij,kj->i", blocks.astype(np.complex64).astype(np.complex128), xs32)
        got32 = y32[r * nc:(r + 1) * nc].cpu().numpy()
        assert np.abs(got32 - want32).max() <= 1e-5 * np.abs(blocks).max() * np.abs(xs32).max() * len(cols)


def test_kernel_timers_count_solver_launches(D):
    """HIP-event timers inside the library: a GMRES solve from x = 0 that takes
    k Arnoldi steps records k product SpMVs and one residual SpMV per restart
    after the first; the assembly kernel is recorded once per assembly."""
    spec = IN.Spec(d=2, n=[6, 17, 9], lens=[1.0, 0.9, 1.1], m=0.7)
    psi = IN.gaussian_packet(spec, [0.4, 0.5], [3.0, 1.0], 0.2, np.ones(2) / np.sqrt(2))
    D.timing(True)
    op, b = D.assemble(spec, dev(psi))
    x, info = D.gmres(op, b, restart=5, max_it=23, rtol=1e-14, pc="bj")
    n_spmv, ms_spmv = D.timing_read("spmv64")
    n_res, _ = D.timing_read("resid64")
    n_asm, ms_asm = D.timing_read("assemble")
    D.timing(False)
    assert n_asm == 1 and ms_asm > 0.0
    assert n_spmv == info["iters"] and ms_spmv > 0.0
    assert n_res == info["cycles"]  # one residual after each cycle, none before the first
