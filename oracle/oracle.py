"""CPU FP64 oracle for the spacetime finite-element Dirac solve (arXiv:2103.14588).

TEST INFRASTRUCTURE ONLY: imported by the tests, by the smoke check and by the
CPU-baseline leg of the benchmark, never by the product library.  It shares no
code with the HIP path; the two meet only through seeded input arrays.

The heavy pieces (element-by-element assembly, block products, the spectral
exact solve, restarted GMRES) live in ``dirac_oracle.c`` and are reached
through ctypes.  This module adds the closed-form physics used to pin them:

* the positive-energy plane wave of App. B (eigenvector of H = alpha p + beta m);
* the charge integral per time slice (the "energy" monitor of Sec. 4.1);
* dense LU on tiny meshes.

Function-level citations name sections and equations of the paper.
"""
from __future__ import annotations

import ctypes as C
import os
import subprocess
import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_SRC = os.path.join(_HERE, "dirac_oracle.c")
_LIB = os.path.join(_HERE, "liboracle.so")


def build(force: bool = False) -> str:
    """Compile the C oracle with gcc (plain -O2, OpenMP)."""
    if force or not os.path.exists(_LIB) or os.path.getmtime(_LIB) < os.path.getmtime(_SRC):
        tmp = _LIB + ".tmp%d" % os.getpid()
        subprocess.check_call(["gcc", "-O2", "-std=gnu11", "-fopenmp", "-fPIC", "-shared",
                               _SRC, "-o", tmp, "-lm"])
        os.replace(tmp, _LIB)
    return _LIB


class Problem(C.Structure):
    """Mesh, mass and potential.  n[0] = time elements, n[1..d] spatial elements
    (periodic).  vkind 0: V = 0; 1: V = v0 for x > x0 (Sec. 4.3 step);
    2: V = v0/2 (1 + tanh((x - x0)/lw)) (Sec. 4.3 smooth step)."""
    _fields_ = [("d", C.c_int32), ("nc", C.c_int32), ("n", C.c_int32 * 4), ("len", C.c_double * 4),
                ("m", C.c_double), ("vkind", C.c_int32), ("v0", C.c_double), ("x0", C.c_double),
                ("lw", C.c_double)]


def problem(d, n, lens=None, m=1.0, vkind=0, v0=0.0, x0=0.5, lw=1.0) -> Problem:
    """n = [n_t, n_1, ..., n_d]; lens = [T, L_1, ..., L_d] (default all 1)."""
    p = Problem()
    p.d = d
    p.nc = 4 if d == 3 else 2
    for a in range(4):
        p.n[a] = n[a] if a < len(n) else 1
        p.len[a] = (lens[a] if lens is not None else 1.0) if a < len(n) else 1.0
    p.m, p.vkind, p.v0, p.x0, p.lw = m, vkind, v0, x0, lw
    return p


class Stats(C.Structure):
    _fields_ = [("iters", C.c_int32), ("restarts", C.c_int32), ("converged", C.c_int32),
                ("breakdown", C.c_int32), ("relres", C.c_double), ("est", C.c_double)]


PCFN = C.CFUNCTYPE(None, C.c_void_p, C.c_void_p, C.c_void_p)

_lib = None


def lib():
    global _lib
    if _lib is None:
        L = C.CDLL(build())
        P = C.POINTER(Problem)
        vp, i64 = C.c_void_p, C.c_int64
        L.orc_gamma.argtypes = [C.c_int, C.c_int, vp]
        L.orc_build.argtypes = [P]
        L.orc_build.restype = vp
        L.orc_free.argtypes = [vp]
        L.orc_nnzb.argtypes = [vp]
        L.orc_nnzb.restype = i64
        L.orc_nnzb0.argtypes = [vp]
        L.orc_nnzb0.restype = i64
        L.orc_nrows.argtypes = [P]
        L.orc_nrows.restype = i64
        L.orc_spatial_nodes.argtypes = [P]
        L.orc_spatial_nodes.restype = i64
        L.orc_export.argtypes = [vp, vp, vp, vp]
        L.orc_export0.argtypes = [vp, vp, vp, vp]
        L.orc_element_matrix.argtypes = [P, vp, vp]
        L.orc_row.argtypes = [P, i64, vp, vp]
        L.orc_row.restype = C.c_int
        L.orc_spmv.argtypes = [vp, vp, vp]
        L.orc_rhs.argtypes = [vp, vp, vp]
        L.orc_block_jacobi.argtypes = [vp, vp]
        L.orc_block_jacobi.restype = i64
        L.orc_spectral_solve.argtypes = [P, C.c_double, vp, vp]
        L.orc_spectral_solve.restype = C.c_int
        L.orc_gmres.argtypes = [vp, C.c_int, C.c_double, PCFN, vp, vp, vp, C.c_int, C.c_int,
                                C.c_double, C.c_int, C.POINTER(Stats), vp]
        L.orc_gmres.restype = C.c_int
        L.orc_bicgstab.argtypes = [vp, C.c_int, C.c_double, PCFN, vp, vp, vp, C.c_int, C.c_double,
                                   C.POINTER(Stats), vp]
        L.orc_bicgstab.restype = C.c_int
        L.orc_dense.argtypes = [vp, vp]
        L.orc_dense_solve.argtypes = [i64, vp, vp]
        L.orc_dense_solve.restype = C.c_int
        L.orc_potential.argtypes = [P, C.c_double]
        L.orc_potential.restype = C.c_double
        _lib = L
    return _lib


def _ptr(a: np.ndarray):
    assert a.flags["C_CONTIGUOUS"]
    return a.ctypes.data_as(C.c_void_p)


def nrows(p: Problem) -> int:
    return int(lib().orc_nrows(C.byref(p)))


def nunknowns(p: Problem) -> int:
    """Unknowns of the reduced system D_w22 (Sec. 2.1): every node with tau >= 1,
    times the spinor components."""
    return nrows(p) * p.nc


def gamma(d: int, mu: int) -> np.ndarray:
    nc = 4 if d == 3 else 2
    g = np.zeros((nc, nc), np.complex128)
    lib().orc_gamma(d, mu, _ptr(g))
    return g


def element_matrix(p: Problem, e) -> np.ndarray:
    """Element block matrix [2^D, 2^D, nc, nc] (App. A, eq. (diracWeak1p1))."""
    D = p.d + 1
    nl = 1 << D
    B = np.zeros((nl, nl, p.nc, p.nc), np.complex128)
    ee = np.zeros(4, np.int32)
    ee[:len(e)] = e
    lib().orc_element_matrix(C.byref(p), _ptr(ee), _ptr(B))
    return B


def potential(p: Problem, x: float) -> float:
    return float(lib().orc_potential(C.byref(p), x))


class Matrix:
    """Globally assembled reduced operator A = D_w22 (block rows) plus the
    t = 0 columns D_w21 (Sec. 2.1, eq. (dirac_weakIVP); Alg. 1 steps 3-5)."""

    def __init__(self, p: Problem):
        self.p = p
        self.h = lib().orc_build(C.byref(p))
        if not self.h:
            raise ValueError("invalid problem")
        self.nrows = nrows(p)
        self.nc = p.nc
        self.N = self.nrows * self.nc

    def __del__(self):
        if getattr(self, "h", None):
            lib().orc_free(self.h)
            self.h = None

    def export(self):
        nnzb = int(lib().orc_nnzb(self.h))
        rp = np.zeros(self.nrows + 1, np.int64)
        col = np.zeros(nnzb, np.int64)
        val = np.zeros((nnzb, self.nc, self.nc), np.complex128)
        lib().orc_export(self.h, _ptr(rp), _ptr(col), _ptr(val))
        return rp, col, val

    def export0(self):
        nnzb = int(lib().orc_nnzb0(self.h))
        S = int(lib().orc_spatial_nodes(C.byref(self.p)))
        rp = np.zeros(S + 1, np.int64)
        col = np.zeros(max(nnzb, 1), np.int64)
        val = np.zeros((max(nnzb, 1), self.nc, self.nc), np.complex128)
        lib().orc_export0(self.h, _ptr(rp), _ptr(col), _ptr(val))
        return rp, col[:nnzb], val[:nnzb]

    def spmv(self, x: np.ndarray) -> np.ndarray:
        x = np.ascontiguousarray(x, np.complex128)
        y = np.empty(self.N, np.complex128)
        lib().orc_spmv(self.h, _ptr(x), _ptr(y))
        return y

    def rhs(self, psi0: np.ndarray) -> np.ndarray:
        """b = -D_w21 psi0 (Sec. 2.1, eq. (dirac_weakIVP))."""
        psi0 = np.ascontiguousarray(psi0, np.complex128)
        b = np.empty(self.N, np.complex128)
        lib().orc_rhs(self.h, _ptr(psi0), _ptr(b))
        return b

    def block_jacobi(self):
        inv = np.zeros((self.nrows, self.nc, self.nc), np.complex128)
        bad = int(lib().orc_block_jacobi(self.h, _ptr(inv)))
        return inv, bad

    def dense(self) -> np.ndarray:
        if self.N > 6000:
            raise ValueError("dense copy only for tiny meshes")
        Dm = np.zeros((self.N, self.N), np.complex128)
        lib().orc_dense(self.h, _ptr(Dm))
        return Dm

    def gmres(self, b, x0=None, restart=50, max_it=20000, rtol=1e-8, pc="bj", vbar=0.0,
              pcfn=None, flexible=False, history=False):
        """Restarted GMRES(m) with right preconditioning (Sec. 2.2; Alg. 1 step 6).
        pc: 'none' | 'bj' (node-block Jacobi) | 'spectral' (exact inverse with the
        potential replaced by the constant vbar) | 'fn' (python callable pcfn)."""
        b = np.ascontiguousarray(b, np.complex128)
        x = np.zeros(self.N, np.complex128) if x0 is None else np.array(x0, np.complex128)
        kind = {"none": 0, "bj": 1, "spectral": 2, "fn": 3}[pc]
        cb = PCFN(0)
        if kind == 3:
            N = self.N

            def _cb(pin, pout, ctx):
                vin = np.ctypeslib.as_array(C.cast(pin, C.POINTER(C.c_double)), shape=(2 * N,))
                vout = np.ctypeslib.as_array(C.cast(pout, C.POINTER(C.c_double)), shape=(2 * N,))
                z = pcfn(vin.view(np.complex128).copy())
                vout[:] = np.ascontiguousarray(z, np.complex128).view(np.float64)
            cb = PCFN(_cb)
        st = Stats()
        hist = np.zeros(max(max_it, 1), np.float64)
        rc = lib().orc_gmres(self.h, kind, vbar, cb, None, _ptr(b), _ptr(x), restart, max_it, rtol,
                             1 if flexible else 0, C.byref(st), _ptr(hist))
        info = dict(rc=rc, iters=st.iters, restarts=st.restarts, converged=bool(st.converged),
                    breakdown=bool(st.breakdown), relres=st.relres, est=st.est)
        if history:
            info["history"] = hist[:st.iters].copy()
        return x, info


def _pc_callback(N, pc, pcfn):
    kind = {"none": 0, "bj": 1, "spectral": 2, "fn": 3}[pc]
    cb = PCFN(0)
    if kind == 3:
        def _cb(pin, pout, ctx):
            vin = np.ctypeslib.as_array(C.cast(pin, C.POINTER(C.c_double)), shape=(2 * N,))
            vout = np.ctypeslib.as_array(C.cast(pout, C.POINTER(C.c_double)), shape=(2 * N,))
            z = pcfn(vin.view(np.complex128).copy())
            vout[:] = np.ascontiguousarray(z, np.complex128).view(np.float64)
        cb = PCFN(_cb)
    return kind, cb


def bicgstab(A: "Matrix", b, x0=None, max_it=20000, rtol=1e-8, pc="bj", vbar=0.0, pcfn=None, history=False):
    """BiCGSTAB with right preconditioning (the paper's second solver, Sec. 4.4;
    van der Vorst 1992), restarting from the true residual when the updated one
    has drifted.  pc as for Matrix.gmres."""
    b = np.ascontiguousarray(b, np.complex128)
    x = np.zeros(A.N, np.complex128) if x0 is None else np.array(x0, np.complex128)
    kind, cb = _pc_callback(A.N, pc, pcfn)
    st = Stats()
    hist = np.zeros(max(max_it, 1), np.float64)
    rc = lib().orc_bicgstab(A.h, kind, vbar, cb, None, _ptr(b), _ptr(x), max_it, rtol, C.byref(st), _ptr(hist))
    info = dict(rc=rc, iters=st.iters, restarts=st.restarts, converged=bool(st.converged),
                breakdown=bool(st.breakdown), relres=st.relres, est=st.est)
    if history:
        info["history"] = hist[:st.iters].copy()
    return x, info


def row(p: Problem, r: int):
    """Block row r computed alone from the elements that contain its node.
    Returns (cols, blocks); t = 0 columns are encoded as -(spatial index) - 1."""
    D = p.d + 1
    cap = 3 ** D
    cols = np.zeros(cap, np.int64)
    blocks = np.zeros((cap, p.nc, p.nc), np.complex128)
    k = lib().orc_row(C.byref(p), int(r), _ptr(cols), _ptr(blocks))
    if k < 0:
        raise ValueError("invalid problem")
    return cols[:k].copy(), blocks[:k].copy()


def spectral_solve(p: Problem, vbar: float, v: np.ndarray) -> np.ndarray:
    """Exact solve with the constant-potential operator A(vbar) on the periodic
    mesh (spatial DFT + block elimination along time per mode)."""
    v = np.ascontiguousarray(v, np.complex128)
    out = np.empty_like(v)
    rc = lib().orc_spectral_solve(C.byref(p), float(vbar), _ptr(v), _ptr(out))
    if rc != 0:
        raise FloatingPointError("singular pivot in spectral solve")
    return out


def time_slab_problem(p: Problem, slabs: int) -> Problem:
    """The problem of one time slab: n_t / slabs time elements of the same
    length h_t, the same spatial mesh and potential.  Every potential of the
    method depends on x only (Sec. 4.3), so all slabs share this operator."""
    nt = p.n[0]
    if slabs < 1 or nt % slabs:
        raise ValueError("slabs must divide n_t")
    L = nt // slabs
    q = Problem()
    C.memmove(C.byref(q), C.byref(p), C.sizeof(Problem))
    q.n[0] = L
    q.len[0] = p.len[0] * L / nt
    return q


def time_slab_solve(p: Problem, v: np.ndarray, slabs: int) -> np.ndarray:
    """Time decomposition (the preconditioner direction named in the
    concluding section: time-additive Schwarz), non-overlapping: the time
    interval is cut into `slabs` equal slabs and on each one the Galerkin
    problem of Sec. 2.1 posed on the slab's own interval is solved exactly,
    z_k = A_slab^{-1} v_k.  Posing it on the slab's interval means: the slab's
    first row takes the field before the slab as known data (dropped here, as
    in the preconditioner's zero initial state) and its last row ends like the
    last row of the whole interval.  Exact solve: the spectral solve for a
    constant potential, dense LU otherwise (tiny meshes)."""
    q = time_slab_problem(p, slabs)
    v = np.ascontiguousarray(v, np.complex128)
    n = v.size // slabs
    out = np.empty_like(v)
    As = None
    if p.vkind != 0:
        As = Matrix(q).dense()
    for k in range(slabs):
        vk = v[k * n:(k + 1) * n]
        if As is None:
            out[k * n:(k + 1) * n] = spectral_solve(q, 0.0, vk)
        else:
            out[k * n:(k + 1) * n] = dense_solve(As, vk)
    return out


def dense_solve(Adense: np.ndarray, b: np.ndarray) -> np.ndarray:
    """Dense LU with partial pivoting (own code, in the C oracle)."""
    a = np.array(Adense, np.complex128, order="C")
    x = np.array(b, np.complex128)
    if lib().orc_dense_solve(a.shape[0], _ptr(a), _ptr(x)) != 0:
        raise FloatingPointError("singular")
    return x


# ---------------------------------------------------------------- physics
def plane_wave_spinor(k: float, m: float = 1.0) -> np.ndarray:
    """u_+(k) of App. B: positive-energy eigenvector of H = sigma_1 k + sigma_3 m,
    the 1+1 Hamiltonian that follows from the App. A gamma pair."""
    E = np.sqrt(k * k + m * m)
    return np.array([np.sqrt(1 + m / E), np.sign(k) * np.sqrt(1 - m / E)], np.complex128) / np.sqrt(2)


def plane_wave_solution(p: Problem, k: float) -> np.ndarray:
    """Closed-form 1+1 plane wave u_+ exp(i(kx - Et)) at every unknown node
    (tau = 1..n_t), laid out like the solution vector."""
    assert p.d == 1
    m = p.m
    E = np.sqrt(k * k + m * m)
    u = plane_wave_spinor(k, m)
    nt, nx = p.n[0], p.n[1]
    t = (np.arange(1, nt + 1) * p.len[0] / nt)[:, None]
    x = (np.arange(nx) * p.len[1] / nx)[None, :]
    ph = np.exp(1j * (k * x - E * t))
    return (ph[..., None] * u).reshape(-1)


def charge(p: Problem, psi0: np.ndarray, x: np.ndarray) -> np.ndarray:
    """Integral of psi^dagger psi over space at every time node tau = 0..n_t
    (the conserved quantity monitored in Sec. 4.1).  On a periodic uniform
    mesh the trapezoid rule is the nodal sum times the cell volume."""
    S = int(np.prod([p.n[a] for a in range(1, p.d + 1)]))
    vol = float(np.prod([p.len[a] / p.n[a] for a in range(1, p.d + 1)]))
    allv = np.concatenate([psi0, x]).reshape(p.n[0] + 1, S, p.nc)
    return vol * np.sum(np.abs(allv) ** 2, axis=(1, 2))


def slice_moments(p: Problem, psi0: np.ndarray, x: np.ndarray, x_split: float) -> np.ndarray:
    """Per time node tau = 0..n_t, trapezoid sums over space (on the periodic
    uniform mesh: nodal sums times the cell volume) of
      [ |psi|^2,  |psi|^2 where x_1 > x_split,  x_1 |psi|^2, ..., x_d |psi|^2 ]
    with node coordinates x_a = i_a h_a.  Column 0 is the charge of Sec. 4.1,
    columns 2.. the numerators of <x(t)> (Sec. 4.2), columns 1 and 0 - 1 the
    numerators of T and R (Sec. 4.3, eq. (klein:coeffs)).  Shape [n_t + 1, 2 + d]."""
    d = p.d
    ns = [p.n[a] for a in range(1, d + 1)]
    S = int(np.prod(ns))
    vol = float(np.prod([p.len[a] / p.n[a] for a in range(1, d + 1)]))
    allv = np.concatenate([psi0, x]).reshape(p.n[0] + 1, S, p.nc)
    dens = np.sum(np.abs(allv) ** 2, axis=2)  # [tau][s]
    idx = np.arange(S)
    coords = []
    for a in range(d):
        coords.append((idx % ns[a]) * (p.len[a + 1] / ns[a]))
        idx = idx // ns[a]
    out = np.empty((p.n[0] + 1, 2 + d))
    out[:, 0] = vol * dens.sum(1)
    out[:, 1] = vol * dens[:, coords[0] > x_split].sum(1)
    for a in range(d):
        out[:, 2 + a] = vol * (dens * coords[a][None, :]).sum(1)
    return out


def free_evolution_1p1(p: Problem, psi0: np.ndarray, t: float) -> np.ndarray:
    """Exact 1+1 free Dirac evolution on the periodic interval (H = sigma_1 k +
    sigma_3 m, the Hamiltonian of the App. A gamma pair, App. B) of the
    trigonometric interpolant of the nodal psi0: every Fourier mode k moves by
    exp(-i H(k) t) = cos(E t) - i sin(E t) H(k) / E, E = sqrt(k^2 + m^2).  The
    reference for the Zitterbewegung of Sec. 4.2.  Returns nodal values [n_1][2]."""
    assert p.d == 1 and p.vkind == 0
    nx, L, m = p.n[1], p.len[1], p.m
    u = np.asarray(psi0, np.complex128).reshape(nx, 2)
    k = 2 * np.pi * np.fft.fftfreq(nx, d=L / nx)
    a, b = np.fft.fft(u[:, 0]), np.fft.fft(u[:, 1])
    E = np.sqrt(k * k + m * m)
    c, s = np.cos(E * t), np.sin(E * t) / E
    na = c * a - 1j * s * (m * a + k * b)
    nb = c * b - 1j * s * (k * a - m * b)
    return np.stack([np.fft.ifft(na), np.fft.ifft(nb)], 1)
