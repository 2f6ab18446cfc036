"""Seeded synthetic inputs: problem descriptors and initial data at t = 0.

This module holds no arithmetic of the solver.  It only describes the meshes
and draws the initial spinor fields that both the product path and the oracle
receive as plain arrays.  The workloads follow the shapes of the paper's test
cases (Sec. 4): plane waves and Gaussian packets on a periodic box, step
potentials for the Klein setting.  Random draws use numpy's PCG64
(``numpy.random.default_rng(seed)``).

Layout of every field: [spatial node][component], spatial index with axis 1
fastest, complex128.
"""
from __future__ import annotations

from dataclasses import dataclass, field
import numpy as np


@dataclass
class Spec:
    """Mesh + physics of one system.  n = [n_t, n_1, .., n_d] elements,
    lens = [T, L_1, .., L_d]; space periodic.  vkind: 0 none, 1 step V0 for
    x_1 > x0, 2 smooth step V0/2 (1 + tanh((x_1 - x0)/lw))."""
    d: int
    n: list
    lens: list = None
    m: float = 1.0
    vkind: int = 0
    v0: float = 0.0
    x0: float = 0.5
    lw: float = 1.0

    def __post_init__(self):
        if self.lens is None:
            self.lens = [1.0] * (self.d + 1)

    @property
    def nc(self):
        return 4 if self.d == 3 else 2

    @property
    def spatial(self):
        return int(np.prod(self.n[1:self.d + 1]))

    @property
    def nrows(self):
        return self.n[0] * self.spatial

    @property
    def nunknowns(self):
        return self.nrows * self.nc


def grid(spec: Spec):
    """Node coordinates of the t = 0 slice, one array per spatial axis, each of
    shape [n_d, .., n_1] (axis 1 last / fastest)."""
    axes = [np.arange(spec.n[a]) * spec.lens[a] / spec.n[a] for a in range(1, spec.d + 1)]
    mesh = np.meshgrid(*axes[::-1], indexing="ij")
    return mesh[::-1]


def positive_energy_spinor(p, m=1.0, nc=2):
    """Unit positive-energy spinor for momentum p.  For two components,
    (E + m, p_x + i p_y)/norm is the eigenvector of sigma_1 p_x + sigma_2 p_y +
    sigma_3 m with eigenvalue +E; four components use the Dirac-representation
    form (chi, sigma.p chi/(E + m)) with chi = (1, 0)."""
    p = np.asarray(p, float)
    E = np.sqrt(np.dot(p, p) + m * m)
    if nc == 2:
        px = p[0]
        py = p[1] if len(p) > 1 else 0.0
        u = np.array([E + m, px + 1j * py], np.complex128)
    else:
        px, py, pz = (list(p) + [0.0, 0.0])[:3]
        u = np.array([E + m, 0, pz, px + 1j * py], np.complex128)
    return u / np.linalg.norm(u)


def plane_wave(spec: Spec, k: float):
    """psi0 = u_+(k) exp(i k x) along axis 1 (the closed-form check case)."""
    x = grid(spec)[0]
    u = positive_energy_spinor([k] + [0.0] * (spec.d - 1), spec.m, spec.nc)
    return (np.exp(1j * k * x).reshape(-1)[:, None] * u[None, :]).reshape(-1)


def gaussian_packet(spec: Spec, center, p, sigma, spinor):
    """psi0 = (2 pi sigma^2)^(-d/4) exp(-|x - c|^2 / (4 sigma^2) + i p.x) s with the
    minimum-image distance on the periodic box."""
    X = grid(spec)
    env = np.zeros(X[0].shape)
    phase = np.zeros(X[0].shape)
    for a in range(spec.d):
        L = spec.lens[a + 1]
        dx = (X[a] - center[a] + 0.5 * L) % L - 0.5 * L
        env += dx * dx
        phase += p[a] * X[a]
    amp = (2 * np.pi * sigma * sigma) ** (-spec.d / 4.0) * np.exp(-env / (4 * sigma * sigma) + 1j * phase)
    s = np.asarray(spinor, np.complex128)
    return (amp.reshape(-1)[:, None] * s[None, :]).reshape(-1)


# ------------------------------------------------------------ workloads
@dataclass
class Workload:
    name: str
    spec: Spec
    psi0: np.ndarray
    restart: int
    rtol: float
    meta: dict = field(default_factory=dict)


def plane_wave_1p1(n=64, k=2 * np.pi):
    """1+1 plane wave on [0,1] x [0,1], m = 1, n x n elements."""
    spec = Spec(d=1, n=[n, n])
    return Workload("1+1D plane wave %dx%d" % (n, n), spec, plane_wave(spec, k), 30, 1e-10, {"k": k})


def packet_2p1(n=128, seed=0, nt=None, sigma=0.05):
    """2+1 Gaussian packet mixing positive and negative energies, spinor
    (1, 1)/sqrt(2); centre ~ U[0.3, 0.7]^2, |p| ~ U[5, 20], direction ~ U[0, 2 pi)."""
    rng = np.random.default_rng(seed)
    c = rng.uniform(0.3, 0.7, 2)
    pm = rng.uniform(5, 20)
    ang = rng.uniform(0, 2 * np.pi)
    p = [pm * np.cos(ang), pm * np.sin(ang)]
    spec = Spec(d=2, n=[nt or n, n, n])
    psi0 = gaussian_packet(spec, c, p, sigma, np.array([1, 1]) / np.sqrt(2))
    return Workload("2+1D packet %dx%dx%d" % (nt or n, n, n), spec, psi0, 50, 1e-8,
                    {"center": c.tolist(), "p": p, "seed": seed})


def packet_3p1(n=32, seed=0, sigma=0.05):
    """3+1 Gaussian packet, spinor (1, 0, 1, 0)/sqrt(2), direction uniform on S^2."""
    rng = np.random.default_rng(seed)
    c = rng.uniform(0.3, 0.7, 3)
    pm = rng.uniform(5, 20)
    v = rng.standard_normal(3)
    p = (pm * v / np.linalg.norm(v)).tolist()
    spec = Spec(d=3, n=[n, n, n, n])
    psi0 = gaussian_packet(spec, c, p, sigma, np.array([1, 0, 1, 0]) / np.sqrt(2))
    return Workload("3+1D packet %d^4" % n, spec, psi0, 50, 1e-8,
                    {"center": c.tolist(), "p": p, "seed": seed})


def klein_step_2p1(n=128, v0=2.5, seed=0, nt=None, sigma=0.05):
    """2+1 packet incident on the step V = v0 for x > 0.5: centre x ~ U[0.15, 0.35],
    y ~ U[0.3, 0.7]; |p| ~ U[5, 20] within 30 degrees of +x; positive-energy spinor."""
    rng = np.random.default_rng(seed)
    c = [rng.uniform(0.15, 0.35), rng.uniform(0.3, 0.7)]
    pm = rng.uniform(5, 20)
    ang = rng.uniform(-np.pi / 6, np.pi / 6)
    p = [pm * np.cos(ang), pm * np.sin(ang)]
    spec = Spec(d=2, n=[nt or n, n, n], vkind=1, v0=v0, x0=0.5)
    psi0 = gaussian_packet(spec, c, p, sigma, positive_energy_spinor(p, spec.m, 2))
    return Workload("2+1D Klein step %dx%dx%d V0=%.3g" % (nt or n, n, n, v0), spec, psi0, 50, 1e-8,
                    {"center": c, "p": p, "seed": seed, "v0": v0})


def klein_batch(count=64, seed=0, nmin=32, nmax=96):
    """Batch of Klein-step systems on uneven cubic meshes n^3, n ~ U{nmin..nmax},
    V0 ~ U[0, 3m]; per-system sub-seeds drawn from the batch seed."""
    rng = np.random.default_rng(seed)
    ns = rng.integers(nmin, nmax + 1, count)
    v0s = rng.uniform(0.0, 3.0, count)
    subs = rng.integers(0, 2 ** 31 - 1, count)
    return [klein_step_2p1(int(n), float(v), int(s)) for n, v, s in zip(ns, v0s, subs)]
