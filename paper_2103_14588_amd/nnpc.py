"""Learned preconditioner: training pairs from the plain solver and the GPU
training loop (every arithmetic step runs in libdirac_st.so; this module
only orchestrates calls through the C ABI).

Training pairs.  For a seeded 2+1D Klein-step system A (inputs.klein_step_2p1)
a known solution x* is drawn (a sum of random spacetime wave packets) and
b = A x*.  Plain restarted GMRES is run on A x = b one cycle at a time; after
every cycle k the pair (r_k, e_k) = (b - A x_k, x* - x_k) is recorded.  The
network input is r_k and its target is the part of the error the base
preconditioner M misses, e_k - M^{-1} r_k, both scaled by sqrt(n)/||r_k|| (n
complex entries), so the learned preconditioner is
z = M^{-1} v + (||v||/sqrt(n)) N(v sqrt(n)/||v||), scale-equivariant like M.
"""
from __future__ import annotations

import math

import numpy as np
import torch

from . import dirac_st as D
from . import inputs as IN


def he_init(seed=0):
    """He-normal weights (std sqrt(2/fan_in)), zero biases, parameter layout of
    the C ABI (per layer W[27][cin][cout] then b[cout])."""
    rng = np.random.default_rng(seed)
    ch = [4, 16, 16, 16, 4]
    parts = []
    for l in range(4):
        ci, co = ch[l], ch[l + 1]
        parts.append(rng.standard_normal(27 * ci * co) * math.sqrt(2.0 / (27 * ci)))
        parts.append(np.zeros(co))
    p = np.concatenate(parts)
    assert p.size == D.NN_PARAMS
    return p


def manufactured_solution(spec, rng, npk=4):
    """x*: a sum of npk spacetime Gaussian wave packets with random centres,
    widths, frequencies and spinors, at the unknown nodes tau = 1..n_t."""
    nt, ny, nx = spec.n[0], spec.n[2], spec.n[1]
    t = (np.arange(1, nt + 1) * spec.lens[0] / nt)[:, None, None]
    y = (np.arange(ny) * spec.lens[2] / ny)[None, :, None]
    x = (np.arange(nx) * spec.lens[1] / nx)[None, None, :]
    out = np.zeros((nt, ny, nx, 2), np.complex128)
    for _ in range(npk):
        c = rng.uniform(0, 1, 3)
        sg = rng.uniform(0.08, 0.25, 3)
        k = rng.uniform(-20, 20, 3)
        dx = (x - c[0] + 0.5) % 1.0 - 0.5
        dy = (y - c[1] + 0.5) % 1.0 - 0.5
        dt = t - c[2]
        env = np.exp(-dx ** 2 / (2 * sg[0] ** 2) - dy ** 2 / (2 * sg[1] ** 2) - dt ** 2 / (2 * sg[2] ** 2))
        ph = np.exp(1j * (k[0] * x + k[1] * y + k[2] * t))
        s = rng.standard_normal(2) + 1j * rng.standard_normal(2)
        out += (env * ph)[..., None] * s
    return out.reshape(-1)


def _c64_view(v: torch.Tensor) -> torch.Tensor:
    return torch.view_as_real(v.to(torch.complex64)).reshape(-1).contiguous()


def make_pairs(n_systems=32, per_system=8, nmin=16, nmax=32, v0=2.5, base="bj", vbar=0.0,
               restart=20, seed=1):
    """List of (shape, input float32 [V*4], target float32 [V*4]) on the GPU."""
    rng = np.random.default_rng(seed)
    pairs = []
    for sidx in range(n_systems):
        n = int(rng.integers(nmin, nmax + 1))
        spec = IN.Spec(d=2, n=[n, n, n], vkind=1, v0=v0, x0=0.5)
        op, _ = D.assemble(spec, None)
        xs = torch.from_numpy(manufactured_solution(spec, rng)).cuda()
        b = D.spmv(op, xs)
        x = torch.zeros_like(b)
        shape = (n, n, n)
        work = None
        for k in range(per_system):
            x, _ = D.gmres(op, b, x=x, restart=restart, max_it=10 ** 6, max_cycles=1, rtol=1e-14,
                           pc=base if base != "none" else "none", vbar=vbar)
            r = b - D.spmv(op, x)
            e = xs - x
            if base != "none":
                mr = D.pc_apply(op, r, base, vbar, work=work)
                e = e - mr
            s = math.sqrt(r.numel()) / float(torch.linalg.vector_norm(r))
            pairs.append((shape, _c64_view(r * s), _c64_view(e * s)))
    return pairs


def make_pairs_direct(n_systems=32, per_system=8, nmin=16, nmax=32, v0_range=(2.5, 2.5), base="bj",
                      vbar=None, seed=2):
    """Pairs without a solve: a random error field e (manufactured_solution), its
    residual r = A e, target e - M^{-1} r, scaled by sqrt(n)/||r||.  vbar None
    uses V0/2 of each system for the spectral base."""
    rng = np.random.default_rng(seed)
    pairs = []
    for _ in range(n_systems):
        n = int(rng.integers(nmin, nmax + 1))
        v0 = float(rng.uniform(*v0_range))
        spec = IN.Spec(d=2, n=[n, n, n], vkind=1, v0=v0, x0=0.5)
        op, _ = D.assemble(spec, None)
        vb = 0.5 * v0 if vbar is None else vbar
        for _ in range(per_system):
            e = torch.from_numpy(manufactured_solution(spec, rng, npk=int(rng.integers(1, 6)))).cuda()
            r = D.spmv(op, e)
            if base != "none":
                e = e - D.pc_apply(op, r, base, vb)
            s = math.sqrt(r.numel()) / float(torch.linalg.vector_norm(r))
            pairs.append(((n, n, n), _c64_view(r * s), _c64_view(e * s)))
    return pairs


def normalise_targets(pairs):
    """Divide every target by the median ratio ||target|| / ||input|| so the
    network regresses O(1) values; returns (gain, pairs).  The preconditioner
    multiplies the network output by the gain (dirac_st_nn.out_gain)."""
    ratios = [float(torch.linalg.vector_norm(t) / torch.linalg.vector_norm(x)) for _, x, t in pairs]
    gain = float(np.median(ratios))
    return gain, [(s, x, (t / gain).contiguous()) for s, x, t in pairs]


def train(net: D.Net, pairs, epochs=2, lr=1e-3, seed=0, log_every=0):
    """Adam over the pairs (one pair per step, shuffled per epoch).  Returns
    the per-step losses (read back once at the end)."""
    rng = np.random.default_rng(seed)
    nsteps = epochs * len(pairs)
    losses = torch.zeros(nsteps, dtype=torch.float64, device="cuda")
    works = {}
    step = 0
    for ep in range(epochs):
        for i in rng.permutation(len(pairs)):
            shape, xin, tgt = pairs[i]
            works[shape] = D.nn_train_step(net, xin, tgt, shape, lr, loss_out=losses[step:step + 1],
                                           work=works.get(shape))
            step += 1
            if log_every and step % log_every == 0:
                print("step %d loss %.4f" % (step, float(losses[step - 1])), flush=True)
    return losses.cpu().numpy()


def eval_loss(net: D.Net, pairs):
    """Mean relative squared error of the network on pairs (no update)."""
    tot = 0.0
    for shape, xin, tgt in pairs:
        out = D.nn_forward(net, xin, shape)
        tot += float(torch.sum((out - tgt) ** 2) / torch.sum(tgt ** 2))
    return tot / max(len(pairs), 1)
