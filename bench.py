"""Benchmark of the spacetime finite-element Dirac solve on one MI355X.

Workload: 2+1D, 128^3 trilinear spacetime elements on [0,1]^2 x [0,1] (periodic
space), 2-component spinor, m = 1, seeded Gaussian packet (sigma = 0.05,
|p| in [5, 20]) mixing positive and negative energies; 4,194,304 unknowns.

One step = the whole hot path on that input, already resident in HBM:
assembly of the block-CSR operator (complex128 + complex64 values, node-block
Jacobi inverses) and of b, then the complex128 GMRES(50) solve to true
relative residual 1e-8 with the spectral preconditioner (exact for this
potential-free workload, so one Arnoldi step suffices).  Beside the timed
steps the script measures the same solve with complex64 inner cycles inside
FP64 refinement (two cycles: with an exact preconditioner the second FP64
residual costs more than the cheaper inner step saves), plain GMRES(50) with
node-block Jacobi over the 100-iteration window of the paper's scaling runs,
and the BSR SpMV kernels on their own with HIP events.  The CPU oracle is
timed on the host on the same workload.

Prints one JSON line.  Usage: python bench.py [--gpus 1] [--steps K] [--warmup W]
"""
from __future__ import annotations

import argparse
import json
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

METRIC = "2+1D 128³ solve time @1e-8: FP64 GMRES vs FP32-IR+NN-FGMRES; SpMV HBM GB/s"
HBM_PEAK_GBS = 8000.0


def spmv_bytes(op, cs):
    """Algorithmic bytes of one single-system SpMV: block values, x and y once
    each; for 2x2 blocks the kernel computes block addresses and columns from
    the stencil structure, for 4x4 blocks it reads the block-CSR indices."""
    if op.nc == 4:
        return spmv_bytes_indexed(op, cs)
    return op.nnzb * op.nc * op.nc * cs + 2 * op.n * cs


def spmv_bytes_indexed(op, cs):
    """Algorithmic bytes of one indexed BSR SpMV (the grouped batched kernel):
    values, column indices, row pointers, x and y once each."""
    return op.nnzb * (op.nc * op.nc * cs + 4) + 4 * (op.nrows + 1) + 2 * op.n * cs


def counter_traffic(kernel_key):
    """HBM bytes per launch of the SpMV measured with rocprofv3 counters
    (profiles/pmc_traffic_2p1d_128cubed.json), or None if the SpMV source has
    changed since the counters were taken."""
    import hashlib
    path = os.path.join(ROOT, "profiles", "pmc_traffic_2p1d_128cubed.json")
    if not os.path.exists(path):
        return None
    doc = json.load(open(path))
    h = hashlib.sha256()
    for f in ("paper_2103_14588_amd/csrc/spmv.hpp", "paper_2103_14588_amd/csrc/common.hpp"):
        h.update(open(os.path.join(ROOT, f), "rb").read())
    if h.hexdigest() != doc.get("spmv_source_sha256"):
        return None
    k = doc["kernels"].get(kernel_key)
    return None if k is None else int(k["traffic_bytes"])


def time_launches(fn, reps, torch):
    """Average duration of fn() launches on the current stream, HIP events."""
    s = torch.cuda.current_stream()
    fn()
    torch.cuda.synchronize()
    e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    e0.record(s)
    for _ in range(reps):
        fn()
    e1.record(s)
    e1.synchronize()
    return e0.elapsed_time(e1) / reps


def cpu_baseline(wl, x_gpu_list):
    """The oracle as it stands, on the host cores: element-loop assembly and
    GMRES(50) with the same spectral preconditioner to rtol 1e-8 on the full
    workload.  Also returns the forward error of the GPU solutions against it."""
    import numpy as np
    from oracle import oracle as O
    s = wl.spec
    p = O.problem(s.d, s.n, s.lens, s.m, s.vkind, s.v0, s.x0, s.lw)
    t0 = time.perf_counter()
    A = O.Matrix(p)
    b = A.rhs(wl.psi0)
    x, info = A.gmres(b, restart=wl.restart, max_it=200, rtol=wl.rtol, pc="spectral", vbar=0.0)
    sec = time.perf_counter() - t0
    errs = [float(np.linalg.norm(xg - x) / np.linalg.norm(x)) for xg in x_gpu_list]
    cores = int(os.environ.get("OMP_NUM_THREADS", os.cpu_count() or 1))
    cpu_model = "unknown"
    try:
        with open("/proc/cpuinfo") as f:
            cpu_model = next((ln.split(":", 1)[1].strip() for ln in f if ln.startswith("model name")), cpu_model)
    except OSError:
        pass
    return {"value": sec * 1e3, "unit": "ms", "cores": cores, "cpu_model": cpu_model, "kind": "oracle",
            "sample": "full workload: oracle element-loop assembly + GMRES(%d) spectral PC to %g "
                      "(%d iterations, relres %.2e)" % (wl.restart, wl.rtol, info["iters"], info["relres"])}, errs


def klein_bench(args):
    """2+1D 128^3 Klein step (V0 = 2.5 m): the learned preconditioner trained on
    the GPU on 2k (residual, error) pairs from plain GMRES restart iterates on
    32^3-64^3 Klein-step systems, then FGMRES(50) (complex64 inner cycles, FP64
    refinement) to 1e-8 with node-block Jacobi, node-block Jacobi + network,
    node-block Jacobi + untrained network, spectral, spectral + network, line
    (exact for this potential), line + network."""
    import torch
    from paper_2103_14588_amd import dirac_st as D
    from paper_2103_14588_amd import inputs as IN
    from paper_2103_14588_amd import nnpc

    torch.cuda.set_device(0)
    t0 = time.perf_counter()
    pairs = nnpc.make_pairs(n_systems=250, per_system=8, nmin=32, nmax=64, base="bj", restart=20, seed=1)
    gain, pairs = nnpc.normalise_targets(pairs)
    torch.cuda.synchronize()
    t_gen = time.perf_counter() - t0
    val = nnpc.make_pairs(n_systems=4, per_system=4, nmin=48, nmax=48, base="bj", restart=20, seed=99)
    val = [(s, x, (t / gain).contiguous()) for s, x, t in val]
    net, ctrl = D.Net(nnpc.he_init(0)), D.Net(nnpc.he_init(0), training=False)
    net.s.out_gain = ctrl.s.out_gain = gain
    l0 = nnpc.eval_loss(ctrl, val)
    t0 = time.perf_counter()
    losses = nnpc.train(net, pairs, epochs=2, lr=1e-3)
    torch.cuda.synchronize()
    t_train = time.perf_counter() - t0
    l1 = nnpc.eval_loss(net, val)
    del pairs

    wl = IN.klein_step_2p1(128, v0=2.5, seed=0)
    op, b = D.assemble(wl.spec, torch.from_numpy(wl.psi0).cuda())
    runs = {}
    cap = args.max_it
    for name, pc, nn in (("bj", "bj", None), ("bj+nn", "bj", net), ("bj+untrained_nn", "bj", ctrl),
                         ("spectral", "spectral", None), ("spectral+nn", "spectral", net),
                         ("line", "line", None), ("line+nn", "line", net)):
        if name == "line":
            # first use of the line preconditioner builds its tables: untimed,
            # as for the complex128 run below
            D.fgmres_nn(op, b, None, restart=50, max_it=cap, rtol=1e-8, pc=pc, vbar=1.25,
                        precision=32, inner_rtol=1e-5)
        x, info = D.fgmres_nn(op, b, nn, restart=50, max_it=cap, rtol=1e-8, pc=pc, vbar=1.25,
                              precision=32, inner_rtol=1e-5)
        runs[name] = {"iters": info["iters"], "relres": info["relres"], "converged": info["converged"],
                      "ms": round(info["ms"], 1), "fallback": info["fallback"]}
        print(name, runs[name], file=sys.stderr, flush=True)
    # the exact preconditioner in complex128: one Arnoldi step
    x = torch.zeros_like(b)
    D.gmres(op, b, x, restart=50, max_it=cap, rtol=1e-8, pc="line")
    x.zero_()
    _, info = D.gmres(op, b, x, restart=50, max_it=cap, rtol=1e-8, pc="line")
    runs["line_fp64"] = {"iters": info["iters"], "relres": info["relres"], "converged": info["converged"],
                         "ms": round(info["ms"], 2), "fallback": False}
    print("line_fp64", runs["line_fp64"], file=sys.stderr, flush=True)
    print(json.dumps({"workload": "2+1D 128^3 Klein step V0=2.5, FGMRES(50) FP32-IR to 1e-8, cap %d" % cap,
                      "train": {"pairs": 2000, "gen_s": round(t_gen, 2), "train_s": round(t_train, 2),
                                "steps": len(losses), "gain": gain, "heldout_untrained": l0,
                                "heldout_trained": l1},
                      "runs": runs}))


def slabs_bench(args):
    """Time decomposition on the 2+1D 128^3 packet and Klein step: complex128
    GMRES(50) to 1e-8 with the time-slab preconditioner for 1 (the exact line
    inverse), 2, 4, 8 and 32 slabs; iterations, residual and wall time."""
    import torch
    from paper_2103_14588_amd import dirac_st as D
    from paper_2103_14588_amd import inputs as IN

    torch.cuda.set_device(0)
    cap = args.max_it
    runs = []
    for name, wl in (("packet", IN.packet_2p1(128, seed=0)), ("klein", IN.klein_step_2p1(128, v0=2.5, seed=0))):
        op, b = D.assemble(wl.spec, torch.from_numpy(wl.psi0).cuda())
        for slabs in (1, 2, 4, 8, 32):
            D.gmres(op, b, restart=50, max_it=2, rtol=1e-8, pc="slabs", slabs=slabs)
            _, info = D.gmres(op, b, restart=50, max_it=cap, rtol=1e-8, pc="slabs", slabs=slabs)
            r = {"workload": name, "slabs": slabs, "iters": info["iters"], "converged": info["converged"],
                 "relres": info["relres"], "ms": round(info["ms"], 2),
                 "ms_per_iter": round(info["ms"] / max(info["iters"], 1), 3)}
            print(r, file=sys.stderr, flush=True)
            runs.append(r)
    print(json.dumps({"workload": "2+1D 128^3 packet and Klein step (V0=2.5), complex128 GMRES(50) to 1e-8 with "
                                  "the time-slab preconditioner, cap %d" % cap, "runs": runs}))


def cnn_bench(args):
    """The learned preconditioner's network on the 2+1D 128^3 grid (the Klein
    step workload's size): inference (four 3x3x3 convolutions, 4-16-16-16-4
    channels, bfloat16 on the matrix cores, FP32 accumulation) and one training
    step (forward, backward data and weights, Adam), timed with HIP events;
    achieved dense bf16 TFLOP/s against the MI355X peak."""
    import torch
    from paper_2103_14588_amd import dirac_st as D
    from paper_2103_14588_amd import nnpc

    torch.cuda.set_device(0)
    shape = (128, 128, 128)
    vox = shape[0] * shape[1] * shape[2]
    gen = torch.Generator(device="cuda").manual_seed(0)
    x = torch.randn(vox * 4, dtype=torch.float32, device="cuda", generator=gen)
    tgt = torch.randn(vox * 4, dtype=torch.float32, device="cuda", generator=gen)
    net = D.Net(nnpc.he_init(0))
    wf = torch.empty(D.nn_workspace_bytes(*shape), dtype=torch.uint8, device="cuda")
    wt = torch.empty(D.nn_workspace_bytes(*shape, training=True), dtype=torch.uint8, device="cuda")
    t_fwd = time_launches(lambda: D.nn_forward(net, x, shape, 1.0, wf), args.kernel_reps, torch)
    t_train = time_launches(lambda: D.nn_train_step(net, x, tgt, shape, 1e-6, work=wt), max(args.kernel_reps // 4, 2),
                            torch)
    macs = 27 * (4 * 16 + 16 * 16 + 16 * 16 + 16 * 4)  # per voxel
    fl = 2.0 * macs * vox
    peak = 2500.0  # dense bf16 TFLOP/s
    print(json.dumps({"workload": "network 4-16-16-16-4, 3x3x3 convolutions, 128^3 grid, bfloat16 MFMA",
                      "forward_ms": round(t_fwd, 4), "forward_gflop": round(fl / 1e9, 2),
                      "forward_tflops": round(fl / t_fwd / 1e9, 1),
                      "forward_frac_of_bf16_peak": round(fl / t_fwd / 1e9 / peak, 4),
                      "train_step_ms": round(t_train, 4),
                      "train_step_tflops_fwd_plus_2x_bwd": round(3 * fl / t_train / 1e9, 1)}))


def batch_bench(args):
    """64 Klein-step systems on uneven meshes n^3, n ~ U{32..96}, V0 ~ U[0, 3m]
    (seeded): one step = assembly of all 64 operators and right-hand sides,
    then one batched complex128 FGMRES call with the line preconditioner
    (exact for these potentials: one Arnoldi step per system) to relres 1e-8
    for every system.  Beside it: the batched solve with complex64 inner
    cycles in FP64 refinement, the same systems solved one after the other
    with the single-system solver, and the grouped SpMV over the whole batch
    for every lane count the autotuner may choose."""
    import numpy as np
    import torch
    from paper_2103_14588_amd import dirac_st as D
    from paper_2103_14588_amd import inputs as IN

    torch.cuda.set_device(0)
    wls = IN.klein_batch(64, seed=0, nmin=32, nmax=96)
    psis = [torch.from_numpy(w.psi0).cuda() for w in wls]
    ops, bs = [], []
    for w, p in zip(wls, psis):
        op, b = D.assemble(w.spec, p, block_jacobi=False)
        ops.append(op)
        bs.append(b)
    # the timed step's operators: its complex128 FGMRES with the line
    # preconditioner reads only the complex128 blocks, so the step assembles
    # those (no complex64 copies); the operators above serve the FP32-IR
    # comparison and the complex64 SpMV measurements
    ops64 = [D.assemble(w.spec, None, fp32=False, block_jacobi=False)[0] for w in wls]
    xs = [torch.zeros_like(b) for b in bs]
    kw = dict(restart=10, max_it=200, rtol=1e-8, pc="line", inner_rtol=1e-5)
    o32 = D.make_opts(precision=32, **kw)
    o64 = D.make_opts(precision=64, **{k: v for k, v in kw.items() if k != "inner_rtol"})
    work = torch.empty(max(D.batched_workspace_bytes(ops, o32), D.batched_workspace_bytes(ops, o64)),
                       dtype=torch.uint8, device="cuda")

    def step():
        for op, p, b in zip(ops64, psis, bs):
            D.assemble_into(op, p, b)
        for x in xs:
            x.zero_()
        _, infos, rc = D.fgmres_batched(ops64, bs, xs, opts=o64, work=work)
        return infos

    for _ in range(args.warmup):
        step()
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for _ in range(args.steps):
        infos = step()
    torch.cuda.synchronize()
    ms_step = (time.perf_counter() - t0) * 1e3 / max(args.steps, 1)

    def timed(fn):
        torch.cuda.synchronize()
        t = time.perf_counter()
        r = fn()
        torch.cuda.synchronize()
        return (time.perf_counter() - t) * 1e3, r

    for x in xs:
        x.zero_()
    D.fgmres_batched(ops, bs, xs, opts=o32, work=work)  # first call: lane autotuning for complex64
    for x in xs:
        x.zero_()
    ms_b32, (_, inf32, _) = timed(lambda: D.fgmres_batched(ops, bs, xs, opts=o32, work=work))
    x32 = [x.clone() for x in xs]
    for x in xs:
        x.zero_()
    ms_b64, (_, inf64, _) = timed(lambda: D.fgmres_batched(ops, bs, xs, opts=o64, work=work))
    err = max(float(torch.linalg.vector_norm(a - b) / torch.linalg.vector_norm(b)) for a, b in zip(x32, xs))

    def sequential():
        out = []
        for op, b in zip(ops, bs):
            x = torch.zeros_like(b)
            _, inf = D.gmres(op, b, x, **{k: v for k, v in kw.items() if k != "inner_rtol"})
            out.append(inf)
        return out
    sequential()
    ms_seq, inf_seq = timed(sequential)

    rows = sum(op.nrows for op in ops)
    lanes = {"c128": D.batched_lanes(2, 64, rows), "c64": D.batched_lanes(2, 32, rows)}
    spmv = {}
    gen = torch.Generator(device="cuda").manual_seed(0)
    v32 = [torch.randn(op.n, dtype=torch.complex64, device="cuda", generator=gen) for op in ops]
    y32 = [torch.empty_like(v) for v in v32]
    nbytes = sum(spmv_bytes(op, 8) for op in ops)
    swork = torch.empty(D.spmv_batched_workspace_bytes(ops), dtype=torch.uint8, device="cuda")
    for g in (1, 4, 8, 16, 32):  # 1: the x-staged line-tile kernel
        ms = time_launches(lambda: D.spmv_batched(ops, v32, y32, lanes=g, work=swork), args.kernel_reps, torch)
        spmv["lds_tile" if g == 1 else str(g)] = {"ms": round(ms, 4), "GBps": round(nbytes / ms / 1e6, 1)}
    it = np.array([i["iters"] for i in infos])
    print(json.dumps({
        "workload": "64 Klein-step 2+1D systems, n^3 with n ~ U{32..96}, V0 ~ U[0,3] (seed 0): assemble all "
                    "(complex128 blocks) + batched complex128 FGMRES(10) line PC, rtol 1e-8",
        "systems": len(ops), "block_rows": rows, "unknowns": 2 * rows,
        "step_ms": round(ms_step, 2), "steps": args.steps, "warmup": args.warmup,
        "converged": int(sum(i["converged"] for i in infos)),
        "max_relres": max(i["relres"] for i in infos),
        "iters": {"min": int(it.min()), "max": int(it.max()), "mean": round(float(it.mean()), 2)},
        "cycles_max": max(i["cycles"] for i in infos),
        "solve_only_ms": {"batched_fp64": round(ms_b64, 2), "batched_fp32_ir": round(ms_b32, 2),
                          "sequential_fp64": round(ms_seq, 2)},
        "fp32_ir_converged": int(sum(i["converged"] for i in inf32)),
        "sequential_converged": int(sum(i["converged"] for i in inf_seq)),
        "max_rel_diff_fp32ir_vs_fp64": err,
        "autotuned_lanes": lanes,
        "grouped_spmv_c64": spmv, "grouped_spmv_bytes": nbytes,
        "memory_GB": round((sum(op.bytes() for op in ops + ops64) + work.numel()) / 1e9, 2),
    }))


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=5)
    ap.add_argument("--warmup", type=int, default=2)
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--kernel-reps", type=int, default=20)
    ap.add_argument("--only", choices=["spmv64", "spmv32", "assemble", "copy", "mf64"], default=None,
                    help="launch only this kernel --kernel-reps times (for counter runs)")
    ap.add_argument("--workload", choices=["packet", "packet3", "plane1", "klein", "batch", "slabs", "cnn"],
                    default="packet",
                    help="packet: the 2+1D 128^3 packet step (default bench line); packet3: the 3+1D "
                         "32^4 packet; plane1: the 1+1D 64x64 plane wave; klein: the "
                         "learned-preconditioner comparison on the 128^3 Klein step; batch: 64 "
                         "uneven Klein-step systems in one batched solve; slabs: the time-slab "
                         "preconditioner for 1-32 slabs on the 128^3 packet and Klein step; cnn: the "
                         "learned preconditioner's network alone on the 128^3 grid")
    ap.add_argument("--max-it", type=int, default=1500)
    args = ap.parse_args()
    if args.gpus != 1 or int(os.environ.get("WORLD_SIZE", "1")) != 1:
        print("bench.py measures one GPU only (this build has no multi-GPU path); "
              "run it with --gpus 1", file=sys.stderr)
        sys.exit(2)
    if args.workload == "klein":
        return klein_bench(args)
    if args.workload == "batch":
        return batch_bench(args)
    if args.workload == "slabs":
        return slabs_bench(args)
    if args.workload == "cnn":
        return cnn_bench(args)

    import numpy as np
    import torch
    from paper_2103_14588_amd import dirac_st as D
    from paper_2103_14588_amd import inputs as IN

    torch.cuda.set_device(0)
    wl = {"packet": lambda: IN.packet_2p1(128, seed=0), "packet3": lambda: IN.packet_3p1(32, seed=0),
          "plane1": lambda: IN.plane_wave_1p1(64)}[args.workload]()
    spec = wl.spec
    psi0 = torch.from_numpy(wl.psi0).cuda()
    op, b = D.assemble(spec, psi0)
    x = torch.zeros_like(b)
    if args.only:
        # one kernel, --kernel-reps launches, nothing else on the GPU
        xx = torch.randn(op.n, dtype=torch.complex128, device="cuda")
        yy = torch.empty_like(xx)
        xx32, yy32 = xx.to(torch.complex64), torch.empty(op.n, dtype=torch.complex64, device="cuda")
        fn = {"spmv64": lambda: D.spmv(op, xx, yy), "spmv32": lambda: D.spmv(op, xx32, yy32),
              "assemble": lambda: D.assemble_into(op, psi0, b), "copy": lambda: yy.copy_(xx),
              "mf64": lambda: D.spmv_mf(op, xx, yy)}[args.only]
        ms = time_launches(fn, args.kernel_reps, torch)
        nbytes = {"spmv64": spmv_bytes(op, 16), "spmv32": spmv_bytes(op, 8),
                  "assemble": op.bytes() + op.n * 16 + psi0.numel() * 16, "copy": 2 * op.n * 16,
                  "mf64": 2 * op.n * 16}[args.only]
        print(json.dumps({"only": args.only, "reps": args.kernel_reps, "ms": ms, "bytes": nbytes,
                          "GBps": nbytes / ms / 1e6}))
        return
    m, rtol = wl.restart, wl.rtol
    # The timed step's operator: its complex128 GMRES with the spectral
    # preconditioner reads only the complex128 blocks (with their pattern), so
    # the step assembles those and not the complex64 copy or the node-block
    # inverses; the full operator above serves the FP32-IR, block-Jacobi and
    # BiCGSTAB comparisons and the isolated kernel timings.
    op64, b64 = D.assemble(spec, psi0, fp32=False, block_jacobi=False)
    asm64_bytes = op64.bytes() + op64.n * 16 + psi0.numel() * 16
    o32 = D.make_opts(restart=m, max_it=2000, pc="spectral", precision=32, rtol=rtol,
                      inner_rtol=1e-4, vbar=0.0)
    o64 = D.make_opts(restart=m, max_it=2000, pc="spectral", precision=64, rtol=rtol, vbar=0.0)
    work = torch.empty(max(D.workspace_bytes(op, o32, flexible=True), D.workspace_bytes(op, o64, flexible=True)),
                       dtype=torch.uint8, device="cuda")

    def step():
        D.assemble_into(op64, psi0, b64)
        x.zero_()
        _, info = D.gmres(op64, b64, x, opts=o64, work=work)
        return info

    for _ in range(args.warmup):
        step()
    torch.cuda.synchronize()
    # HIP events around the SpMV, residual and assembly launches inside the
    # timed steps (recorded by the library on its launch stream)
    D.timing(True)
    t0 = time.perf_counter()
    infos = [step() for _ in range(args.steps)]
    torch.cuda.synchronize()
    ms_step = (time.perf_counter() - t0) * 1e3 / max(args.steps, 1)
    live = {k: D.timing_read(k) for k in ("spmv64", "resid64", "assemble")}
    D.timing(False)
    info_step = infos[-1]

    # complex128 GMRES(50) on the same system (assembly excluded from both solve times)
    def solve(o):
        x.zero_()
        torch.cuda.synchronize()
        t = time.perf_counter()
        _, inf = D.gmres(op, b, x, opts=o, work=work)
        torch.cuda.synchronize()
        return (time.perf_counter() - t) * 1e3, inf
    solve(o64)
    ms64, info64 = solve(o64)
    x64 = x.clone()
    solve(o32)
    ms32, info32b = solve(o32)
    x32 = x.clone()

    # the same complex128 solve with the matrix-free operator
    omf = D.make_opts(restart=m, max_it=2000, pc=o64.pc, vbar=o64.vbar, precision=64, rtol=rtol, matrix_free=True)
    solve(omf)
    ms_mf, info_mf = solve(omf)

    # plain GMRES(50) with node-block Jacobi: the 100-iteration window
    obj = D.make_opts(restart=m, max_it=100, pc="bj", precision=64, rtol=rtol)
    ms_bj, info_bj = solve(obj)
    # the same 100-iteration window with FP32-IR (complex64 inner cycles): the
    # regime where iterations dominate and the reduced precision pays
    obj32 = D.make_opts(restart=m, max_it=100, pc="bj", precision=32, rtol=rtol, inner_rtol=1e-4)
    solve(obj32)
    ms_bj32, info_bj32 = solve(obj32)

    # BiCGSTAB (the paper's second solver): with the step's preconditioner, and
    # the 100-iteration window with node-block Jacobi
    def solve_bi(o):
        x.zero_()
        torch.cuda.synchronize()
        t = time.perf_counter()
        try:
            _, inf = D.bicgstab(op, b, x, opts=o)
        except D.DiracError as e:  # a non-finite residual ends the window
            inf = {"iters": -1, "relres": float("nan"), "error": str(e)}
        torch.cuda.synchronize()
        return (time.perf_counter() - t) * 1e3, inf
    obi = D.make_opts(max_it=args.max_it, pc=o64.pc, vbar=o64.vbar, precision=64, rtol=rtol)
    solve_bi(obi)
    ms_bi, info_bi = solve_bi(obi)
    obibj = D.make_opts(max_it=100, pc="bj", precision=64, rtol=rtol)
    solve_bi(obibj)
    ms_bibj, info_bibj = solve_bi(obibj)

    # kernels on their own (HIP events on the launch stream)
    reps = args.kernel_reps
    xx = torch.randn(op.n, dtype=torch.complex128, device="cuda")
    yy = torch.empty_like(xx)
    xx32, yy32 = xx.to(torch.complex64), torch.empty(op.n, dtype=torch.complex64, device="cuda")
    t_spmv64 = time_launches(lambda: D.spmv(op, xx, yy), reps, torch)
    t_spmv32 = time_launches(lambda: D.spmv(op, xx32, yy32), reps, torch)
    t_asm = time_launches(lambda: D.assemble_into(op, psi0, b), max(reps // 4, 2), torch)
    pcw = torch.empty(D.workspace_bytes(op, o32), dtype=torch.uint8, device="cuda")
    t_pc32 = time_launches(lambda: D.pc_apply(op, xx32, "spectral", 0.0, yy32, pcw), max(reps // 4, 2), torch)
    # the matrix-free operator: x read and y written once (the stencil
    # coefficients are computed, not read)
    t_mf64 = time_launches(lambda: D.spmv_mf(op, xx, yy), reps, torch)
    t_mf32 = time_launches(lambda: D.spmv_mf(op, xx32, yy32), reps, torch)
    # achievable bandwidth of a plain device copy on this GPU (2 GiB read + 2 GiB
    # written by torch's copy kernel), reported beside the fractions of peak
    cbig = torch.empty(2 ** 31 // 16, dtype=torch.complex128, device="cuda")
    cdst = torch.empty_like(cbig)
    t_copy = time_launches(lambda: cdst.copy_(cbig), 5, torch)
    copy_gbs = 2 * cbig.numel() * 16 / t_copy / 1e6
    del cbig, cdst
    by64, by32 = spmv_bytes(op, 16), spmv_bytes(op, 8)
    gbs64, gbs32 = by64 / t_spmv64 / 1e6, by32 / t_spmv32 / 1e6
    asm_bytes = op.bytes() + op.n * 16 + psi0.numel() * 16

    def live_avg(k):
        n, ms = live[k]
        return (ms / n if n else None), n
    l_spmv, n_spmv = live_avg("spmv64")
    l_res, n_res = live_avg("resid64")
    l_asm, n_asm = live_avg("assemble")
    res_bytes = by64 + op.n * 16  # the residual form also reads b
    rl_kernel = ("spmv_lds_kernel<double,%d,16,2,false> (structured block SpMV, x staged in LDS, complex128)" % spec.d
                 if op.nc == 2 else "spmv_kernel<double,4,64,false> (BSR SpMV, complex128)")
    if l_spmv is None:  # no product in the timed steps: fall back to the isolated launches
        l_spmv, n_spmv = t_spmv64, 0
    g_live = by64 / l_spmv / 1e6

    out = {
        "metric": METRIC,
        "value": round(ms_step, 3),
        "unit": "ms",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": round(ms_step, 3),
        "higher_is_better": False,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "c128",
        "data": "synthetic",
        "config": {"workload": "%s Q1 spacetime Dirac (seed 0); assemble (complex128 blocks) + complex128 "
                               "GMRES(%d) (spectral PC) to relres %g" % (wl.name, m, rtol),
                   "mesh_elements": spec.n, "unknowns": op.n, "blocks": op.nnzb, "restart": m,
                   "rtol": rtol},
        "solve": {
            "fp32_ir_ms": round(ms32, 3), "fp32_ir_iters": info32b["iters"],
            "fp32_ir_cycles": info32b["cycles"], "fp32_ir_relres": info32b["relres"],
            "fp64_ms": round(ms64, 3), "fp64_iters": info64["iters"], "fp64_relres": info64["relres"],
            "speedup_fp32ir_vs_fp64": round(ms64 / ms32, 3),
            "step_relres": info_step["relres"], "step_iters": info_step["iters"],
            "plain_bj_100it_ms": round(ms_bj, 3), "plain_bj_100it_relres": info_bj["relres"],
            "plain_bj_ms_per_iter": round(ms_bj / max(info_bj["iters"], 1), 4),
            "fp32_ir_bj_100it_ms": round(ms_bj32, 3), "fp32_ir_bj_100it_relres": info_bj32["relres"],
            "fp32_ir_bj_ms_per_iter": round(ms_bj32 / max(info_bj32["iters"], 1), 4),
            "speedup_fp32ir_vs_fp64_per_iter_bj": round((ms_bj / max(info_bj["iters"], 1))
                                                        / (ms_bj32 / max(info_bj32["iters"], 1)), 3),
            "fp64_matrix_free_ms": round(ms_mf, 3), "fp64_matrix_free_iters": info_mf["iters"],
            "fp64_matrix_free_relres": info_mf["relres"],
            "bicgstab_ms": round(ms_bi, 3), "bicgstab_iters": info_bi["iters"],
            "bicgstab_relres": info_bi["relres"],
            "bicgstab_bj_100it_ms": round(ms_bibj, 3), "bicgstab_bj_100it_relres": info_bibj["relres"],
            "bicgstab_bj_ms_per_iter": round(ms_bibj / max(info_bibj["iters"], 1), 4),
        },
        "kernels_ms": {"spmv_c128": round(t_spmv64, 4), "spmv_c64": round(t_spmv32, 4),
                       "assemble": round(t_asm, 4), "spectral_pc_c64": round(t_pc32, 4),
                       "spmv_matrix_free_c128": round(t_mf64, 4), "spmv_matrix_free_c64": round(t_mf32, 4)},
        "spmv": {"c128_GBps": round(gbs64, 1), "c64_GBps": round(gbs32, 1),
                 "c128_frac": round(gbs64 / HBM_PEAK_GBS, 4), "c64_frac": round(gbs32 / HBM_PEAK_GBS, 4),
                 "c128_bytes": by64, "c64_bytes": by32,
                 "device_copy_2GiB_GBps": round(copy_gbs, 1),
                 "c128_frac_of_device_copy": round(gbs64 / copy_gbs, 4),
                 "c128_in_step_frac_of_device_copy": round(by64 / l_spmv / 1e6 / copy_gbs, 4)},
        "roofline": {"kernel": rl_kernel, "bound": "hbm",
                     "achieved": round(g_live, 1), "peak": HBM_PEAK_GBS, "unit": "GB/s",
                     "frac": round(g_live / HBM_PEAK_GBS, 4),
                     "traffic": counter_traffic("spmv64") if args.workload == "packet" else None,
                     "algorithmic_bytes": by64, "avg_launch_ms": round(l_spmv, 4),
                     "launches_timed": n_spmv,
                     "measured": "HIP events on the launch stream around every launch in the timed steps"},
        "roofline_other": {
            "resid_c128": None if l_res is None else
            {"bound": "hbm", "avg_launch_ms": round(l_res, 4), "launches_timed": n_res,
             "algorithmic_bytes": res_bytes, "achieved": round(res_bytes / l_res / 1e6, 1),
             "frac": round(res_bytes / l_res / 1e6 / HBM_PEAK_GBS, 4)},
            "assemble": None if l_asm is None else
            {"bound": "hbm", "avg_launch_ms": round(l_asm, 4), "launches_timed": n_asm,
             "writes": "complex128 blocks, pattern, right-hand side (the step's operator)",
             "algorithmic_bytes": asm64_bytes, "achieved": round(asm64_bytes / l_asm / 1e6, 1),
             "frac": round(asm64_bytes / l_asm / 1e6 / HBM_PEAK_GBS, 4)},
            "spmv_matrix_free_c128": {"bound": "hbm", "avg_launch_ms": round(t_mf64, 4),
                                      "algorithmic_bytes": 2 * op.n * 16,
                                      "achieved": round(2 * op.n * 16 / t_mf64 / 1e6, 1),
                                      "frac": round(2 * op.n * 16 / t_mf64 / 1e6 / HBM_PEAK_GBS, 4),
                                      "speedup_vs_stored_blocks": round(t_spmv64 / t_mf64, 2)}},
        "assembly": {"ms": round(t_asm, 4), "bytes_written": asm_bytes,
                     "GBps": round(asm_bytes / t_asm / 1e6, 1),
                     "writes": "complex128 and complex64 blocks, pattern, node-block inverses in both "
                               "precisions, right-hand side (the full operator, isolated launches)"},
        "memory_GB": round((op.bytes() + op64.bytes() + work.numel()) / 1e9, 3),
        "paper_context": "the paper prints no runtime: its scaling runs timed 100 GMRES iterations "
                         "(2+1D up to 128^3) with PETSc on dual-socket 18-core Intel Broadwell E5-2695 v4 "
                         "nodes, 32 MPI ranks per node; the same window here is solve.plain_bj_100it_ms",
    }
    if not args.no_cpu_baseline:
        cb, errs = cpu_baseline(wl, [x32.cpu().numpy(), x64.cpu().numpy()])
        out["cpu_baseline"] = cb
        out["forward_error_vs_oracle"] = {"fp32_ir": errs[0], "fp64": errs[1]}
    print(json.dumps(out))


if __name__ == "__main__":
    main()
