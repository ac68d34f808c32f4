#!/usr/bin/env python3
"""Benchmark of the MI355X Newton step (one GPU).

A step is one Newton iteration of the given-length load sequence of the 3D
penny-shaped crack workload in its precision form (Kuhn n=40 -> 384,000 P2
tetrahedra, 11.52M displacement DOF, viscosity-dominated parameters mu = 0.1,
sigma_c = 1e-3, G_c = 1e-6): assemble R and J, build the two-level block
preconditioner (element blocks, P1 vertex coarse space, Schur pressure
block), GMRES to a true relative residual of 1e-10, update.  The sequence
starts from the uniform-pressure elastic predictor (computed once, untimed);
the timed steps continue the load sequence from there (a load step that
converges ends with w_old <- w(u)), after W untimed warm-up steps and a
reset.

Printed JSON line: value = FP64 Newton steps/s.  Extra fields: GMRES
throughput, the same steps in FP32-IR mode (speed-up and state error
against FP64), the roofline of the dominant kernel (block-sparse Jacobian
product, timed with HIP events on the library stream inside the timed
region: the GMRES iterations replay captured HIP graphs, so the events time
the products outside them -- each incremental assembly's residual rows and
the coarse operator's A P columns -- the same kernel and pattern as the
iterations' products), the batched ensemble workload (64 2D instances, see
``ensemble_block``), and the CPU oracle timed on a bounded sample of the
same workload.
"""
from __future__ import annotations

import argparse
import json
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

METRIC = "Newton steps/s & GMRES iters/s (MDOF), FP32-IR vs FP64 at rel.res 1e-10"
HBM_PEAK_GBS = 8000.0


def spmv_traffic(workload_name):
    """HBM bytes per FP64 Jacobian product from the committed hardware-counter
    summary of this workload, or None when there is none or the product's
    kernel source has changed since the counters were taken."""
    import hashlib
    import re
    path = os.path.join(ROOT, "profiles", f"spmv_fp64_{workload_name}.md")
    src = os.path.join(ROOT, "paper_1911_10275_amd", "csrc", "hf_kernels_spmv.hip")
    if not os.path.exists(path):
        return None
    text = open(path).read()
    t = re.search(r"^traffic_bytes_per_launch = (\d+)$", text, re.M)
    h = re.search(r"^source_sha256 = ([0-9a-f]{64})$", text, re.M)
    if not t or not h:
        return None
    if hashlib.sha256(open(src, "rb").read()).hexdigest() != h.group(1):
        return None
    return int(t.group(1))


def host_info():
    """CPU model, logical CPU count and RAM of the host (Linux /proc)."""
    model, mem_kb = "unknown", 0
    try:
        for line in open("/proc/cpuinfo"):
            if line.startswith("model name"):
                model = line.split(":", 1)[1].strip()
                break
        for line in open("/proc/meminfo"):
            if line.startswith("MemTotal"):
                mem_kb = int(line.split()[1])
                break
    except OSError:
        pass
    return {"cpu_model": model, "nproc": os.cpu_count(), "ram_gib": round(mem_kb / 2**20, 1)}


def run_steps(ctx, st0, K, W, profile):
    """W warm-up Newton iterations, reset, then K timed iterations of the
    load sequence.  Returns (seconds, per-step stats, final state)."""
    import torch
    ctx.set_state(st0.u, st0.p, st0.w_old)
    for _ in range(W):
        ns = ctx.newton_step()
        if ns.converged:
            ctx.end_load_step()
    ctx.set_state(st0.u, st0.p, st0.w_old)
    ctx.reset_profile()
    ctx.set_options(profile=1 if profile else 0)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    stats = []
    for _ in range(K):
        ts = time.perf_counter()
        ns = ctx.newton_step()  # returns after the step's work has finished on the GPU
        if ns.converged:
            ctx.end_load_step()
        stats.append((ns.lin.gmres_iters, ns.lin.ir_steps, ns.lin.true_relres, ns.du_rel,
                      ns.dp_rel, ns.converged, ns.lin.fp64_iters, time.perf_counter() - ts))
    torch.cuda.synchronize()
    dt = time.perf_counter() - t0
    prof = ctx.profile()
    ctx.set_options(profile=0)
    return dt, stats, prof, ctx.get_state()


def cpu_baseline(prob, gpu_iters_per_step, n_el=4000, n_face=8000, n_blk=24000, n_it=2):
    """The oracle on a bounded sample of the same workload, single thread:
    bulk terms of about n_el elements and interface terms of about n_face
    faces (plus the fluid faces), each scaled to the whole mesh; the
    block-Jacobi setup (element-block inverses and Schur pressure block) on
    about n_blk element blocks, scaled; n_it GMRES(60) iterations on the full
    block pattern (with the block-Jacobi application over every element
    block), scaled with the GPU's GMRES iteration count per Newton step (the
    oracle's own solver is block-Jacobi GMRES, which needs more iterations
    than the GPU's two-level preconditioner: the scaling favours the CPU).
    Building the oracle's mesh tables is set-up, untimed."""
    import types
    from threadpoolctl import threadpool_limits
    import numpy as np
    from oracle import assemble as asm
    from oracle import newton, solve
    from oracle.newton import Case
    none = np.zeros(0, dtype=np.int64)
    with threadpool_limits(limits=1):
        case = Case.from_problem(prob)
        st = newton.initial_state(case)
        m = case.mesh
        args = (m, case.itf, case.prm, st.u, st.p, st.w_old, st.s_p, case.src_pnode, case.src_q0)
        t = time.perf_counter()
        asm.assemble(*args, faces=none, elements=none)
        t_fixed = time.perf_counter() - t          # per-call costs independent of the sample
        el = np.arange(0, m.ne, max(m.ne // n_el, 1))
        t = time.perf_counter()
        asm.assemble(*args, faces=none, elements=el)
        t_vol = max(time.perf_counter() - t - t_fixed, 0.0) * m.ne / len(el)
        fs = np.union1d(np.arange(0, m.nf, max(m.nf // n_face, 1)), case.itf.active_faces)
        t = time.perf_counter()
        S = asm.assemble(*args, faces=fs, elements=el)
        t_faces = max(time.perf_counter() - t - t_fixed - t_vol * len(el) / m.ne, 0.0) * m.nf / len(fs)
        # blocks outside the sample hold no terms: shift every block so that the
        # (timed) factorisation sees invertible blocks
        S.A_diag += np.eye(m.bu)[None] * max(np.abs(S.A_diag).max(), 1.0)
        fa = case.itf.active_faces   # with the elements that carry the coupling strips
        sub = np.union1d(np.arange(0, m.ne, max(m.ne // n_blk, 1)),
                         np.concatenate([m.face_em[fa], m.face_ep[fa]]))
        rows = (sub[:, None] * m.bu + np.arange(m.bu)[None, :]).reshape(-1)
        part = types.SimpleNamespace(A_diag=S.A_diag[sub], D=S.D, C=S.C.tocsc()[:, rows],
                                     B=S.B.tocsr()[rows])
        t = time.perf_counter()
        pc = solve.BlockJacobi(types.SimpleNamespace(ne=len(sub), bu=m.bu), part)
        t_bj = (time.perf_counter() - t) * m.ne / len(sub)
        # the iterations apply block-Jacobi over every element block: same shapes,
        # the (already timed) inverses' values do not change the work
        pc.ne, pc.inv = m.ne, S.A_diag
        op = solve.Operator(m, S)
        t = time.perf_counter()
        solve.gmres(op, -S.R, pc, m=60, rtol=1e-30, maxit=n_it)
        t_it = (time.perf_counter() - t) / n_it
    t_step = t_fixed + t_vol + t_faces + t_bj + gpu_iters_per_step * t_it
    return {"value": 1.0 / t_step, "unit": "Newton steps/s", "cores": 1, "kind": "oracle",
            "host": host_info(),
            "sample": (f"oracle (numpy, 1 thread) on the same workload: bulk terms of "
                       f"{len(el)}/{m.ne} elements and interface terms of {len(fs)}/{m.nf} "
                       f"faces, each scaled to the mesh ({t_vol:.1f} s + {t_faces:.1f} s, plus "
                       f"{t_fixed:.1f} s of per-call work), block-Jacobi setup on "
                       f"{len(sub)}/{m.ne} element blocks scaled ({t_bj:.1f} s), {n_it} GMRES(60) "
                       f"iterations ({t_it:.3f} s each) scaled to the GPU's "
                       f"{gpu_iters_per_step:.0f} iterations per Newton step")}


def counters_probe(prob):
    """Launches for hardware-counter runs: one copy of 1 GiB between two
    device buffers (a kernel of known traffic: 1 GiB read, 1 GiB written),
    then five FP64 block-sparse Jacobian products of the workload."""
    import numpy as np
    import torch
    import paper_1911_10275_amd as hf
    stream = torch.cuda.current_stream().cuda_stream
    ctx = hf.context_for_problem(prob, device=0, stream=stream)
    sz = ctx.sizes
    ctx.set_state(np.zeros(sz.n_u), np.full(sz.n_p, prob.material.sigma_c))
    ctx.assemble()
    cache = os.path.join(ROOT, "paper_1911_10275_amd", "tuning_cache.txt")
    if os.path.exists(cache):  # the schedule the benchmark chose (cache lookup, no timing)
        ctx.autotune(level=-1, cache_path=cache)
    a = torch.ones(1 << 27, dtype=torch.float64, device="cuda")
    b = torch.empty_like(a)
    b.copy_(a)
    x = torch.randn(sz.n_total, dtype=torch.float64, device="cuda")
    y = torch.empty_like(x)
    for _ in range(5):
        ctx.apply_jacobian(x.data_ptr(), y.data_ptr())
    torch.cuda.synchronize()
    # one FP32-IR preconditioner build (the solve stops after one iteration)
    ctx.set_options(precision=hf.HF_FP32_IR, gmres_maxit=1)
    ctx.solve(check=False)
    torch.cuda.synchronize()
    print(f"counters probe done: copy 1 GiB, 5 products, N = {sz.n_total}, "
          f"tuning {ctx.tuning().as_dict()}", file=sys.stderr)
    ctx.close()


def assembly_probe(prob, n):
    """n full assemblies of the workload (incremental assembly off), timed
    with HIP events on the library stream, after one untimed; one 1 GiB device
    copy first (a kernel of known traffic, for calibrating the hardware
    counters).  Prints one JSON line: ms per assembly and the rate of its
    algorithmic bytes (the Jacobian blocks written once, u read, R written)."""
    import numpy as np
    import torch
    import paper_1911_10275_amd as hf
    stream = torch.cuda.current_stream().cuda_stream
    ctx = hf.context_for_problem(prob, device=0, stream=stream, incremental_assembly=0, profile=1)
    sz = ctx.sizes
    a = torch.ones(1 << 27, dtype=torch.float64, device="cuda")
    b = torch.empty_like(a)
    b.copy_(a)
    del a, b
    rng = np.random.default_rng(0)
    ctx.set_state(rng.normal(0.0, 1e-3, sz.n_u), np.full(sz.n_p, prob.material.sigma_c),
                  np.zeros((sz.n_face, sz.nq_face)))
    ctx.assemble()
    ctx.reset_profile()
    for _ in range(n):
        ctx.assemble()
    torch.cuda.synchronize()
    pr = ctx.profile()
    ms = pr.ms_assemble / max(pr.n_assemble, 1)
    nbytes = sz.n_blocks * sz.block_size ** 2 * 8 + 2 * sz.n_u * 8
    print(json.dumps({"probe": "full assembly", "workload": prob.name, "elements": int(sz.n_elem),
                      "assemblies": int(pr.n_assemble), "ms_per_assembly": ms,
                      "algorithmic_bytes": int(nbytes), "GBps": nbytes / (ms * 1e-3) / 1e9,
                      "frac_hbm": nbytes / (ms * 1e-3) / (HBM_PEAK_GBS * 1e9)}), flush=True)
    ctx.close()


def ensemble_block(K, gmres_m, tune_level=1, two_level=0):
    """The batched 2D KGD ensemble: 64 instances (1k-20k triangles, mixed P1 /
    P2, materials and injection drawn per instance).  The P1 and the P2
    instances each form one batched context (every kernel launch covers all
    instances of the context); the two contexts run concurrently on two
    streams from two host threads.  One ensemble step = one Newton iteration
    (assemble, block-Jacobi, GMRES to 1e-10, update) of every instance, from
    the uniform-pressure predictor; K timed steps after one warm-up step and
    a reset, in FP64 and in FP32-IR, each context autotuned (untimed, cached)
    on its predictor state first.  A linear solve that has not reached
    1e-10 within 6,000 GMRES iterations counts as failed (reported; its
    instance keeps its state and its step is not counted)."""
    import threading
    import numpy as np
    import torch
    import paper_1911_10275_amd as hf
    import synth
    probs = synth.ensemble(64, seed=4)
    groups = [[p for p in probs if p.order == o] for o in (1, 2)]
    ctxs, starts, streams = [], [], []
    for ps in groups:
        stm = torch.cuda.Stream()
        c = hf.context_for_problems(ps, device=0, stream=stm.cuda_stream, gmres_m=gmres_m,
                                    two_level=two_level)
        for i, p in enumerate(ps):
            s = c.isizes[i]
            c.set_state(np.zeros(s.n_u), np.full(s.n_p, p.material.sigma_c),
                        np.zeros((s.n_face, s.nq_face)), inst=i)
        c.initial_guess()
        c.set_options(gmres_maxit=6000)
        starts.append([c.get_state(i) for i in range(len(ps))])
        ctxs.append(c)
        streams.append(stm)

    def reset(c, st):
        for i, (u, p, _, wo) in enumerate(st):
            c.set_state(u, p, wo, inst=i)

    def steps(c, n, sink):
        for _ in range(n):
            sink.append(c.newton_step(check=False))

    res = {}
    cache = os.path.join(ROOT, "paper_1911_10275_amd", "tuning_cache.txt")
    for name, prec in (("fp64", hf.HF_FP64), ("fp32_ir", hf.HF_FP32_IR)):
        tuned = []
        for c, st in zip(ctxs, starts):
            c.set_options(precision=prec)
            reset(c, st)
            c.assemble()
            tuned.append(c.autotune(level=tune_level, cache_path=cache).as_dict())
            reset(c, st)
            c.newton_step(check=False)
            reset(c, st)
        torch.cuda.synchronize()
        sinks = [[] for _ in ctxs]
        threads = [threading.Thread(target=steps, args=(c, K, sk)) for c, sk in zip(ctxs, sinks)]
        t0 = time.perf_counter()
        for th in threads:
            th.start()
        for th in threads:
            th.join()
        torch.cuda.synchronize()
        dt = time.perf_counter() - t0
        flat = [n for sk in sinks for step in sk for n in step]
        ok = [n for n in flat if n.lin.status == 0]
        dof = sum(c.sizes.n_total for c in ctxs)
        gits = sum(n.lin.gmres_iters for n in flat)
        res[name] = {"steps_per_s": K / dt, "instance_newton_steps_per_s": len(ok) / dt,
                     "ms_per_step": 1e3 * dt / K, "gmres_iters_per_s": gits / dt,
                     "failed_solves": len(flat) - len(ok),
                     "fp64_finished_solves": sum(1 for n in flat if n.lin.fp64_iters > 0),
                     "max_true_relres_converged": max(n.lin.true_relres for n in ok),
                     "tuning": tuned}
        print(f"bench: ensemble {name} {K} steps in {dt:.3f} s", file=sys.stderr, flush=True)
    for c in ctxs:
        c.close()
    res["speedup_fp32_ir_vs_fp64"] = res["fp32_ir"]["steps_per_s"] / res["fp64"]["steps_per_s"]
    res["config"] = {"instances": len(probs), "p1": len(groups[0]), "p2": len(groups[1]),
                     "triangles": int(sum(p.n_elem for p in probs)), "dof": int(dof),
                     "contexts": 2, "streams": 2}
    return res


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=6)
    ap.add_argument("--warmup", type=int, default=1)
    ap.add_argument("--workload", type=int, default=3, help="synthetic workload index (1, 2, 3, 5)")
    ap.add_argument("--no-cpu", action="store_true", help="skip the CPU oracle baseline")
    ap.add_argument("--no-ir", action="store_true", help="skip the FP32-IR comparison")
    ap.add_argument("--gmres-m", type=int, default=60, help="GMRES restart length")
    ap.add_argument("--no-ensemble", action="store_true", help="skip the batched ensemble")
    ap.add_argument("--tune", type=int, default=1, choices=(-1, 0, 1),
                    help="autotune level before timing (-1: apply a cached choice only, never "
                         "time); choices cached in paper_1911_10275_amd/tuning_cache.txt")
    ap.add_argument("--ensemble-steps", type=int, default=3)
    ap.add_argument("--ensemble-m", type=int, default=120, help="GMRES restart length, ensemble")
    ap.add_argument("--coarse-fp32", type=int, default=1, choices=(0, 1),
                    help="1: FP64 solves apply the coarse factorisation rounded to FP32")
    ap.add_argument("--coarse-reuse", type=int, default=16,
                    help="two-level builds that keep the last coarse factorisation (0: refactorise "
                         "at every build)")
    ap.add_argument("--two-level", type=int, default=1, choices=(0, 1),
                    help="1: two-level block preconditioner, 0: block-Jacobi")
    ap.add_argument("--counters", action="store_true",
                    help="hardware-counter probe: 5 FP64 Jacobian products of the workload and "
                         "one 1 GiB device copy (calibration), then one FP32-IR preconditioner "
                         "build (matrix-core block inverses), nothing else")
    ap.add_argument("--assembly", type=int, default=0, metavar="N",
                    help="assembly probe: N full assemblies of the workload timed with HIP "
                         "events (after one 1 GiB device copy for counter calibration), nothing else")
    args = ap.parse_args()
    if args.gpus != 1:
        print(f"bench.py: runs on one GPU only (asked for {args.gpus}); sharding over "
              "several GPUs is designed, not implemented", file=sys.stderr)
        sys.exit(2)
    import numpy as np
    import torch
    import paper_1911_10275_amd as hf
    import synth

    prob = synth.config(args.workload)
    if args.counters:
        counters_probe(prob)
        return
    if args.assembly > 0:
        assembly_probe(prob, args.assembly)
        return
    print(f"bench: workload {prob.name}: {prob.n_elem} elements, {prob.n_udof} displacement DOF",
          file=sys.stderr, flush=True)
    stream = torch.cuda.current_stream().cuda_stream
    ctx = hf.context_for_problem(prob, device=0, stream=stream, gmres_m=args.gmres_m,
                                 two_level=args.two_level, coarse_fp32=args.coarse_fp32,
                                 coarse_reuse=args.coarse_reuse)
    sz = ctx.sizes
    N = sz.n_u + sz.n_p

    class St:  # start of the load sequence: the uniform-pressure elastic predictor
        w_old = np.zeros((sz.n_face, sz.nq_face))

    ctx.set_state(np.zeros(sz.n_u), np.full(sz.n_p, prob.material.sigma_c), St.w_old)
    p0 = ctx.initial_guess()
    St.u, St.p, _, _ = ctx.get_state()
    print(f"bench: predictor p0 = {p0:.4e}", file=sys.stderr, flush=True)

    K, W = args.steps, args.warmup
    tuned = {}
    tune_cache = os.path.join(ROOT, "paper_1911_10275_amd", "tuning_cache.txt")

    def tune(name):
        ctx.set_state(St.u, St.p, St.w_old)
        ctx.assemble()
        t0 = time.perf_counter()
        tuned[name] = ctx.autotune(level=args.tune, cache_path=tune_cache).as_dict()
        print(f"bench: {name} tuning {tuned[name]} ({time.perf_counter() - t0:.1f} s, untimed)",
              file=sys.stderr, flush=True)

    tune("fp64")
    dt64, st64, prof, state64 = run_steps(ctx, St, K, W, profile=True)
    iters64 = [s[0] for s in st64]
    for s in st64:
        assert s[2] <= 1e-10, "FP64 solve missed the 1e-10 true residual"
    print(f"bench: fp64 {K} steps in {dt64:.3f} s, GMRES iterations {iters64}", file=sys.stderr,
          flush=True)
    # dominant kernel: the FP64 block-sparse Jacobian product
    bs = sz.block_size
    spmv_bytes = sz.n_blocks * bs * bs * 8 + sz.n_blocks * 4 + (sz.n_elem + 1) * 8 + 2 * N * 8
    spmv_ms = prof.ms_spmv64 / max(prof.n_spmv64, 1)
    asm_ms = prof.ms_assemble / max(prof.n_assemble, 1)
    achieved = spmv_bytes / (spmv_ms * 1e-3) / 1e9
    out = {
        "metric": METRIC,
        "value": K / dt64,
        "unit": "Newton steps/s",
        "n_gpus": 1,
        "steps": K,
        "warmup": W,
        "ms_per_step": 1e3 * dt64 / K,
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f64",
        "data": "synthetic",
        "config": {"workload": prob.name, "elements": int(sz.n_elem), "dof": int(N),
                   "u_dof": int(sz.n_u), "p_dof": int(sz.n_p), "element": f"P{prob.order}",
                   "dim": prob.dim, "precision": "fp64",
                   "preconditioner": ("two-level" + (", coarse factor in FP32" if args.coarse_fp32 else ""))
                   if args.two_level else "block-Jacobi",
                   "gmres_m": tuned.get("fp64", {}).get("gmres_m", args.gmres_m), "rtol": 1e-10},
        "median_step_ms": 1e3 * float(np.median([x[7] for x in st64])),
        "gmres": {"iters_per_step": float(np.mean(iters64)),
                  "iters_per_s": float(sum(iters64) / dt64),
                  "mdof_iters_per_s": float(sum(iters64) * N / dt64 / 1e6)},
        "roofline": {"bound": "hbm", "kernel": "k_bsr_spmv<double,30>", "achieved": achieved,
                     "peak": HBM_PEAK_GBS, "unit": "GB/s", "frac": achieved / HBM_PEAK_GBS,
                     "traffic": spmv_traffic(prob.name), "bytes_per_launch": int(spmv_bytes),
                     "avg_launch_ms": spmv_ms, "launches": int(prof.n_spmv64)},
        # HIP-event times of the launches outside the graph-replayed GMRES chunks
        "kernel_ms_outside_graphs": {"assemble": prof.ms_assemble, "spmv64": prof.ms_spmv64,
                                     "precond": prof.ms_precond, "blockinv": prof.ms_blockinv,
                                     "resid": prof.ms_resid},
        # the timed steps' assemblies are incremental (the context's first, full one ran
        # before timing): the product with the cached blocks (its bytes are a lower bound of
        # the assembly's algorithmic bytes) plus the crack elements and the fluid rows
        "assembly_incremental": {
            "avg_ms": asm_ms, "bytes_lower_bound": int(spmv_bytes),
            "GBps": spmv_bytes / (asm_ms * 1e-3) / 1e9 if asm_ms > 0 else None,
            "frac": spmv_bytes / (asm_ms * 1e-3) / 8e12 if asm_ms > 0 else None,
            "calls": int(prof.n_assemble)},
    }
    if not args.no_ir:
        ctx.set_options(precision=hf.HF_FP32_IR)
        tune("fp32_ir")
        dt32, st32, prof32, state32 = run_steps(ctx, St, K, W, profile=False)
        iters32 = [s[0] for s in st32]
        for s in st32:
            assert s[2] <= 1e-10, "FP32-IR solve missed the 1e-10 true residual"
        u64, p64, w64, _ = state64
        u32, p32, w32, _ = state32
        rel = lambda a, b: float(np.linalg.norm(a - b) / max(np.linalg.norm(b), 1e-300))
        out["fp32_ir"] = {"newton_steps_per_s": K / dt32, "speedup_vs_fp64": dt64 / dt32,
                          "median_step_ms": 1e3 * float(np.median([x[7] for x in st32])),
                          "iters_per_step": float(np.mean(iters32)),
                          "ir_steps_per_step": float(np.mean([s[1] for s in st32])),
                          "fp64_finish_iters_per_step": float(np.mean([s[6] for s in st32])),
                          "mdof_iters_per_s": float(sum(iters32) * N / dt32 / 1e6),
                          "rel_err_vs_fp64": {"u": rel(u32, u64), "p": rel(p32, p64),
                                              "w": rel(w32, w64)}}
        print(f"bench: fp32-ir {K} steps in {dt32:.3f} s, GMRES iterations {iters32}",
              file=sys.stderr, flush=True)
    ctx.close()
    out["tuning"] = tuned
    if not args.no_ensemble:
        out["ensemble"] = ensemble_block(args.ensemble_steps, args.ensemble_m, args.tune, args.two_level)
    if not args.no_cpu:
        print("bench: timing the CPU oracle on a bounded sample", file=sys.stderr, flush=True)
        out["cpu_baseline"] = cpu_baseline(prob, float(np.mean(iters64)))
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
