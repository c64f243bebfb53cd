#!/usr/bin/env python3
"""Benchmark of the synchronous Jacobi sweep on one MI355X.

Workload (one "step"): the 128^3 7-point FP64 Laplacian (n = 2,097,152,
nnz = 14,581,760, b = A x* with x* seeded uniform in [-1,1]) swept 2000 times
from x0 = 0 under each of the three splits of the paper's section 4, 64 parts
each: naive band rows (JB), band rows with sparsity-pattern lists (JBO), and
substructuring on an 8x8x8 subdomain grid grouped into 64 parts (JSS), with the
residual 2-norm of every sweep recorded on the device.

value = algorithmic bytes of all sweeps of the timed steps / their time, with
the lean byte model 12 nnz + 4 (n+1) + 24 n per sweep (values and int32
columns, row pointers, b, x_k read and x_{k+1} written; the diagonal comes
from the row's own values, so no D^{-1} vector is counted: the sweep kernels
read none).  Inputs are resident in HBM before timing starts.  One 128^3
sweep streams about 188 MiB, which the 256 MiB Infinity Cache keeps between
sweeps: the headline is a cache-resident figure.  The HBM-bound control is
the same Laplacian at 192^3 (727 MiB per sweep, matrix streamed) under the
same three splits, reported as roofline_hbm.

Prints one JSON line.  --gpus above 1 is refused: this build runs on one GPU.
"""
from __future__ import annotations

import argparse
import hashlib
import json
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
METRIC = "Jacobi sweep GB/s (% HBM peak) at 128^3 FP64; batched/adjoint/FP32 vs plain"
HBM_PEAK_GBS = 8000.0
BYTE_MODEL = ("lean: 12 nnz + 4 (n+1) + 24 n per sweep (values, int32 columns, row pointers, b and x_k read, "
              "x_k+1 written; the diagonal is read with the row's values, no D^-1 vector)")


def parse():
    ap = argparse.ArgumentParser(description=__doc__, formatter_class=argparse.RawDescriptionHelpFormatter)
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=10)
    ap.add_argument("--warmup", type=int, default=3)
    ap.add_argument("--N", type=int, default=128)
    ap.add_argument("--sweeps", type=int, default=2000)
    ap.add_argument("--modes", default="JB,JBO,JSS")
    ap.add_argument("--no-cpu", action="store_true", help="skip the CPU oracle baseline")
    ap.add_argument("--cpu-seconds", type=float, default=12.0, help="CPU oracle baseline sample length")
    ap.add_argument("--loop", type=int, default=0, help="0 = one launch per sweep, 1 = persistent loop")
    ap.add_argument("--tile-rows", type=int, default=0)
    ap.add_argument("--block", type=int, default=0)
    ap.add_argument("--wg-per-cu", type=int, default=0)
    ap.add_argument("--lds-elems", type=int, default=0)
    ap.add_argument("--no-secondary", action="store_true",
                    help="skip the FP32-refinement, batched and adjoint comparisons")
    ap.add_argument("--no-hbm", action="store_true", help="skip the HBM-bound 192^3 control of the three splits")
    ap.add_argument("--hbm-N", type=int, default=192, help="grid edge of the HBM-bound control")
    ap.add_argument("--hbm-sweeps", type=int, default=200, help="sweeps per timed loop of the HBM-bound control")
    ap.add_argument("--no-persistent", action="store_true",
                    help="skip the batched solve in one persistent (cooperative) launch")
    ap.add_argument("--secondary-legs", default="refine,batched,adjoint,set1,partitions,async,controls",
                    help="comma-separated secondary comparisons to run")
    ap.add_argument("--copy-mib", type=int, default=0,
                    help="only run 5 device-to-device copies of this many MiB (counter calibration) and exit")
    ap.add_argument("--batched-probe", type=int, default=0,
                    help="only run this many lockstep sweeps of the 256-system, 4-column batch (counter "
                         "runs of the batched kernel) and exit")
    return ap.parse_args()


KERNEL_SOURCES = ("kernels.hip", "kernels.h", "launch.h")


def log(msg):
    """Progress on stderr (the JSON line alone goes to stdout)."""
    print(f"[bench {time.strftime('%H:%M:%S')}] {msg}", file=sys.stderr, flush=True)


def src_digest():
    """Digest of the device code: the kernel source and the headers of its
    launch interface (host-only sources do not change what a kernel does)."""
    h = hashlib.sha256()
    for f in KERNEL_SOURCES:
        with open(os.path.join(ROOT, "paper_2112_02377_amd", "csrc", f), "rb") as fh:
            h.update(fh.read())
    return h.hexdigest()[:16]


def traffic_from_profile(kernel_tag, N):
    """HBM-side bytes per launch of a sweep kernel on the N^3 Laplacian
    (FETCH_SIZE and WRITE_SIZE counters scaled by a copy-kernel calibration)
    from the committed counter summary profiles/traffic.json, when it was
    taken on the current kernel sources; else None."""
    path = os.path.join(ROOT, "profiles", "traffic.json")
    if not os.path.exists(path):
        return None
    with open(path) as f:
        t = json.load(f)
    rec = t.get(f"{kernel_tag} @ {N}^3")
    if not rec or rec.get("src_digest") != src_digest():
        return None
    return rec.get("hbm_bytes_per_launch")


def host_cpu():
    """The host's CPU model, its logical CPU count, the CPUs this process may
    run on, and the threads the oracle uses: the affinity set, capped by
    OMP_NUM_THREADS when the machine sets it (a shared host gives each job a
    share of its cores that way)."""
    model = "unknown"
    try:
        with open("/proc/cpuinfo") as f:
            for line in f:
                if line.startswith("model name"):
                    model = line.split(":", 1)[1].strip()
                    break
    except OSError:
        pass
    nproc = os.cpu_count() or 1
    try:
        affinity = len(os.sched_getaffinity(0))
    except AttributeError:
        affinity = nproc
    omp = os.environ.get("OMP_NUM_THREADS", "")
    threads = min(affinity, int(omp)) if omp.isdigit() and int(omp) > 0 else affinity
    return model, nproc, affinity, threads


def cpu_baseline(sysm, seconds, batch16=None):
    """The oracle on the host cores, same byte model as the GPU figure:
    (1) all the threads this process may use, chunks of sweeps of the same
    system, each continuing from the previous chunk's iterate, until about
    `seconds` of CPU work have run; (2) one thread (the parity mode) for a few
    sweeps; (3) the batched workload's seeded 16-system subset, every
    right-hand side solved to 1e-8 with all threads."""
    from oracle import ref
    from paper_2112_02377_amd.workloads import lean_bytes_per_sweep
    model, nproc, affinity, threads = host_cpu()
    bps = lean_bytes_per_sweep(sysm.n, sysm.nnz)
    ref.sweeps(sysm.row_ptr, sysm.col_idx, sysm.vals, sysm.b[0], 2, threads=threads)
    chunk, done, x = 100, 0, None
    t0 = time.perf_counter()
    while True:
        _, x, _ = ref.sweeps(sysm.row_ptr, sysm.col_idx, sysm.vals, sysm.b[0], chunk, x0=x, threads=threads)
        done += chunk
        dt = time.perf_counter() - t0
        if dt >= seconds:
            break
    edge = round(sysm.n ** (1 / 3))
    out = {"value": round(done * bps / dt / 1e9, 3), "unit": "GB/s", "cores": threads, "kind": "oracle",
           "sample": f"{done} sweeps of the same {edge}^3 system from x0 = 0 in chunks of {chunk} "
                     f"(residual norm per sweep), plain C FP64 oracle, {threads} OpenMP threads, {dt:.1f} s; "
                     f"lean byte model",
           "sweeps_per_s": round(done / dt, 3), "cpu_model": model, "nproc": nproc, "affinity_cpus": affinity}
    k1 = 20
    t0 = time.perf_counter()
    ref.sweeps(sysm.row_ptr, sysm.col_idx, sysm.vals, sysm.b[0], k1, threads=1)
    dt = time.perf_counter() - t0
    out["single_thread"] = {"GBps": round(k1 * bps / dt / 1e9, 3), "sweeps_per_s": round(k1 / dt, 3),
                            "sample": f"{k1} sweeps of the {edge}^3 system, 1 thread (parity mode), {dt:.2f} s"}
    if batch16:
        t0 = time.perf_counter()
        sweeps, byts = 0, 0
        for s in batch16:
            for c in range(s.b.shape[0]):
                st, _, k, _ = ref.solve(s.row_ptr, s.col_idx, s.vals, s.b[c], 1e-8, 1000000, threads=threads)
                sweeps += k
                byts += (k + 1) * lean_bytes_per_sweep(s.n, s.nnz)
        dt = time.perf_counter() - t0
        out["batched_subset16"] = {"s": round(dt, 3), "GBps": round(byts / dt / 1e9, 3), "column_sweeps": sweeps,
                                   "sample": f"16 seeded systems of the batched workload (n total "
                                             f"{sum(s.n for s in batch16)}), 4 right-hand sides each solved to "
                                             f"relative 1e-8, {threads} OpenMP threads"}
    return out


def batch_subset16(systems):
    """The seeded 16-system subset of the batched workload that the CPU
    baseline solves (and the parity tests check against the oracle)."""
    import numpy as np
    pick = sorted(np.random.default_rng(2112).choice(len(systems), 16, replace=False).tolist())
    return pick, [systems[i] for i in pick]


def copy_bandwidth(torch, mib=1024, reps=10):
    """Device-to-device copy rate on this GPU (bytes read + written / time):
    the plain-copy reference the sweep's traffic is compared with."""
    a = torch.empty(mib << 17, dtype=torch.float64, device="cuda").fill_(1.0)
    c = torch.empty_like(a)
    for _ in range(3):
        c.copy_(a)
    torch.cuda.synchronize()
    e0 = torch.cuda.Event(enable_timing=True)
    e1 = torch.cuda.Event(enable_timing=True)
    e0.record()
    for _ in range(reps):
        c.copy_(a)
    e1.record()
    torch.cuda.synchronize()
    gbs = reps * 2 * a.numel() * 8 / (e0.elapsed_time(e1) / 1e3) / 1e9
    del a, c
    return round(gbs, 1)


def _timed(torch, stream, fn):
    e0 = torch.cuda.Event(enable_timing=True)
    e1 = torch.cuda.Event(enable_timing=True)
    torch.cuda.synchronize()
    e0.record(stream)
    r = fn()
    e1.record(stream)
    torch.cuda.synchronize()
    return e0.elapsed_time(e1), r


SECONDARY_LEGS = ("refine", "batched", "adjoint", "set1", "partitions", "async", "controls")


def secondary(B, W, torch, stream, with_oracle=True, persistent=True, legs=SECONDARY_LEGS):
    """The comparisons the metric names, each against the plain FP64 sweep on
    the same GPU: FP32 inner sweeps with FP64 refinement (96^3 27-point
    FE-like matrix, to 1e-10), the batched persistent solve (256 diffusion
    systems x 4 right-hand sides, to 1e-8) against 256 separate solves, and
    the adjoint (64^3 diffusion, K = 400, checkpoint every 20) against its
    forward sweeps; then the Q1 FE stand-ins of the paper's Set-1 cubes solved
    with its stop test, beside its iteration counts and CPU-cluster times, the
    weighted partitioners against equal-row bands, the asynchronous
    relaxation against the synchronous solve, and the control configurations
    (20^3 solves, 128^3 with 4x4x4 subdomains).  `legs` selects among them.
    Times are HIP-event times on the handles' stream."""
    out = {}
    if "refine" in legs:
        log("secondary: FP32 refinement")
        out["fp32_refine"] = refine_leg(B, W, torch, stream, with_oracle)
    if "batched" in legs:
        log("secondary: batched")
        out["batched"] = batched_leg(B, W, torch, stream, persistent)
    if "adjoint" in legs:
        log("secondary: adjoint")
        out["adjoint"] = adjoint_leg(B, W, torch, stream)
    if "set1" in legs:
        # the paper's Set-1 cubes (Q1 FE stand-ins) with its stop test
        log("secondary: Set-1 cubes")
        out["paper_set1"] = set1(B, W, torch, stream)
    if "partitions" in legs:
        # weighted partitions against equal-row bands
        log("secondary: partitioners")
        out["partitions"] = partitions(B, W, torch, stream)
    if "async" in legs:
        # asynchronous relaxation against the synchronous solve
        log("secondary: asynchronous")
        out["async"] = async_vs_sync(B, W, torch, stream)
    if "controls" in legs:
        # the small configuration's solves and the 128^3 substructuring control
        log("secondary: controls")
        out["controls"] = controls(B, W, torch, stream)
    return out


def refine_leg(B, W, torch, stream, with_oracle):
    """FP32 inner sweeps under FP64 refinement against the FP64 solve, on the
    96^3 27-point FE-like matrix to relative 1e-10: default inner stop
    parameters, then the autotuner's tile shape and parameters."""
    import numpy as np
    sc = stream.cuda_stream
    s = W.fe27(96, workload=3)
    h = B.jac_create(s.n, s.row_ptr, s.col_idx, s.vals, 1, s.b.reshape(-1), stream=sc)
    B.jac_partition(h, B.JAC_BANDROW, 64)
    info = B.jac_get_info(h)
    res = {}
    for prec, name in ((B.JAC_FP64, "fp64"), (B.JAC_FP32_REFINE, "fp32_refine")):
        B.jac_set_x(h, None)
        B.jac_solve(h, 1e-10, 100000, B.JAC_NORM_L2_REL, prec)      # warm
        B.jac_set_x(h, None)
        ms, (st, sw, rr) = _timed(torch, stream, lambda: B.jac_solve(h, 1e-10, 100000, B.JAC_NORM_L2_REL, prec))
        x = torch.empty(s.n, dtype=torch.float64, device="cuda")
        B.jac_get_x(h, x)
        torch.cuda.synchronize()
        res[name] = dict(ms=round(ms, 3), sweeps=int(sw[0]), relres=float(rr[0]), x=x.cpu().numpy())
    # the autotuner's tile shape and inner stop parameters (tuning not timed)
    B.jac_autotune(h, 20)
    tuned = {"tile_rows": B.jac_get_option(h, B.JAC_OPT_TILE_ROWS), "block": B.jac_get_option(h, B.JAC_OPT_BLOCK),
             "grid": B.jac_get_option(h, B.JAC_OPT_GRID),
             "inner_tol": B.jac_get_option(h, B.JAC_OPT_INNER_TOL) * 1e-9,
             "inner_max": B.jac_get_option(h, B.JAC_OPT_INNER_MAX)}
    for prec, name in ((B.JAC_FP64, "fp64_tuned"), (B.JAC_FP32_REFINE, "fp32_refine_tuned")):
        B.jac_set_x(h, None)
        B.jac_solve(h, 1e-10, 100000, B.JAC_NORM_L2_REL, prec)      # warm
        B.jac_set_x(h, None)
        ms, (st, sw, rr) = _timed(torch, stream, lambda: B.jac_solve(h, 1e-10, 100000, B.JAC_NORM_L2_REL, prec))
        x = torch.empty(s.n, dtype=torch.float64, device="cuda")
        B.jac_get_x(h, x)
        torch.cuda.synchronize()
        res[name] = dict(ms=round(ms, 3), sweeps=int(sw[0]), relres=float(rr[0]), x=x.cpu().numpy())
    bytes64 = W.lean_bytes_per_sweep(s.n, s.nnz)
    bytes32 = 8 * info["nnz"] + 4 * (s.n + 1) + 16 * s.n
    ref_err = None
    if with_oracle:
        from oracle import ref
        st, xo, ko, rro = ref.refine_reference(s.row_ptr, s.col_idx, s.vals, s.b[0], 1e-10,
                                               threads=min(16, os.cpu_count() or 1))
        scale = float(abs(xo).max())
        ref_err = {k: float(abs(v["x"] - xo).max() / scale) for k, v in res.items()}
        ref_err["oracle_sweeps"] = int(ko)
    out = {
        "workload": f"fe27 96^3 (n={s.n}, nnz={s.nnz}), 1.05-dominant, tol 1e-10, 64 bands",
        "fp64_matrix_loads": "kept" if info["keep_matrix"] else "streamed",
        "fp64_ms": res["fp64"]["ms"], "fp64_sweeps": res["fp64"]["sweeps"], "fp64_relres": res["fp64"]["relres"],
        "refine_ms": res["fp32_refine"]["ms"], "refine_inner_sweeps": res["fp32_refine"]["sweeps"],
        "refine_relres": res["fp32_refine"]["relres"],
        "speedup_vs_fp64": round(res["fp64"]["ms"] / res["fp32_refine"]["ms"], 3),
        "fp64_GBps": round(res["fp64"]["sweeps"] * bytes64 / res["fp64"]["ms"] / 1e6, 1),
        "inner_GBps_fp32_model": round(res["fp32_refine"]["sweeps"] * bytes32 / res["fp32_refine"]["ms"] / 1e6, 1),
        "tuned": dict(tuned, fp64_ms=res["fp64_tuned"]["ms"], refine_ms=res["fp32_refine_tuned"]["ms"],
                      refine_inner_sweeps=res["fp32_refine_tuned"]["sweeps"],
                      refine_relres=res["fp32_refine_tuned"]["relres"],
                      speedup_vs_fp64=round(res["fp64_tuned"]["ms"] / res["fp32_refine_tuned"]["ms"], 3)),
        "default_inner": {"inner_tol": 1e-5, "inner_max": 256},
        "byte_model": "FP64 sweep: lean (12 nnz + 4 (n+1) + 24 n); FP32 inner sweep: 8 nnz + 4 (n+1) + 16 n",
        "max_rel_err_vs_fp64_oracle": ref_err}
    B.jac_destroy(h)
    return out


def batched_leg(B, W, torch, stream, persistent):
    """256 diffusion systems x 4 right-hand sides to relative 1e-8: batched
    (per-sweep launches, default and tuned tiles; one persistent launch)
    against 256 separate solves, and the seeded 16-system subset."""
    import numpy as np
    sc = stream.cuda_stream
    systems = W.diffusion_batch(256, workload=4)
    hs = [B.jac_create(x.n, x.row_ptr, x.col_idx, x.vals, 4, x.b.reshape(-1), stream=sc) for x in systems]
    # 256 separate solves and the batched solve, both on the default tile
    # shape (identical arithmetic: equal sweep counts)
    def seq():
        return [B.jac_solve(hh, 1e-8, 1000000) for hh in hs]
    ms_s, rs = _timed(torch, stream, seq)
    for hh in hs:
        B.jac_set_x(hh, None)
    ms_d, (st, swd, rrd) = _timed(torch, stream, lambda: B.jac_solve_batched(hs, 1e-8, 1000000))
    same = all(int((swd[i, :4] != r[1]).sum()) == 0 for i, r in enumerate(rs))
    # then one tile shape for the whole batch from the batched autotuner
    # (not timed), persistent launch, and the default one launch per sweep
    for hh in hs:
        B.jac_set_x(hh, None)
    t0 = time.perf_counter()
    B.jac_autotune_batched(hs, 32)
    t_tune = time.perf_counter() - t0
    shape = (B.jac_get_option(hs[0], B.JAC_OPT_TILE_ROWS), B.jac_get_option(hs[0], B.JAC_OPT_BLOCK))
    ms_p, swp = None, None
    if persistent:
        B.jac_set_option(hs[0], B.JAC_OPT_LOOP, 1)
        ms_p, (st, swp, rrp) = _timed(torch, stream, lambda: B.jac_solve_batched(hs, 1e-8, 1000000))
        B.jac_set_option(hs[0], B.JAC_OPT_LOOP, 0)
    for hh in hs:
        B.jac_set_x(hh, None)
    ms_b, (st, swb, rrb) = _timed(torch, stream, lambda: B.jac_solve_batched(hs, 1e-8, 1000000))
    # the seeded 16-system subset the CPU baseline solves
    pick, _ = batch_subset16(systems)
    sub = [hs[i] for i in pick]
    for hh in sub:
        B.jac_set_x(hh, None)
    ms_16, _ = _timed(torch, stream, lambda: B.jac_solve_batched(sub, 1e-8, 1000000))
    alg = 0
    for x, k in zip(systems, swb):
        alg += W.lean_bytes_per_sweep(x.n, x.nnz, 4) * (int(k[:4].max()) + 1)
    out = {
        "workload": f"256 diffusion systems, edges U[16,64], n total {sum(x.n for x in systems)}, 4 rhs, tol 1e-8",
        "batched_ms": round(ms_b, 3), "persistent_ms": None if ms_p is None else round(ms_p, 3),
        "sequential_ms": round(ms_s, 3), "batched_default_tiles_ms": round(ms_d, 3),
        "subset16_batched_ms": round(ms_16, 3), "subset16_systems": pick,
        "speedup_vs_sequential": round(ms_s / ms_b, 3), "max_sweeps": int(swb[:, :4].max()),
        "sum_system_sweeps": int(swb[:, :4].max(axis=1).sum()),
        "byte_model": "lean, 4 right-hand sides: 12 nnz + 4 (n+1) + 96 n per system sweep",
        "batched_alg_GBps": round(alg / ms_b / 1e6, 1),
        "persistent_alg_GBps": None if ms_p is None else round(alg / ms_p / 1e6, 1),
        "sequential_alg_GBps": round(alg / ms_s / 1e6, 1),
        "sweep_counts_equal_to_separate_solves": bool(same),
        "tuned_vs_default_max_sweep_diff": int(np.abs(swb[:, :4] - swd[:, :4]).max()),
        "persistent_equals_per_sweep_launches": None if swp is None else bool(np.array_equal(swb, swp)),
        "tuned_tile_rows": int(shape[0]), "tuned_block": int(shape[1]), "tune_s": round(t_tune, 2),
        "note": "separate solves use the default tile shape (512 rows), the tuned batch the shape "
                "jac_autotune_batched picked for the batch"}
    for hh in hs:
        B.jac_destroy(hh)
    return out


def adjoint_leg(B, W, torch, stream):
    """The adjoint of 400 sweeps at 64^3 (checkpoint every 20) against its
    forward sweeps: all iterates stored, checkpoints reused from the
    forward, and checkpoints every 20 with recomputed segments."""
    sc = stream.cuda_stream
    s = W.diffusion_adjoint(64, workload=5)
    h = B.jac_create(s.n, s.row_ptr, s.col_idx, s.vals, 1, s.b.reshape(-1), stream=sc)
    gx = torch.from_numpy(s.extra["x_target"]).cuda()
    gb = torch.empty_like(gx)
    gv = torch.empty(s.nnz, dtype=torch.float64, device="cuda")
    B.jac_set_x(h, None)
    B.jac_sweep(h, 400)
    B.jac_set_x(h, None)
    ms_f, _ = _timed(torch, stream, lambda: B.jac_sweep(h, 400))
    # the adjoint on its own (it takes its checkpoints itself)
    B.jac_adjoint(h, 400, 20, gx, gb, gv)
    B.jac_set_x(h, None)                                       # invalidates the checkpoints
    ms_a, _ = _timed(torch, stream, lambda: B.jac_adjoint(h, 400, 20, gx, gb, gv))
    # forward that keeps its checkpoints, then the reverse pass reusing them
    # (what the autograd Function does)
    ms_fc, _ = _timed(torch, stream, lambda: B.jac_sweep_checkpointed(h, 400, 20))
    ms_r, _ = _timed(torch, stream, lambda: B.jac_adjoint(h, 400, 20, gx, gb, gv))
    fb = W.lean_bytes_per_sweep(s.n, s.nnz)
    # the same adjoint with checkpoints every 20 sweeps and recomputed
    # segments (a 200 MiB cap leaves no room for all 401 iterates)
    B.jac_set_option(h, B.JAC_OPT_CKPT_MEM_MB, 200)
    B.jac_set_x(h, None)
    B.jac_adjoint(h, 400, 20, gx, gb, gv)
    B.jac_set_x(h, None)
    ms_rc, _ = _timed(torch, stream, lambda: B.jac_adjoint(h, 400, 20, gx, gb, gv))
    out = {"workload": "diffusion 64^3, K = 400 sweeps, reverse segments of 20; all 401 iterates "
                                  "stored (841 MB, within the default 4 GiB cap)", "forward_ms": round(ms_f, 3),
                      "adjoint_ms": round(ms_a, 3), "adjoint_over_forward": round(ms_a / ms_f, 3),
                      "forward_checkpointed_ms": round(ms_fc, 3), "reverse_reusing_checkpoints_ms": round(ms_r, 3),
                      "forward_plus_backward_over_forward": round((ms_fc + ms_r) / ms_f, 3),
                      "adjoint_checkpoint_every_20_ms": round(ms_rc, 3),
                      "adjoint_checkpoint_every_20_over_forward": round(ms_rc / ms_f, 3),
                      "forward_GBps": round(400 * fb / ms_f / 1e6, 1)}
    B.jac_destroy(h)
    return out


def controls(B, W, torch, stream):
    """The 20^3 Laplacian solved to relative 1e-8 under each split (4 parts;
    substructuring on 2x2x1 blocks) and the 128^3 substructuring with one
    subdomain per part (4x4x4 subdomains of 32^3, 64 parts)."""
    sc = stream.cuda_stream
    res = {}
    s = W.laplace7(20, workload=1)
    h = B.jac_create(s.n, s.row_ptr, s.col_idx, s.vals, 1, s.b.reshape(-1), stream=sc)
    B.jac_set_grid(h, 20, 20, 20)
    c1 = {}
    for name, mode, sub in (("JB", B.JAC_BANDROW, None), ("JBO", B.JAC_BANDROW_SP, None),
                            ("JSS", B.JAC_SUBSTRUCT, (2, 2, 1))):
        B.jac_partition(h, mode, 4, sub)
        B.jac_set_x(h, None)
        B.jac_solve(h, 1e-8, 5000)
        B.jac_set_x(h, None)
        ms, (st, sw, rr) = _timed(torch, stream, lambda: B.jac_solve(h, 1e-8, 5000))
        c1[name] = {"sweeps": int(sw[0]), "ms": round(ms, 3), "relres": float(rr[0]),
                    "sweeps_per_s": round(int(sw[0]) / (ms / 1e3), 1)}
    B.jac_destroy(h)
    res["laplace7_20_solve"] = c1
    for name, N, mode, P, sub, K in (("laplace7_128_jss_4x4x4", 128, B.JAC_SUBSTRUCT, 64, (4, 4, 4), 500),):
        s = W.laplace7(N, workload=2)
        h = B.jac_create(s.n, s.row_ptr, s.col_idx, s.vals, 1, s.b.reshape(-1), stream=sc)
        B.jac_set_grid(h, N, N, N)
        B.jac_partition(h, mode, P, sub)
        B.jac_set_option(h, B.JAC_OPT_TIMING, 1)
        B.jac_set_x(h, None)
        B.jac_sweep(h, 20)
        B.jac_sweep(h, K)
        info = B.jac_get_info(h)
        us = info["last_loop_ms"] * 1e3 / K
        lb = W.lean_bytes_per_sweep(s.n, s.nnz)
        res[name] = {"us_per_sweep": round(us, 3), "GBps": round(lb / us / 1e3, 1),
                     "pct_hbm_peak": round(100 * lb / us / 1e3 / HBM_PEAK_GBS, 2),
                     "halo_entries": int(info["halo_entries"]), "col_bytes": int(info["col_bytes"]), "n": s.n,
                     "nnz": s.nnz, "matrix_loads": "kept" if info["keep_matrix"] else "streamed"}
        B.jac_destroy(h)
    return res


def async_vs_sync(B, W, torch, stream):
    """Time to solution and passes of the asynchronous relaxation (16 and 64
    passes per launch between stop tests) against the synchronous solve's
    sweeps, from x_0 = 0, on the 20^3 Laplacian (relative 2-norm 1e-8), the
    Set-1 cubes (the paper's absolute infinity-norm test) and the 64^3
    diffusion system (relative 2-norm 1e-8)."""
    sc = stream.cuda_stream
    cases = [("laplace7_20", W.laplace7(20, workload=1), B.JAC_BANDROW_SP, 4, None, B.JAC_NORM_L2_REL),
             ("q1_cube_33", W.fe_q1_cube(33), B.JAC_SUBSTRUCT, 8, (2, 2, 2), B.JAC_NORM_INF_ABS),
             ("q1_cube_65", W.fe_q1_cube(65), B.JAC_BANDROW_SP, 64, None, B.JAC_NORM_INF_ABS),
             ("diffusion_64", W.diffusion_adjoint(64, workload=5), B.JAC_BANDROW_SP, 64, None, B.JAC_NORM_L2_REL)]
    res = {}
    for name, s, mode, P, sub, norm in cases:
        h = B.jac_create(s.n, s.row_ptr, s.col_idx, s.vals, 1, s.b.reshape(-1), stream=sc)
        B.jac_set_grid(h, *s.grid)
        B.jac_partition(h, mode, P, sub)
        B.jac_set_x(h, None)
        B.jac_solve(h, 1e-8, 1000000, norm)                          # warm
        B.jac_set_x(h, None)
        ms, (st, sw, rr) = _timed(torch, stream, lambda: B.jac_solve(h, 1e-8, 1000000, norm))
        r = {"sync": {"sweeps": int(sw[0]), "ms": round(ms, 3), "res": float(rr[0])}}
        for R in (16, 64):
            B.jac_set_x(h, None)
            B.jac_solve_async(h, 1e-8, 1000000, norm, R)            # warm
            B.jac_set_x(h, None)
            ms, (st, rd, rr) = _timed(torch, stream, lambda: B.jac_solve_async(h, 1e-8, 1000000, norm, R))
            r[f"async_R{R}"] = {"passes": int(rd[0]), "ms": round(ms, 3), "res": float(rr[0]),
                                "passes_over_sweeps": round(int(rd[0]) / max(int(sw[0]), 1), 3),
                                "speedup_vs_sync": round(r["sync"]["ms"] / ms, 3)}
        res[name] = r
        B.jac_destroy(h)
    return res


def partitions(B, W, torch, stream):
    """Equal-row bands against nnz-weighted bands and the weighted graph
    partition (section 4.2.2's load-balanced split): receive-list volume (the
    per-sweep exchange of a multi-device run), stored-entry imbalance, host
    partitioning time, and the one-GPU sweep time of the sparsity-pattern
    band-row split on each (64 parts; 128^3 Laplacian and the 96^3 27-point
    matrix)."""
    import numpy as np
    sc = stream.cuda_stream
    res = {}
    for name, s, K in (("laplace7_128", W.laplace7(128, workload=2), 500), ("fe27_96", W.fe27(96, workload=3), 300)):
        h = B.jac_create(s.n, s.row_ptr, s.col_idx, s.vals, 1, s.b.reshape(-1), stream=sc)
        nnz_row = np.diff(s.row_ptr)
        r = {}
        for label, part in (("equal_rows", B.PART_ROWS), ("equal_nnz", B.PART_NNZ), ("graph", B.PART_GRAPH)):
            B.jac_set_option(h, B.JAC_OPT_PARTITIONER, part)
            t0 = time.perf_counter()
            B.jac_partition(h, B.JAC_BANDROW_SP, 64)
            t_part = time.perf_counter() - t0
            got = B.jac_get_partition(h)
            owner = np.zeros(s.n, dtype=np.int64)
            owner[got["perm"]] = np.searchsorted(got["bounds"], np.arange(s.n), side="right") - 1
            w = np.bincount(owner, weights=nnz_row, minlength=64)
            B.jac_set_option(h, B.JAC_OPT_TIMING, 1)
            B.jac_set_x(h, None)
            B.jac_sweep(h, 20)
            B.jac_sweep(h, K)
            info = B.jac_get_info(h)
            B.jac_set_option(h, B.JAC_OPT_TIMING, 0)
            r[label] = {"halo_entries": int(info["halo_entries"]), "nnz_imbalance": round(float(w.max() / w.mean()), 4),
                        "partition_s": round(t_part, 2),
                        "us_per_sweep": round(info["last_loop_ms"] * 1e3 / K, 3)}
        r["n"], r["nnz"] = s.n, s.nnz
        res[name] = r
        B.jac_destroy(h)
    return res


# The paper's p = 1 iteration count and solver time, and its p = 64 solver
# times per splitting (Xeon E5410 cores over Ethernet; results tables of
# section 6), quoted as context beside the one-GPU times.
PAPER_SET1 = {33: dict(name="luf_cube-35937", iters=746, p1_s=10.9, p64_s={"JB": 734.7, "JBO": 2.1, "JSS": 2.4}),
              65: dict(name="luf_cube-274625", iters=2216, p1_s=238.4,
                       p64_s={"JB": 7058.6, "JBO": 28.0, "JSS": 23.0})}


def set1(B, W, torch, stream):
    """Time to solution on the Q1 FE cubes under the paper's stop test
    (absolute infinity norm of the residual below 1e-8, from x_0 = 0), 64
    parts per splitting; iterations counted as the paper does (the final
    iterate included)."""
    sc = stream.cuda_stream
    res = {}
    for N, sub in ((33, (4, 4, 4)), (65, (4, 4, 4))):
        s = W.fe_q1_cube(N)
        h = B.jac_create(s.n, s.row_ptr, s.col_idx, s.vals, 1, s.b.reshape(-1), stream=sc)
        B.jac_set_grid(h, N, N, N)
        info = None
        r = {"paper": PAPER_SET1[N]}
        for name, mode, sg in (("JB", B.JAC_BANDROW, None), ("JBO", B.JAC_BANDROW_SP, None),
                               ("JSS", B.JAC_SUBSTRUCT, sub)):
            # default tile shape, then the autotuner's pick (tuning not timed)
            B.jac_set_option(h, B.JAC_OPT_TILE_ROWS, 512)
            B.jac_set_option(h, B.JAC_OPT_BLOCK, 256)
            B.jac_set_option(h, B.JAC_OPT_GRID, 0)
            B.jac_partition(h, mode, 64, sg)
            for tuned in (False, True):
                if tuned:
                    B.jac_autotune(h, 100)
                info = B.jac_get_info(h)
                B.jac_set_x(h, None)
                B.jac_solve(h, 1e-8, 100000, B.JAC_NORM_INF_ABS)          # warm
                B.jac_set_x(h, None)
                ms, (st, sw, rr) = _timed(torch, stream, lambda: B.jac_solve(h, 1e-8, 100000, B.JAC_NORM_INF_ABS))
                e = {"iters": int(sw[0]) + 1, "ms": round(ms, 3), "final_res_inf": float(rr[0]),
                     "GBps": round((int(sw[0]) + 1) * W.lean_bytes_per_sweep(s.n, s.nnz) / ms / 1e6, 1),
                     "tile_rows": B.jac_get_option(h, B.JAC_OPT_TILE_ROWS),
                     "block": B.jac_get_option(h, B.JAC_OPT_BLOCK), "grid": B.jac_get_option(h, B.JAC_OPT_GRID)}
                if tuned:
                    r[name]["tuned"] = e
                else:
                    r[name] = e
        r["n"], r["nnz"] = s.n, s.nnz
        res[PAPER_SET1[N]["name"] + "_standin"] = r
        B.jac_destroy(h)
    return res


MODES = {"JB": (1, 64, None), "JBO": (2, 64, None), "JSS": (3, 64, (8, 8, 8))}


def make_handles(B, s, N, sel, stream, args):
    handles, infos, setup_s = {}, {}, {}
    for m in sel:
        mode, P, sub = MODES[m]
        t0 = time.perf_counter()
        h = B.jac_create(s.n, s.row_ptr, s.col_idx, s.vals, 1, s.b.reshape(-1), stream=stream.cuda_stream)
        B.jac_set_option(h, B.JAC_OPT_LOOP, args.loop)
        if args.tile_rows:
            B.jac_set_option(h, B.JAC_OPT_TILE_ROWS, args.tile_rows)
        if args.block:
            B.jac_set_option(h, B.JAC_OPT_BLOCK, args.block)
        if args.wg_per_cu:
            B.jac_set_option(h, B.JAC_OPT_WG_PER_CU, args.wg_per_cu)
        if args.lds_elems:
            B.jac_set_option(h, B.JAC_OPT_LDS_ELEMS, args.lds_elems)
        B.jac_set_grid(h, N, N, N)
        B.jac_partition(h, mode, P, sub)
        B.jac_set_option(h, B.JAC_OPT_TIMING, 1)
        setup_s[m] = time.perf_counter() - t0
        handles[m] = h
        infos[m] = B.jac_get_info(h)
    return handles, infos, setup_s


def run_steps(B, torch, stream, handles, sel, K, steps, warmup):
    """`warmup` untimed then `steps` timed steps; a step sweeps every split K
    times from x0 = 0 with the residual norm of each sweep recorded.  Returns
    (total ms by HIP events on the handles' stream, per-split loop ms of each
    timed step, wall s)."""
    hist = torch.zeros(K, dtype=torch.float64, device="cuda")
    loop_ms = {m: [] for m in sel}

    def step(record):
        for m in sel:
            B.jac_set_x(handles[m], None)
            B.jac_sweep(handles[m], K, hist)
            if record:
                loop_ms[m].append(B.jac_get_info(handles[m])["last_loop_ms"])

    with torch.cuda.stream(stream):
        for _ in range(warmup):
            step(False)
        torch.cuda.synchronize()
        e0 = torch.cuda.Event(enable_timing=True)
        e1 = torch.cuda.Event(enable_timing=True)
        t0 = time.perf_counter()
        e0.record(stream)
        for _ in range(steps):
            step(True)
        e1.record(stream)
        torch.cuda.synchronize()
        wall = time.perf_counter() - t0
    return e0.elapsed_time(e1), loop_ms, wall


def split_report(W, B, s, N, sel, infos, loop_ms, setup_s, K, loop):
    """Per-split figures and the roofline of every sweep kernel of the step,
    the dominant one (most time per step) first.  One launch is one sweep."""
    lean = W.lean_bytes_per_sweep(s.n, s.nnz)
    per_mode = {}
    for m in sel:
        avg = sum(loop_ms[m]) / len(loop_ms[m])
        gbs = lean * K / (avg / 1e3) / 1e9
        i = infos[m]
        med = sorted(loop_ms[m])[len(loop_ms[m]) // 2]
        per_mode[m] = {"loop_ms": round(avg, 3), "loop_ms_median": round(med, 3), "us_per_sweep": round(avg * 1e3 / K, 3),
                       "sweeps_per_s": round(K / (avg / 1e3), 1), "GBps": round(gbs, 1),
                       "pct_hbm_peak": round(100 * gbs / HBM_PEAK_GBS, 2),
                       "csr_model_GBps": round(i["alg_bytes_per_sweep"] * K / (avg / 1e3) / 1e9, 1),
                       "dev_GBps": round(i["dev_bytes_per_sweep"] * K / (avg / 1e3) / 1e9, 1),
                       "dev_bytes_per_sweep": i["dev_bytes_per_sweep"],
                       "col_bytes": i["col_bytes"], "col_format": i["col_format"], "halo_entries": i["halo_entries"],
                       "staged_entries": i["staged_entries"], "ntiles": i["ntiles"], "grid": i["loop_grid"],
                       "matrix_loads": "kept" if i["keep_matrix"] else "streamed", "setup_s": round(setup_s[m], 2)}
    kern = {}
    for m in sel:
        kname = "k_loop" if loop else "k_sweep"
        cm = infos[m]["col_format"]
        nt = "false" if infos[m]["keep_matrix"] else "true"       # nontemporal matrix loads
        kern.setdefault(f"{kname}<double, 1, {cm}, {nt}>", []).append(m)
    order = sorted(kern, key=lambda t: -sum(per_mode[m]["loop_ms"] for m in kern[t]))
    rows = []
    for t in order:
        ms_l = sum(per_mode[m]["loop_ms"] for m in kern[t]) / len(kern[t]) / K
        rows.append({"kernel": t, "modes": kern[t], "avg_launch_ms": round(ms_l, 5), "alg_bytes_per_launch": lean,
                     "achieved": round(lean / (ms_l / 1e3) / 1e9, 1),
                     "frac": round(lean / (ms_l / 1e3) / 1e9 / HBM_PEAK_GBS, 4),
                     "traffic": traffic_from_profile(t, N)})
    dom = rows[0]
    roof = {"bound": "hbm", "achieved": dom["achieved"], "peak": HBM_PEAK_GBS, "unit": "GB/s", "frac": dom["frac"],
            "traffic": dom["traffic"], "kernel": dom["kernel"], "modes": dom["modes"],
            "alg_bytes_per_launch": lean, "avg_launch_ms": dom["avg_launch_ms"], "model": BYTE_MODEL,
            "kernels": rows}
    return per_mode, roof


def hbm_bound(B, W, torch, stream, args):
    """The three splits on the N^3 Laplacian (default 192^3: 727 MiB per
    sweep, more than the Infinity Cache holds, so the matrix is streamed from
    HBM every sweep), 64 parts each (substructuring: 8x8x8 subdomains of
    24^3), timed like the headline with fewer sweeps."""
    N, K = args.hbm_N, args.hbm_sweeps
    s = W.laplace7(N, workload=2)
    sel = list(MODES)
    handles, infos, setup_s = make_handles(B, s, N, sel, stream, args)
    _, loop_ms, _ = run_steps(B, torch, stream, handles, sel, K, 3, 1)
    per_mode, roof = split_report(W, B, s, N, sel, infos, loop_ms, setup_s, K, args.loop)
    for h in handles.values():
        B.jac_destroy(h)
    roof["workload"] = (f"laplace7 {N}^3 FP64 (n={s.n}, nnz={s.nnz}), {K} sweeps x (JB+JBO+JSS), 64 parts each "
                        f"(JSS: 8x8x8 subdomains)")
    roof["regime"] = (f"HBM-bound: one sweep streams {per_mode['JB']['dev_bytes_per_sweep'] / 2**20:.0f} MiB or more, "
                      f"above the 256 MiB Infinity Cache; matrix loads nontemporal")
    return per_mode, roof


def main():
    args = parse()
    if args.gpus != 1:
        print(f"bench.py runs on one GPU only (asked for --gpus {args.gpus}); this build has no multi-GPU path",
              file=sys.stderr)
        sys.exit(2)
    import torch
    if args.copy_mib:
        a = torch.empty(args.copy_mib << 17, dtype=torch.float64, device="cuda").fill_(1.0)
        c = torch.empty_like(a)
        torch.cuda.synchronize()
        for _ in range(5):
            c.copy_(a)
        torch.cuda.synchronize()
        print(json.dumps({"copy_mib": args.copy_mib, "bytes_read_per_copy": a.numel() * 8,
                          "bytes_written_per_copy": a.numel() * 8}), flush=True)
        return
    from paper_2112_02377_amd import binding as B
    from paper_2112_02377_amd import workloads as W

    if args.batched_probe:
        systems = W.diffusion_batch(256, workload=4)
        hs = [B.jac_create(x.n, x.row_ptr, x.col_idx, x.vals, 4, x.b.reshape(-1)) for x in systems]
        # tolerance 0: every column runs the given sweeps (plus the last test)
        B.jac_solve_batched(hs, 0.0, args.batched_probe)
        torch.cuda.synchronize()
        for h in hs:
            B.jac_destroy(h)
        print(json.dumps({"batched_probe_sweeps": args.batched_probe, "systems": len(systems),
                          "rows": sum(x.n for x in systems),
                          "lean_bytes_per_full_sweep": sum(W.lean_bytes_per_sweep(x.n, x.nnz, 4) for x in systems)}),
              flush=True)
        return

    N, K = args.N, args.sweeps
    s = W.laplace7(N, workload=2)
    stream = torch.cuda.Stream()
    sel = [m for m in args.modes.split(",") if m]
    handles, infos, setup_s = make_handles(B, s, N, sel, stream, args)
    torch.cuda.synchronize()
    log(f"{N}^3 splits {sel} set up; timing {args.steps} steps of {K} sweeps each")
    ms_total, loop_ms, wall = run_steps(B, torch, stream, handles, sel, K, args.steps, args.warmup)
    log(f"timed steps done: {ms_total / args.steps:.3f} ms per step")
    lean = W.lean_bytes_per_sweep(s.n, s.nnz)
    total_bytes = args.steps * K * lean * len(sel)
    value = total_bytes / (ms_total / 1e3) / 1e9
    for m in sel:
        infos[m] = B.jac_get_info(handles[m])
    per_mode, roof = split_report(W, B, s, N, sel, infos, loop_ms, setup_s, K, args.loop)
    stream_mib = max(per_mode[m]["dev_bytes_per_sweep"] for m in sel) / 2**20
    roof["regime"] = (f"Infinity-Cache-resident: one sweep streams at most {stream_mib:.0f} MiB, which the 256 MiB "
                      f"Infinity Cache keeps between sweeps (matrix loads temporal); see roofline_hbm for the "
                      f"HBM-bound control")
    csr_bytes = args.steps * K * sum(infos[m]["alg_bytes_per_sweep"] for m in sel)
    out = {"metric": METRIC, "value": round(value, 1), "unit": "GB/s", "n_gpus": 1, "steps": args.steps,
           "warmup": args.warmup, "ms_per_step": round(ms_total / args.steps, 3), "higher_is_better": True,
           "scaling": "weak", "vs_baseline": None, "dtype": "f64", "data": "synthetic",
           "config": {"workload": f"laplace7 {N}^3 FP64, {K} sweeps x ({'+'.join(sel)}), 64 parts each "
                                  f"(JSS: 8x8x8 subdomains)", "n": s.n, "nnz": s.nnz, "sweeps": K,
                      "parallelism": "1 GPU", "pct_hbm_peak": round(100 * value / HBM_PEAK_GBS, 2),
                      "byte_model": BYTE_MODEL,
                      "csr_model_GBps": round(csr_bytes / (ms_total / 1e3) / 1e9, 1)},
           "roofline": roof, "modes": per_mode, "wall_s": round(wall, 3)}
    for h in handles.values():
        B.jac_destroy(h)
    if not args.no_hbm:
        log(f"HBM-bound control {args.hbm_N}^3")
        out["hbm_modes"], out["roofline_hbm"] = hbm_bound(B, W, torch, stream, args)
        log("HBM-bound control done")
    # the traffic the kernels stream (dev_GBps) beside a plain device copy's rate
    out["copy_GBps"] = copy_bandwidth(torch)
    for m in sel:
        per_mode[m]["pct_of_copy"] = round(100 * per_mode[m]["dev_GBps"] / out["copy_GBps"], 1)
    if not args.no_cpu:
        log("CPU oracle baseline")
        _, sub16 = batch_subset16(W.diffusion_batch(256, workload=4))
        out["cpu_baseline"] = cpu_baseline(s, args.cpu_seconds, sub16)
        log("CPU oracle baseline done")
    if not args.no_secondary:
        legs = [x for x in args.secondary_legs.split(",") if x]
        bad = [x for x in legs if x not in SECONDARY_LEGS]
        if bad:
            print(f"unknown secondary legs {bad}; known: {','.join(SECONDARY_LEGS)}", file=sys.stderr)
            sys.exit(2)
        out["secondary"] = secondary(B, W, torch, stream, with_oracle=not args.no_cpu,
                                     persistent=not args.no_persistent, legs=legs)
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
