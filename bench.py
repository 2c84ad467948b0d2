"""Benchmark: FP64 tiled Householder QR of one 8192 x 8192 matrix on one GPU.

Workload: A with entries i.i.d. uniform(-1, 1) (numpy PCG64, seed 0),
nb = 256, ib = 32, the DAG scheduler.  One step = one call of
tileqr_factor_ex on the device-resident matrix (layout conversion in, the
persistent factorisation kernel, layout conversion out); the matrix is
restored from a pristine device copy before each step, outside the timed
stages.  Rate: LAPACK operation count 2mn^2 - 2n^3/3 over the summed device
time of the stages, as the paper reports its rates (Section 5).

Beside the headline, the same line carries two further measurements (skip
them with --no-extras):
  "mixed_ls"  least squares with A 65536 x 1024 (A = U diag(s) V^T, s
              log-spaced to 1/kappa, kappa 1e6, b = A x + 1e-6 noise, seed 0):
              time to solution of the FP64 path (factor + solve) and of the
              split-MFMA paths (factor + solve + refinement until the backward
              error is <= 1e-14), each with its backward error;
  "mixed_ls_square"  the same comparison on a 32768 x 32768 system with 16
              right-hand sides (kappa 1e6; Hadamard-based orthogonal factors
              generated on the GPU);
  "batched"   4000 FP64 matrices, m ~ U{32..768}, n ~ U{16..m}, N(0,1), seed 0,
              in one call of tileqr_factor_batched (blocking and schedule from
              tileqr_tune, run beforehand; the captured graph replayed).

Prints one JSON line.  Flags: --gpus N (only 1 is supported: the build runs
on one GPU), --steps K, --warmup W, --no-cpu-baseline, --no-extras,
--extras LIST (a comma-separated subset of mixed_ls, mixed_ls_square,
batched; default all three).
"""
import argparse
import json
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)

FP64_PEAK_TFLOPS = 78.6      # MI355X FP64 (vector and matrix), spec sheet
PROFILE = os.path.join(ROOT, "profiles", "k_worker_qr8192_fp64.md")
# Sources the worker kernel is compiled from (the traffic figures of the
# profile are valid only for the build whose hash they record).
KERNEL_SRCS = [os.path.join(ROOT, "paper_0709_1272_amd", "csrc", f)
               for f in ("tileqr_kernels.hip", "tileqr_tile.h", "tileqr_dag.h", "tileqr_internal.h")]


def kernel_hash():
    import hashlib
    h = hashlib.sha256()
    for f in KERNEL_SRCS:
        h.update(open(f, "rb").read())
    return h.hexdigest()
M = N = 8192
NB, IB = 256, 32
CPU_SAMPLE_N = 3072


def measured_traffic():
    """HBM bytes per launch of the worker kernel from the committed rocprofv3
    counter summary (FETCH_SIZE + WRITE_SIZE, calibrated on a plain copy), or
    None when the kernel source changed since the counters were taken."""
    import re
    try:
        text = open(PROFILE).read()
    except OSError:
        return None
    if kernel_hash() not in text:
        return None
    m = re.search(r"traffic_bytes_per_launch:\s*([0-9.eE+-]+)", text)
    return float(m.group(1)) if m else None


def cpu_baseline():
    """The oracle (unblocked Householder, 1 thread) on a bounded sample of the
    same workload: a 3072 x 3072 uniform(-1,1) matrix, seed 0."""
    import numpy as np
    import oracle
    from paper_0709_1272_amd import synth
    A = synth.uniform(0, CPU_SAMPLE_N, CPU_SAMPLE_N)
    oracle.default()
    t0 = time.perf_counter()
    oracle.geqr2(A)
    dt = time.perf_counter() - t0
    flops = 2.0 * CPU_SAMPLE_N ** 3 - 2.0 * CPU_SAMPLE_N ** 3 / 3.0
    return {"value": flops / dt / 1e12, "unit": "TFLOP/s", "cores": 1, "kind": "oracle",
            "sample": f"oracle_geqr2 (single thread) on one {CPU_SAMPLE_N}x{CPU_SAMPLE_N} uniform(-1,1) "
                      f"matrix, seed 0: {dt:.2f} s for {flops:.3e} flops (LAPACK count)"}


def mixed_ls(tq, torch, dev, st):
    """FP64 vs split-precision least squares on one 65536 x 1024 system."""
    import numpy as np
    from paper_0709_1272_amd import synth
    m, n, kappa = 65536, 1024, 1e6
    A, b, _ = synth.svd_matrix(0, m, n, kappa)
    At = tq.to_device(A, dev)
    Bt = tq.to_device(b, dev)
    Xt = torch.zeros((1, n), dtype=torch.float64, device=dev)
    flops = tq.flops_lapack(m, n)
    out = {"workload": f"least squares {m}x{n}, kappa {kappa:.0e}, 1 rhs, SVD construction seed 0, nb 256, ib 32",
           "flops_counted": flops, "tol": 1e-14}
    xs = {}
    for name, prec in (("fp64", tq.FP64), ("fp16x2", tq.FP16X2), ("bf16x3", tq.BF16X3), ("bf16x2", tq.BF16X2)):
        best = None
        for _ in range(3):
            info = tq.Info()
            o = tq.opts(precision=prec, nb=256, ib=32, stream=st.cuda_stream)
            rc = tq.solve_ls(m, n, 1, At.data_ptr(), m, Bt.data_ptr(), m, Xt.data_ptr(), n, o, info)
            if best is None or info.ms_total < best[1].ms_total:
                best = (rc, info)
        rc, info = best
        xs[name] = tq.to_host(Xt, n)[:, 0].copy()
        out[name] = {"status": tq.status_string(rc), "ms_total": round(info.ms_total, 3),
                     "ms_factor": round(info.ms_factor, 3), "iterations": info.iterations,
                     "eta": info.eta, "tflops": round(flops / (info.ms_total * 1e-3) / 1e12, 4)}
    for name in ("fp16x2", "bf16x3", "bf16x2"):
        out[name]["speedup_vs_fp64"] = round(out["fp64"]["ms_total"] / out[name]["ms_total"], 3)
        out[name]["rel_diff_x_vs_fp64"] = float(np.linalg.norm(xs[name] - xs["fp64"]) / np.linalg.norm(xs["fp64"]))
    return out


def mixed_ls_square(tq, torch, dev, st, n=32768):
    """FP64 vs split-precision least squares on one n x n system with 16
    right-hand sides (kappa 1e6), the square least-squares workload."""
    import numpy as np
    from paper_0709_1272_amd import synth
    t0 = time.perf_counter()
    At, Bt, _ = synth.svd_matrix_device(0, n, 1e6, nrhs=16, device=dev)
    torch.cuda.synchronize()
    gen_s = time.perf_counter() - t0
    Xt = torch.zeros((16, n), dtype=torch.float64, device=dev)
    flops = tq.flops_lapack(n, n)
    out = {"workload": f"least squares {n}x{n}, kappa 1e6, 16 rhs, A = U diag(s) V^T with Hadamard-based "
                       f"orthogonal U, V (seed 0), nb 256, ib 32",
           "flops_counted": flops, "tol": 1e-14, "generation_s": round(gen_s, 2)}
    xs = {}
    for name, prec in (("fp64", tq.FP64), ("fp16x2", tq.FP16X2), ("bf16x3", tq.BF16X3)):
        info = tq.Info()
        o = tq.opts(precision=prec, nb=256, ib=32, stream=st.cuda_stream)
        rc = tq.solve_ls(n, n, 16, At.data_ptr(), n, Bt.data_ptr(), n, Xt.data_ptr(), n, o, info)
        xs[name] = Xt.clone()
        out[name] = {"status": tq.status_string(rc), "ms_total": round(info.ms_total, 3),
                     "ms_factor": round(info.ms_factor, 3), "iterations": info.iterations,
                     "eta": info.eta, "tflops": round(flops / (info.ms_total * 1e-3) / 1e12, 4)}
    for name in ("fp16x2", "bf16x3"):
        out[name]["speedup_vs_fp64"] = round(out["fp64"]["ms_total"] / out[name]["ms_total"], 3)
        out[name]["rel_diff_x_vs_fp64"] = float(torch.linalg.norm(xs[name] - xs["fp64"]) /
                                                torch.linalg.norm(xs["fp64"]))
    del At, Bt, Xt, xs
    torch.cuda.empty_cache()
    return out


def batched(tq, torch, dev, st):
    """4000 FP64 matrices of uneven sizes in one call."""
    import numpy as np
    from paper_0709_1272_amd import synth
    ms, ns, mats = synth.batch_matrices(0)
    ms = [int(x) for x in ms]
    ns = [int(x) for x in ns]
    flops = sum(tq.flops_lapack(a, b) for a, b in zip(ms, ns))
    off = np.concatenate([[0], np.cumsum([a.size for a in mats])]).astype(np.int64)
    pristine = torch.from_numpy(np.concatenate([a.ravel(order="F") for a in mats])).to(dev)
    work = torch.empty_like(pristine)
    tmax = [max(tq.t_size(a, b, nb, ib) for nb in (64, 128, 256) for ib in (16, 32)) for a, b in zip(ms, ns)]
    toff = np.concatenate([[0], np.cumsum(tmax)]).astype(np.int64)
    T = torch.empty(int(toff[-1]) + 1, dtype=torch.float64, device=dev)
    Ap = [work.data_ptr() + 8 * int(o) for o in off[:-1]]
    Tp = [T.data_ptr() + 8 * int(o) for o in toff[:-1]]
    t0 = time.perf_counter()
    tune = tq.tune(ms, ns, tq.FP64, trials=2)
    tune_s = time.perf_counter() - t0
    times = []
    for r in range(4):
        work.copy_(pristine)
        e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        e0.record(st)
        rc = tq.factor_batched(ms, ns, Ap, ms, None, None, Tp, tq.opts(stream=st.cuda_stream))
        e1.record(st)
        torch.cuda.synchronize()
        tq.check(rc, "tileqr_factor_batched")
        if r:
            times.append(e0.elapsed_time(e1))
    best = min(times)
    return {"workload": "4000 FP64 matrices, m ~ U{32..768}, n ~ U{16..m}, N(0,1), seed 0, one call",
            "flops_counted": flops, "ms": round(best, 3), "tflops": round(flops / (best * 1e-3) / 1e12, 4),
            "tuned": {"nb": tune.nb, "ib": tune.ib, "panel_workers": tune.panel_workers,
                      "tuning_s": round(tune_s, 2)}}


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=10)
    ap.add_argument("--warmup", type=int, default=2)
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--no-extras", action="store_true")
    ap.add_argument("--extras", default="mixed_ls,mixed_ls_square,batched",
                    help="comma-separated extra measurements to run (default: all three)")
    args = ap.parse_args()
    extras = [] if args.no_extras else [e for e in args.extras.split(",") if e]
    for e in extras:
        if e not in ("mixed_ls", "mixed_ls_square", "batched"):
            ap.error(f"unknown extra measurement {e!r}")
    if args.gpus != 1:
        print(f"bench.py: --gpus {args.gpus} is not supported; this build factors on one GPU "
              f"(run with --gpus 1)", file=sys.stderr)
        sys.exit(2)

    import numpy as np
    import torch
    from paper_0709_1272_amd import synth, tileqr as tq

    assert torch.cuda.is_available(), "bench.py needs a GPU"
    dev = torch.device("cuda:0")
    A = synth.uniform(0, M, N)
    pristine = tq.to_device(A, dev)
    work = torch.empty_like(pristine)
    T = torch.empty(tq.t_size(M, N, NB, IB), dtype=torch.float64, device=dev)
    stream = torch.cuda.current_stream(dev)
    o = tq.opts(flags=tq.FLAG_TIMING, stream=stream.cuda_stream)
    flops = tq.flops_lapack(M, N)

    def step():
        work.copy_(pristine)
        tq.check(tq.factor(M, N, work.data_ptr(), M, NB, IB, T.data_ptr(), o), "tileqr_factor_ex")
        return tq.last_timing()

    for _ in range(args.warmup):
        step()
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    stages = [step() for _ in range(args.steps)]
    torch.cuda.synchronize()
    wall = time.perf_counter() - t0

    st = np.array(stages)                  # steps x 4 (ms)
    per_step = st.sum(axis=1)
    ms_per_step = float(per_step.mean())
    worker_ms = float(st[:, 2].mean())
    value = flops / (ms_per_step * 1e-3) / 1e12

    # Light sanity check of the last result: R^T R = A^T A at a few entries.
    R = np.triu(tq.to_host(work, M)[:N])
    for a, b in ((0, 0), (17, 4000), (8191, 8191), (4096, 123)):
        g, r = A[:, a] @ A[:, b], R[:, a] @ R[:, b]
        assert abs(g - r) <= 1e-12 * np.linalg.norm(A[:, a]) * np.linalg.norm(A[:, b]), (a, b)

    achieved = flops / (worker_ms * 1e-3) / 1e12
    out = {
        "metric": "QR TFLOP/s (2mn²−2n³/3): FP64 vs BF16-split+IR at equal 1e-14 backward err",
        "value": round(value, 4),
        "unit": "TFLOP/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": round(ms_per_step, 4),
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f64",
        "data": "synthetic",
        "config": {"workload": "FP64 tiled QR, one 8192x8192 matrix, uniform(-1,1) seed 0, nb=256, ib=32, "
                               "persistent DAG scheduler",
                   "m": M, "n": N, "nb": NB, "ib": IB, "precision": "fp64"},
        "stages_ms": {"layout_in": round(float(st[:, 0].mean()), 4),
                      "sched_setup": round(float(st[:, 1].mean()), 4),
                      "factor_kernel": round(worker_ms, 4),
                      "layout_out": round(float(st[:, 3].mean()), 4)},
        "wall_s_including_restores": round(wall, 4),
        "roofline": {"bound": "mfma", "achieved": round(achieved, 4), "peak": FP64_PEAK_TFLOPS,
                     "unit": "TFLOP/s", "frac": round(achieved / FP64_PEAK_TFLOPS, 4),
                     "traffic": measured_traffic(),
                     "kernel": f"k_worker<{NB},{IB}>",
                     "algorithmic": f"{flops:.4e} flops per launch (2mn^2-2n^3/3)"},
    }
    if "mixed_ls" in extras:
        out["mixed_ls"] = mixed_ls(tq, torch, dev, stream)
    if "mixed_ls_square" in extras:
        out["mixed_ls_square"] = mixed_ls_square(tq, torch, dev, stream)
    if "batched" in extras:
        out["batched"] = batched(tq, torch, dev, stream)
    if not args.no_cpu_baseline:
        out["cpu_baseline"] = cpu_baseline()
    print(json.dumps(out))


if __name__ == "__main__":
    main()
