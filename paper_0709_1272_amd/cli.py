"""Command-line driver: factorisations or least-squares solves of a seeded
synthetic matrix through the C-ABI, printing one JSON line.

    python -m paper_0709_1272_amd.cli factor --m 8192 --n 8192
    python -m paper_0709_1272_amd.cli solve --n 32768 --nrhs 16 --precision bf16x3
    python -m paper_0709_1272_amd.cli cholesky --n 32768 --nb 128
    python -m paper_0709_1272_amd.cli lu --n 8192 --nb 64 --ib 16

`factor` takes entries uniform(-1, 1); `solve` takes the Hadamard SVD
construction of a square matrix (n a power of two) with singular values
logspace(0, -log10 kappa, n) and B = A X + 1e-6 N(0, 1); `cholesky` the
symmetric positive definite U diag(s) U^T of the same construction (tiled
Cholesky, tilechol_factor); `lu` entries N(0, 1) (tiled LU with pairwise
pivoting, tilelu_factor).  Neither input needs
a dense LAPACK routine on the device, so the driver also runs under hardware
counter collection.  Before the first call the input is copied once on the
device with a plain device-to-device copy of `copy_bytes` bytes, a kernel of
known size against which memory counters can be calibrated.

Every computation runs in the library (there is no fallback); a status other
than TILEQR_OK raises.
"""
import argparse
import json
import sys

PRECISIONS = {"fp64": 0, "bf16x2": 1, "fp16x2": 2, "bf16x3": 3}


def main(argv=None):
    ap = argparse.ArgumentParser(prog="python -m paper_0709_1272_amd.cli")
    ap.add_argument("op", choices=("factor", "solve", "cholesky", "lu"))
    ap.add_argument("--m", type=int, default=None, help="rows (factor only; default n)")
    ap.add_argument("--n", type=int, required=True)
    ap.add_argument("--nrhs", type=int, default=1)
    ap.add_argument("--precision", choices=sorted(PRECISIONS), default="fp64")
    ap.add_argument("--nb", type=int, default=256)
    ap.add_argument("--ib", type=int, default=32)
    ap.add_argument("--kappa", type=float, default=1e6)
    ap.add_argument("--tol", type=float, default=1e-14)
    ap.add_argument("--seed", type=int, default=0)
    ap.add_argument("--repeat", type=int, default=1)
    args = ap.parse_args(argv)

    import torch
    from . import synth, tileqr as tq

    if not torch.cuda.is_available():
        sys.exit("paper_0709_1272_amd.cli needs a GPU")
    dev = torch.device("cuda:0")
    st = torch.cuda.current_stream(dev)
    prec = PRECISIONS[args.precision]
    n = args.n
    m = n if args.m is None or args.op == "solve" else args.m
    out = {"op": args.op, "m": m, "n": n, "precision": args.precision, "nb": args.nb, "ib": args.ib,
           "seed": args.seed, "runs": []}

    if args.op == "cholesky":
        from . import tilechol as tc
        nb = args.nb if args.nb in (64, 128) else 128
        A0 = synth.spd_matrix_device(args.seed, n, args.kappa, device=dev)
        A = torch.empty_like(A0)
        out.update(nb=nb, ib=None, kappa=args.kappa, precision="fp64")
        for _ in range(args.repeat):
            A.copy_(A0)
            info = tc.CholInfo()
            tq.check(tc.factor(n, A.data_ptr(), n, nb, tq.opts(stream=st.cuda_stream, flags=tq.FLAG_TIMING), info),
                     "tilechol_factor")
            out["runs"].append({"ms_total": round(info.ms_factor, 3), "ms_worker": round(info.ms_worker, 3)})
        torch.cuda.synchronize()
        out["copy_bytes"] = A.numel() * A.element_size()
        out["flops"] = tc.flops(n)
        print(json.dumps(out), flush=True)
        return 0
    if args.op == "lu":
        from . import tilelu as tl
        g = torch.Generator(device=dev)
        g.manual_seed(args.seed)
        A0 = torch.randn((n, n), generator=g, device=dev, dtype=torch.float64)
        A = torch.empty_like(A0)
        ib = args.ib if args.ib in (16, 32) else 16
        Lup = torch.zeros(tl.lup_size(n, 64, ib), dtype=torch.float64, device=dev)
        piv = torch.zeros(tl.piv_size(n, 64), dtype=torch.int32, device=dev)
        out.update(nb=64, ib=ib, precision="fp64")
        for _ in range(args.repeat):
            A.copy_(A0)
            info = tl.LUInfo()
            tq.check(tl.factor(n, A.data_ptr(), n, 64, ib, Lup.data_ptr(), piv.data_ptr(),
                               tq.opts(stream=st.cuda_stream, flags=tq.FLAG_TIMING), info), "tilelu_factor")
            out["runs"].append({"ms_total": round(info.ms_factor, 3), "ms_worker": round(info.ms_worker, 3)})
        torch.cuda.synchronize()
        out["copy_bytes"] = A.numel() * A.element_size()
        out["flops"] = tl.flops(n)
        print(json.dumps(out), flush=True)
        return 0
    if args.op == "factor":
        g = torch.Generator(device=dev)
        g.manual_seed(args.seed)
        A0 = torch.rand((n, m), generator=g, device=dev, dtype=torch.float64).mul_(2.0).sub_(1.0)
    else:
        A0, B, _ = synth.svd_matrix_device(args.seed, n, args.kappa, nrhs=args.nrhs, device=dev)
        X = torch.zeros((args.nrhs, n), dtype=torch.float64, device=dev)
        out.update(nrhs=args.nrhs, kappa=args.kappa, tol=args.tol)
    A = torch.empty_like(A0)
    A.copy_(A0)
    out["copy_bytes"] = A.numel() * A.element_size()
    T = torch.empty(max(tq.t_size(m, n, args.nb, args.ib), 1), dtype=torch.float64, device=dev)

    for _ in range(args.repeat):
        if args.op == "factor":
            A.copy_(A0)
            o = tq.opts(precision=prec, stream=st.cuda_stream, flags=tq.FLAG_TIMING)
            tq.check(tq.factor(m, n, A.data_ptr(), m, args.nb, args.ib, T.data_ptr(), o), "tileqr_factor_ex")
            t = tq.last_timing()
            out["runs"].append({"ms_total": round(sum(t), 3), "ms_worker": round(t[2], 3)})
        else:
            info = tq.Info()
            o = tq.opts(precision=prec, nb=args.nb, ib=args.ib, stream=st.cuda_stream, tol=args.tol)
            rc = tq.solve_ls(n, n, args.nrhs, A.data_ptr(), n, B.data_ptr(), n, X.data_ptr(), n, o, info)
            tq.check(rc, "tileqr_solve_ls")
            out["runs"].append({"ms_total": round(info.ms_total, 3), "ms_factor": round(info.ms_factor, 3),
                                "ms_worker": round(info.ms_worker, 3), "iterations": info.iterations,
                                "eta": info.eta})
    torch.cuda.synchronize()
    out["flops_lapack"] = tq.flops_lapack(m, n)
    print(json.dumps(out), flush=True)
    return 0


if __name__ == "__main__":
    sys.exit(main())
