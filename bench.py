"""Benchmark: CountSketch S A throughput (nnz/s, fraction of HBM roofline) and
least-squares solves/s at a certified residual ratio <= 1 + 1e-6, on one
MI355X.

One step = one sketch of the sparse workload: CSR A with n = 2^22 rows, d = 256
columns, 16 nonzeros per row at uniform columns, float32 N(0,1) values, sketch
size t = 65536 (hash + bucket plan + segmented reduce, every kernel of the
path from (A, seed) to S A inside the timed region).  Inputs are synthetic and
already resident in device memory when timing starts.

Also reported on the same JSON line: the generalized sparse embedding of the
same input (4 copies), the dense float32 variant (n = 2^20),
sketch-and-solve on the small sparse regression (n = 20000, d = 20), least
squares on the dense heavy-row regression workload (n = 2^21, d = 512,
t = 2^18) in the plain float64 form and the mixed-precision forms,
multiple-response regression by leverage-score sampling on it, leverage
scores on the same workload, a rank-k approximation of a planted low-rank
sparse matrix (n = 65536, about 10M nonzeros, k = 32), learned sketch values
trained on a family of 256
related matrices and compared with the random signs on held-out ones, the
roofline of the dominant kernel (measured with HIP events on the
library's stream), and the oracle timed on the host.
"""

from __future__ import annotations

import argparse
import ctypes
import json
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)

HBM_PEAK = 8.0e12  # B/s, MI355X HBM3E
SKETCH_SRC = os.path.join("paper_1207_6365_amd", "csrc", "sketch.hip")  # source of the sketch kernels


def parse():
    p = argparse.ArgumentParser()
    p.add_argument("--gpus", type=int, default=1)
    p.add_argument("--steps", type=int, default=50)
    p.add_argument("--warmup", type=int, default=5)
    p.add_argument("--variant", default="auto", choices=["auto", "atomic", "sorted", "binned"])
    p.add_argument("--no-extras", action="store_true", help="only the headline sketch workload")
    p.add_argument("--no-lstsq", action="store_true")
    p.add_argument("--no-cpu", action="store_true")
    p.add_argument("--lstsq-steps", type=int, default=3)
    p.add_argument("--only", default=None,
                   choices=["general", "dense", "small", "lstsq", "multi", "leverage", "low_rank", "lp", "learned"],
                   help="run only this extra workload after the headline")
    p.add_argument("--calib-copy-mib", type=int, default=0,
                   help="run a plain device copy of this many MiB first (scale for HBM byte counters)")
    return p.parse_args()


def profile_phases(sk):
    lib = sk.lib()
    out = {}
    name = ctypes.c_char_p()
    cnt = ctypes.c_int64()
    ms = ctypes.c_double()
    for i in range(lib.skls_profile_count()):
        if lib.skls_profile_get(i, ctypes.byref(name), ctypes.byref(cnt), ctypes.byref(ms)) == 0:
            out[name.value.decode()] = (cnt.value, ms.value)
    return out


def stored_traffic(kernel: str, source: str):
    """HBM bytes per launch of `kernel` from its counter summary under
    profiles/ (FETCH_SIZE and WRITE_SIZE scaled by a plain copy's readings),
    or None when there is none or `source` has changed since it was taken."""
    import hashlib

    path = os.path.join(ROOT, "profiles", f"{kernel}_traffic.txt")
    if not os.path.exists(path):
        return None
    fields = {}
    with open(path) as f:
        for line in f:
            if ":" in line and not line.startswith("#"):
                k, v = line.split(":", 1)
                fields[k.strip()] = v.strip()
    with open(os.path.join(ROOT, source), "rb") as f:
        sha = hashlib.sha256(f.read()).hexdigest()
    if fields.get("source_sha256") != sha or "traffic_bytes" not in fields:
        return None
    return float(fields["traffic_bytes"])


def oracle_rows(log, threads=1):
    """The oracle on bounded samples of the other workloads: seconds per call
    and the sample's size, as context for the GPU figures of each row.
    threads=1 holds BLAS to one thread; None lets it use every host core."""
    import numpy as np
    from threadpoolctl import threadpool_limits

    import oracle as O
    import workloads as W

    def timed(fn, reps=1):
        t0 = time.perf_counter()
        for _ in range(reps):
            fn()
        return (time.perf_counter() - t0) / reps

    out = {}
    with threadpool_limits(threads):
        log(f"oracle samples ({threads or 'all'} thread(s)): small regression, heavy-row regression, leverage, "
            "multiple responses, low rank, l_p, learned gradient")
        A1, b1, _ = W.lstsq_small()
        sec = timed(lambda: O.sketch_and_solve(A1, b1, W.sketch_seed(0), 4000), 5)
        out["lstsq_small"] = {"s_per_call": sec, "sample": "sketch-and-solve, the full small workload"}
        n2, d2, t2 = 1 << 15, 512, 1 << 13
        A2, b2, _ = W.pareto_rows(n=n2, d=d2, storage="f32")
        A2 = A2.astype(np.float64)
        sec = timed(lambda: O.lstsq(A2, b2, W.sketch_seed(0), t2, 1e-6))
        out["lstsq"] = {"s_per_call": sec, "rows_per_s": n2 / sec,
                        "sample": f"certified solve (delta 1e-6) of a heavy-row sample n={n2}, d={d2}, t={t2}"}
        Pi2 = np.random.default_rng(7).standard_normal((d2, 32)) / np.sqrt(32.0)
        sec = timed(lambda: O.leverage_approx(A2, W.sketch_seed(0), t2, Pi2))
        out["leverage"] = {"s_per_call": sec, "rows_per_s": n2 / sec,
                           "sample": f"leverage scores (k=32) of the same sample n={n2}, d={d2}, t={t2}"}
        B2 = np.random.default_rng(3).standard_normal((n2, 16))
        sec = timed(lambda: O.multi_response_lstsq(A2, B2, 77, t2, 4096))
        out["multi"] = {"s_per_call": sec, "rows_per_s": n2 / sec,
                        "sample": f"16 responses, the same sample n={n2}, d={d2}, t={t2}, t_s=4096"}
        A4 = W.planted_lowrank_sparse(n=4096, density=0.02)
        sec = timed(lambda: O.low_rank(A4, 32, W.sketch_seed(0), 128, 4096))
        out["low_rank"] = {"s_per_call": sec, "nnz": int(A4.nnz),
                           "sample": "rank 32 of a planted 4096 x 4096 sparse matrix, t_R=128, t_S=4096"}
        A6, b6, _ = W.lp_sparse(n=1 << 17, d=64)
        sec = timed(lambda: O.lp_regression(A6, b6, 1.0, W.sketch_seed(6), 1024, 8, 1, 2048.0, 2048.0))
        out["lp"] = {"s_per_call": sec, "nnz_per_s": A6.nnz / sec,
                     "sample": "p = 1, CSR n=2^17, d=64, 16 nnz/row, F with 2 d^2 rows, s1 = s2 = 32 d"}
        make, _ = W.learned_family()
        A5 = make(0).astype(np.float64)
        w5 = np.ones(A5.shape[0])
        sec = timed(lambda: O.distortion_grad(A5, W.sketch_seed(0), 1024, w5))
        out["learned"] = {"s_per_call": sec, "sample": "distortion loss gradient of one 32768 x 64 matrix, t=1024"}
    return out


def time_steps(fn, steps, warmup, sync):
    import torch

    for _ in range(warmup):
        fn()
    sync()
    e0 = torch.cuda.Event(enable_timing=True)
    e1 = torch.cuda.Event(enable_timing=True)
    e0.record()
    for _ in range(steps):
        fn()
    e1.record()
    sync()
    return e0.elapsed_time(e1) / steps


SPIN_CYCLES = 500_000  # device clock cycles of the spin kernel queued before each profiled call


def profile_steps(fn, steps, sync):
    """Call fn `steps` times with the library's phase events on, each call
    queued behind a spin kernel, so that the host has enqueued the whole call
    (kernels and phase events) before the GPU reaches it: each phase's event
    pair then brackets its kernels only, not the host's launch gaps."""
    import torch

    sync()
    for _ in range(steps):
        torch.cuda._sleep(SPIN_CYCLES)
        fn()
    sync()


def main():
    args = parse()
    if args.gpus != 1:
        print(f"bench.py measures one GPU only; --gpus {args.gpus} is not supported (the row sharding of the "
              "sketch over several GPUs is described, not built)", file=sys.stderr)
        sys.exit(2)
    import numpy as np
    import torch

    import paper_1207_6365_amd as sk
    import workloads as W

    if not torch.cuda.is_available():
        print("bench.py needs a GPU", file=sys.stderr)
        sys.exit(1)
    dev = torch.device("cuda:0")
    lib = sk.lib()
    sync = torch.cuda.synchronize
    t = 65536
    seed = W.sketch_seed(0)

    def log(msg):
        print(msg, file=sys.stderr, flush=True)

    def want(name):
        return args.only is None or args.only == name

    if args.calib_copy_mib > 0:
        # a plain copy of known size: its FETCH_SIZE / WRITE_SIZE per dispatch
        # calibrate the byte counters taken on the sketch kernels
        nb = args.calib_copy_mib << 20
        src = torch.ones(nb // 4, dtype=torch.float32, device=dev)
        dst = torch.empty_like(src)
        for _ in range(3):
            torch.mul(src, 2.0, out=dst)  # an elementwise kernel: reads nb bytes, writes nb bytes
        sync()
        del src, dst

    # ------------------------------------------------------------ headline
    log("generating the sparse sketch workload (n=2^22, d=256, 16 nnz/row)")
    A, b = W.sketch_csr()
    nnz = A.nnz
    Ag = sk.Csr(A.n, A.d, torch.from_numpy(A.row_ptr32()).to(dev), torch.from_numpy(A.col_idx).to(dev),
                torch.from_numpy(A.val).to(dev))
    SA = torch.empty((t, A.d), dtype=torch.float32, device=dev)
    ws_bytes = ctypes.c_size_t(0)
    mat, _ = sk.api._matrix(Ag)
    variant = sk.api._VARIANT[args.variant]
    sk._lib.check(lib.skls_sketch_workspace(ctypes.byref(mat), t, variant, ctypes.byref(ws_bytes)))
    ws = torch.empty(max(ws_bytes.value, 1), dtype=torch.uint8, device=dev)
    stream = torch.cuda.current_stream(dev).cuda_stream

    def step():
        st = lib.skls_sketch(ctypes.byref(mat), None, 0, t, seed, None, variant, SA.data_ptr(), None, 1,
                             ws.data_ptr(), ws.numel(), stream)
        if st != 0:
            sk._lib.check(st)

    log(f"timing {args.steps} sketch steps after {args.warmup} warm-up steps")
    ms_step = time_steps(step, args.steps, args.warmup, sync)
    lib.skls_profile_enable(1)
    profile_steps(step, args.steps, sync)
    phases = profile_phases(sk)
    lib.skls_profile_enable(0)

    alg_bytes = 4 * nnz + 4 * nnz + 4 * (A.n + 1) + 4 * t * A.d  # val + col + row_ptr + write S A
    kname = {"atomic": "k_sketch_csr_atomic", "sorted": "k_sketch_csr_sorted"}.get(args.variant, "k_sketch_csr_binned")
    value = nnz / (ms_step * 1e-3)
    dom = "sketch_apply"
    cnt, tot = phases.get(dom, (0, float("nan")))
    k_ms = tot / max(cnt, 1)
    achieved = alg_bytes / (k_ms * 1e-3)
    plan_cnt, plan_tot = phases.get("sketch_plan", (0, 0.0))
    result = {
        "metric": "SA nnz/s (% HBM roofline); lstsq solves/s at residual ratio <=1+1e-6",
        "value": value,
        "unit": "nnz/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": ms_step,
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f32",
        "data": "synthetic",
        "config": {"workload": "CountSketch S*A of CSR A, n=2^22, d=256, 16 nnz/row, float32 N(0,1), t=65536",
                   "n": A.n, "d": A.d, "nnz": nnz, "t": t, "variant": args.variant, "parallelism": "single GPU"},
        "roofline": {"bound": "hbm", "achieved": achieved / 1e9, "peak": HBM_PEAK / 1e9, "unit": "GB/s",
                     "frac": achieved / HBM_PEAK, "traffic": stored_traffic(kname, SKETCH_SRC),
                     "kernel": kname,
                     "kernel_ms": k_ms, "algorithmic_bytes": alg_bytes},
        "step_roofline_frac": alg_bytes / (ms_step * 1e-3) / HBM_PEAK,
        "phases_ms": {k: v[1] / max(v[0], 1) for k, v in phases.items()},
    }
    if plan_cnt:
        result["phases_ms"]["sketch_plan"] = plan_tot / plan_cnt
    # the apply alone, with the bucket plan of these row pointers built once
    # and reused (a matrix whose values or columns change but whose rows keep
    # their lengths reuses it)
    hplan = sk.sketch_plan(Ag, t, seed, variant=args.variant)
    hdesc, hbuf = hplan.desc, hplan.buf

    def hstep():
        st = lib.skls_sketch_planned(ctypes.byref(mat), None, 0, None, SA.data_ptr(), None, ctypes.byref(hdesc),
                                     hbuf.data_ptr(), hbuf.numel(), stream)
        if st != 0:
            sk._lib.check(st)

    hms = time_steps(hstep, args.steps, args.warmup, sync)
    result["reused_plan"] = {"ms_per_step": hms, "nnz_per_s": nnz / (hms * 1e-3),
                             "frac": (alg_bytes - 4 * (A.n + 1)) / (hms * 1e-3) / HBM_PEAK,
                             "note": "apply only; algorithmic bytes without the row pointers, which only the "
                                     "plan reads"}
    del hplan, hbuf

    if not args.no_extras and want("general"):
        # generalized sparse embedding (Section 5) of the same input: q groups,
        # a copies of v rows each, a q v = t rows in all
        q_g, v_g, a_g = 1024, 16, 4
        log(f"generalized sparse embedding: same CSR input, q={q_g} v={v_g} a={a_g} (t={q_g * v_g * a_g})")
        gws = ctypes.c_size_t(0)
        sk._lib.check(lib.skls_sketch_general_workspace(ctypes.byref(mat), q_g, v_g, variant, ctypes.byref(gws)))
        wsg = torch.empty(max(gws.value, 1), dtype=torch.uint8, device=dev)

        def gstep():
            st = lib.skls_sketch_general(ctypes.byref(mat), None, 0, q_g, v_g, a_g, seed, variant, SA.data_ptr(),
                                         None, 1, wsg.data_ptr(), wsg.numel(), stream)
            if st != 0:
                sk._lib.check(st)

        gms = time_steps(gstep, max(args.steps // 2, 5), 3, sync)
        result["general"] = {"q": q_g, "v": v_g, "a": a_g, "t": q_g * v_g * a_g, "ms_per_call": gms,
                             "nnz_per_s": nnz / (gms * 1e-3), "ms_per_copy": gms / a_g}
        del wsg
    del Ag

    # ------------------------------------------------------------ extras
    small_run = None
    if not args.no_extras:
        if want("dense"):
            log("dense float32 variant (n=2^20, d=256)")
            D, _ = W.sketch_dense()
            Dg = torch.from_numpy(D).to(dev)
            dm, _ = sk.api._matrix(Dg)
            sk._lib.check(lib.skls_sketch_workspace(ctypes.byref(dm), t, variant, ctypes.byref(ws_bytes)))
            wsd = torch.empty(max(ws_bytes.value, 1), dtype=torch.uint8, device=dev)

            def dstep():
                sk._lib.check(lib.skls_sketch(ctypes.byref(dm), None, 0, t, seed, None, variant, SA.data_ptr(), None, 1,
                                              wsd.data_ptr(), wsd.numel(), stream))

            dms = time_steps(dstep, max(args.steps // 2, 5), 3, sync)
            lib.skls_profile_enable(1)
            profile_steps(dstep, max(args.steps // 2, 5), sync)
            dph = profile_phases(sk)
            lib.skls_profile_enable(0)
            dbytes = 4 * D.size + 4 * t * D.shape[1]
            dk = dph.get("sketch_apply", (1, float("nan")))
            # the same sketch with the bucket plan built once and reused: the
            # plan depends only on (seed, n, t), so every dense matrix with
            # these rows can share it
            plan = sk.sketch_plan(Dg, t, seed, variant=args.variant)
            pdesc, pbuf = plan.desc, plan.buf

            def pstep():
                sk._lib.check(lib.skls_sketch_planned(ctypes.byref(dm), None, 0, None, SA.data_ptr(), None,
                                                      ctypes.byref(pdesc), pbuf.data_ptr(), pbuf.numel(), stream))

            pms = time_steps(pstep, max(args.steps // 2, 5), 3, sync)
            result["dense"] = {"entries_per_s": D.size / (dms * 1e-3), "ms_per_step": dms,
                               "kernel_frac": dbytes / (dk[1] / max(dk[0], 1) * 1e-3) / HBM_PEAK,
                               "step_frac": dbytes / (dms * 1e-3) / HBM_PEAK,
                               "phases_ms": {k: v[1] / max(v[0], 1) for k, v in dph.items()},
                               "reused_plan": {"entries_per_s": D.size / (pms * 1e-3), "ms_per_step": pms,
                                               "step_frac": dbytes / (pms * 1e-3) / HBM_PEAK,
                                               "plan_bytes": int(pbuf.numel())}}
            del Dg, D, plan, pbuf

        if want("small"):
            log("small sparse regression: sketch-and-solve, n=20000 d=20 4 nnz/row float64, t=4000")
            A1, b1, _ = W.lstsq_small()
            A1g = sk.Csr(A1.n, A1.d, torch.from_numpy(A1.row_ptr32()).to(dev), torch.from_numpy(A1.col_idx).to(dev),
                         torch.from_numpy(A1.val).to(dev))
            b1g = torch.from_numpy(b1).to(dev)
            for _ in range(3):
                x1, info1 = sk.lstsq(A1g, b1g, 4000, seed, sketch_only=True)
            sync()
            reps = 50
            t0 = time.perf_counter()
            for _ in range(reps):
                x1, info1 = sk.lstsq(A1g, b1g, 4000, seed, sketch_only=True)
            sync()
            el = (time.perf_counter() - t0) / reps
            result["lstsq_small"] = {"solves_per_s": 1.0 / el, "ms_per_solve": el * 1e3,
                                     "note": "sketch-and-solve only (no LSQR), launch-bound; its residual ratio "
                                             "against the oracle's is in cpu_baseline.parity"}
            # certified solves (sketch-and-solve, then LSQR to 1 + 1e-6)
            certified = {}
            for precision in ("plain", "mixed"):
                for _ in range(3):
                    sk.lstsq(A1g, b1g, 4000, seed, delta=1e-6, precision=precision)
                sync()
                t0 = time.perf_counter()
                for _ in range(reps):
                    _, ci = sk.lstsq(A1g, b1g, 4000, seed, delta=1e-6, precision=precision)
                sync()
                el = (time.perf_counter() - t0) / reps
                certified[precision] = {"solves_per_s": 1.0 / el, "ms_per_solve": el * 1e3,
                                        "iterations": ci["iterations"], "refinements": ci["refinements"],
                                        "certified": ci["certified"]}
            result["lstsq_small"]["certified_1e-6"] = certified
            small_run = (A1, b1, x1.cpu().numpy())
            del A1g, b1g

    # ------------------------------------------------------------ least squares
    if not args.no_lstsq:
        n3, d3, t3 = 1 << 21, 512, 1 << 18
        if want("lstsq"):
            res = {}
            for storage, precision in (("f32", "plain"), ("f32", "mixed"), ("bf16", "mixed")):
                log(f"least squares: dense heavy-row workload n=2^21 d=512 t=2^18, {storage} storage, {precision}")
                A3, b3, _ = W.pareto_rows(n=n3, d=d3, storage=storage)
                A3g = (torch.from_numpy(A3.view(np.int16)).to(dev).view(torch.bfloat16) if storage == "bf16"
                       else torch.from_numpy(A3).to(dev))
                del A3
                b3g = torch.from_numpy(b3).to(dev)
                x, info = sk.lstsq(A3g, b3g, t3, seed, delta=1e-6, precision=precision)  # warm-up
                sync()
                t0 = time.perf_counter()
                infos = []
                for _ in range(args.lstsq_steps):
                    x, info = sk.lstsq(A3g, b3g, t3, seed, delta=1e-6, precision=precision)
                    infos.append(info)
                sync()
                el = (time.perf_counter() - t0) / args.lstsq_steps
                # kernel phases from one more solve with the phase events on
                lib.skls_profile_enable(1)
                sk.lstsq(A3g, b3g, t3, seed, delta=1e-6, precision=precision)
                sync()
                ph = profile_phases(sk)
                lib.skls_profile_enable(0)
                key = f"{storage}_{precision}"
                pass_name = "lsqr_pass_f64" if precision == "plain" else "lsqr_pass_f32"
                pc, pt_ = ph.get(pass_name, (1, float("nan")))
                es = 2 if storage == "bf16" else 4
                pass_bytes = n3 * d3 * es + n3 * (8 if precision == "plain" else 4) * 2
                res[key] = {
                    "solves_per_s": 1.0 / el, "ms_per_solve": el * 1e3,
                    "certified": all(i["certified"] == 1 for i in infos),
                    "ratio_bound": max(i["ratio_bound"] for i in infos),
                    "iterations": infos[-1]["iterations"], "refinements": infos[-1]["refinements"],
                    "ms_sketch": infos[-1]["ms_sketch"], "ms_qr": infos[-1]["ms_qr"], "ms_iter": infos[-1]["ms_iter"],
                    "pass_frac": pass_bytes / (pt_ / max(pc, 1) * 1e-3) / HBM_PEAK,
                    "phases_ms": {k: v[1] / max(v[0], 1) for k, v in ph.items()},
                }
                # R from the second stage Pi1 = F S (m = 4 d and 8 d) in place of S A
                stage = {}
                for m2 in (4 * d3, 8 * d3):
                    sk.lstsq(A3g, b3g, t3, seed, delta=1e-6, precision=precision, second_stage=m2)
                    sync()
                    t0 = time.perf_counter()
                    sinfos = []
                    for _ in range(args.lstsq_steps):
                        _, si = sk.lstsq(A3g, b3g, t3, seed, delta=1e-6, precision=precision, second_stage=m2)
                        sinfos.append(si)
                    sync()
                    el2 = (time.perf_counter() - t0) / args.lstsq_steps
                    lib.skls_profile_enable(1)
                    sk.lstsq(A3g, b3g, t3, seed, delta=1e-6, precision=precision, second_stage=m2)
                    sync()
                    ph2 = profile_phases(sk)
                    lib.skls_profile_enable(0)
                    stage[str(m2)] = {
                        "solves_per_s": 1.0 / el2, "ms_per_solve": el2 * 1e3,
                        "certified": all(i["certified"] == 1 for i in sinfos),
                        "iterations": sinfos[-1]["iterations"], "refinements": sinfos[-1]["refinements"],
                        "ms_qr": sinfos[-1]["ms_qr"], "ms_iter": sinfos[-1]["ms_iter"],
                        "ms_second_stage": ph2.get("second_stage", (1, float("nan")))[1],
                    }
                res[key]["second_stage"] = stage
                del A3g, b3g
                torch.cuda.empty_cache()
            result["lstsq"] = res

        if want("multi"):
            # multiple-response regression by leverage-score sampling on the
            # heavy-row workload with d' = 16 responses; the optimum per
            # response from solves certified to 1 + 1e-11
            dp, t_s = 16, 16384
            log(f"multiple-response regression: n=2^21 d=512 float32, d'={dp}, t=2^18, t_s={t_s}")
            A3, _, _ = W.pareto_rows(n=n3, d=d3, storage="f32")
            g5 = np.random.default_rng(W.data_seed(3, 7))
            Y0 = g5.standard_normal((d3, dp))
            B3 = np.empty((n3, dp))
            for r0 in range(0, n3, 1 << 18):
                B3[r0:r0 + (1 << 18)] = A3[r0:r0 + (1 << 18)].astype(np.float64) @ Y0
            B3 += 1e-3 * g5.standard_normal((n3, dp))
            A3g = torch.from_numpy(A3).to(dev)
            B3g = torch.from_numpy(B3).to(dev)
            del A3, B3
            sk.multi_lstsq(A3g, B3g, t3, t_s, seed)  # warm-up
            sync()
            reps = 3
            t0 = time.perf_counter()
            for _ in range(reps):
                Ym, minfo = sk.multi_lstsq(A3g, B3g, t3, t_s, seed)
            sync()
            el = (time.perf_counter() - t0) / reps
            opt2 = 0.0
            for c in range(dp):
                _, ci = sk.lstsq(A3g, B3g[:, c].contiguous(), t3, seed, delta=1e-11)
                opt2 += ci["resid_norm"] ** 2
            result["multi_response"] = {
                "ms_per_call": el * 1e3, "d_rhs": dp, "t": t3, "t_s": t_s, "rows_sampled": minfo["rows_sampled"],
                "residual_ratio": minfo["resid_fro"] / np.sqrt(opt2), "ms_scores": minfo["ms_scores"],
                "ms_solve": minfo["ms_solve"]}
            del A3g, B3g
            torch.cuda.empty_cache()

        if want("leverage"):
            # leverage scores on the same heavy-row workload (float32 storage), k = 32
            log("leverage scores: n=2^21 d=512 float32, t=2^18, k=32")
            A3, b3, _ = W.pareto_rows(n=n3, d=d3, storage="f32")
            A3g = torch.from_numpy(A3).to(dev)
            del A3, b3
            Pi2 = torch.from_numpy(np.random.default_rng(7).standard_normal((d3, 32)) / np.sqrt(32.0)).to(dev)
            sk.leverage_scores(A3g, t3, seed, Pi2)
            sync()
            t0 = time.perf_counter()
            reps = 3
            for _ in range(reps):
                sk.leverage_scores(A3g, t3, seed, Pi2)
            sync()
            el = (time.perf_counter() - t0) / reps
            lib.skls_profile_enable(1)
            profile_steps(lambda: sk.leverage_scores(A3g, t3, seed, Pi2), 1, sync)
            ph = profile_phases(sk)
            lib.skls_profile_enable(0)
            lc, lt = ph.get("leverage", (1, float("nan")))
            result["leverage"] = {"ms_per_call": el * 1e3, "phases_ms": {k: v[1] / max(v[0], 1) for k, v in ph.items()},
                                  "pass_frac": (n3 * d3 * 4 + n3 * 4) / (lt / max(lc, 1) * 1e-3) / HBM_PEAK}
            del A3g
            torch.cuda.empty_cache()

        if want("low_rank"):
            # rank-k approximation of the planted low-rank sparse matrix (65536 x
            # 65536, about 10M nonzeros, k = 32, t_R = 512); error against the
            # stored best rank-k error of the same seeded matrix
            log("low rank: planted sparse n=65536 ~10M nnz, k=32, t_R=512")
            A4 = W.planted_lowrank_sparse()
            A4g = sk.Csr(A4.n, A4.d, torch.from_numpy(A4.row_ptr32()).to(dev), torch.from_numpy(A4.col_idx).to(dev),
                         torch.from_numpy(A4.val).to(dev))
            gold = {}
            with open(os.path.join(ROOT, "tests", "golden", "lowrank_planted_n65536_r32.txt")) as f:
                for line in f:
                    if ":" in line and not line.startswith("#"):
                        key, v = line.split(":", 1)
                        gold[key.strip()] = float(v)
            lr_seed = W.sketch_seed(0)
            sk.low_rank(A4g, 32, lr_seed, t_r=512)  # warm-up
            sync()
            reps = 3
            t0 = time.perf_counter()
            for _ in range(reps):
                _, _, _, linfo = sk.low_rank(A4g, 32, lr_seed, t_r=512)
            sync()
            el = (time.perf_counter() - t0) / reps
            lib.skls_profile_enable(1)
            sk.low_rank(A4g, 32, lr_seed, t_r=512)
            sync()
            ph = profile_phases(sk)
            lib.skls_profile_enable(0)
            result["low_rank"] = {
                "ms_per_call": el * 1e3, "nnz": A4.nnz, "k": 32, "t_r": linfo["t_r"], "t_s": linfo["t_s"],
                "error_ratio": linfo["resid_fro"] / gold["delta_k"], "iterations": linfo["iterations"],
                "rows_sampled": linfo["rows_sampled"],
                "ms_phases": {"sketch_and_basis": linfo["ms_sketch"], "scores_and_sampling": linfo["ms_sample"],
                              "top_k": linfo["ms_topk"], "factors_and_error": linfo["ms_factors"]},
                "kernel_phases_ms": {k: v[1] / max(v[0], 1) for k, v in ph.items()},
            }
            del A4, A4g
            torch.cuda.empty_cache()

        if want("lp"):
            # l_p regression (Section 9) on the CSR workload of the headline
            # sketch (n=2^22, d=256, 16 nnz/row) with b = A x0 + Laplace noise
            # and 1% gross outliers; default sizes (F with 2 d^2 rows, s1 = s2
            # = 32 d); the fit is reported against the planted x0
            log("l_p regression: CSR n=2^22 d=256 16 nnz/row, p = 1 and 1.5")
            A6, b6, x6 = W.lp_sparse()
            A6g = sk.Csr(A6.n, A6.d, torch.from_numpy(A6.row_ptr32()).to(dev), torch.from_numpy(A6.col_idx).to(dev),
                         torch.from_numpy(A6.val).to(dev))
            b6g = torch.from_numpy(b6).to(dev)
            res = {}
            for pp in (1.0, 1.5):
                planted = float(np.sum(np.abs(A6.matvec64(x6) - b6) ** pp))
                lp_seed = W.sketch_seed(6)
                sk.lp_regression(A6g, b6g, pp, lp_seed)  # warm-up
                sync()
                reps = 3
                t0 = time.perf_counter()
                for _ in range(reps):
                    _, pinfo = sk.lp_regression(A6g, b6g, pp, lp_seed)
                sync()
                el = (time.perf_counter() - t0) / reps
                lib.skls_profile_enable(1)
                sk.lp_regression(A6g, b6g, pp, lp_seed)
                sync()
                ph = profile_phases(sk)
                lib.skls_profile_enable(0)
                res[f"p{pp:g}"] = {
                    "ms_per_call": el * 1e3, "calls_per_s": 1.0 / el,
                    "objective_vs_planted": pinfo["obj"] / planted,
                    "stage1_objective_vs_planted": pinfo["obj_stage1"] / planted,
                    "rows": [pinfo["rows_stage1"], pinfo["rows_stage2"]],
                    "fit_iterations": [pinfo["iters_stage1"], pinfo["iters_stage2"]],
                    "converged": pinfo["converged"],
                    "ms_phases": {"condition": pinfo["ms_condition"], "stage1": pinfo["ms_stage1"],
                                  "stage2": pinfo["ms_stage2"]},
                    "phases_ms": {k: v[1] / max(v[0], 1) for k, v in ph.items()},
                }
            result["lp_regression"] = {"workload": "CSR n=2^22 d=256 16 nnz/row float32, Laplace(0.1) noise, "
                                                   "1% outliers", "nnz": int(A6.nnz), **res}
            del A6g, b6g
            torch.cuda.empty_cache()

        if want("learned"):
            # learned per-row values: the full family of 256 matrices, trained on
            # the GPU, then compared with the random signs on held-out matrices by
            # distortion, by the sketch-and-solve residual ratio, and by solves to
            # a certified ratio of 1 + 1e-6 with the values as the sketch.
            nl, tl, steps_l, batch_l = 32768, 1024, 500, 16
            log("learned values: 256 matrices n=32768 d=64 t=1024 (160 train / 32 validation / 64 test), "
                f"{steps_l} Adam steps, batch {batch_l}")
            from paper_1207_6365_amd import train as TR

            make, _ = W.learned_family()
            host = [make(m) for m in range(256)]
            mats = [torch.from_numpy(a).to(dev) for a in host]
            rhs = [torch.from_numpy(W.learned_rhs(host[m], m)).to(dev) for m in range(192, 256)]
            del host
            tr_m, va_m, te_m = mats[:160], mats[160:192], mats[192:]
            sync()
            t0 = time.perf_counter()
            out = TR.train(tr_m, va_m, tl, seed, steps=steps_l, lr=1e-2, batch=batch_l)
            sync()
            train_s = time.perf_counter() - t0
            grams, norms, ws5 = TR.prepare(te_m, tl, seed)
            sgn = TR.signs(nl, tl, seed, dev)
            plain = TR.distortions(te_m, grams, norms, tl, seed, sgn, ws=ws5)
            learned = TR.distortions(te_m, grams, norms, tl, seed, out.learned, ws=ws5)
            norms_a = np.array(norms)

            def ratios(w):
                # residual of the sketch-and-solve x~ (no iteration) over the optimum,
                # the latter from a solve certified to 1 + 1e-11
                r = []
                for A, b in zip(te_m, rhs):
                    _, i0 = sk.lstsq(A, b, tl, seed, max_iter=0, w=w, raise_noconv=False)
                    _, i1 = sk.lstsq(A, b, tl, seed, delta=1e-11, w=w)
                    r.append(i0["resid_norm"] / i1["resid_norm"])
                return np.array(r)

            def solves(w):
                for A, b in zip(te_m[:4], rhs[:4]):
                    sk.lstsq(A, b, tl, seed, delta=1e-6, w=w)
                sync()
                its, cert = [], True
                t0 = time.perf_counter()
                for A, b in zip(te_m, rhs):
                    _, i = sk.lstsq(A, b, tl, seed, delta=1e-6, w=w)
                    its.append(i["iterations"])
                    cert = cert and i["certified"] == 1
                sync()
                el = (time.perf_counter() - t0) / len(te_m)
                return {"solves_per_s": 1.0 / el, "mean_iterations": float(np.mean(its)), "certified": cert}

            rho_p, rho_l = ratios(None), ratios(out.learned)
            result["learned"] = {
                "matrices": {"train": 160, "validation": 32, "test": 64}, "n": nl, "d": 64, "t": tl,
                "train_s": train_s, "steps": steps_l, "batch": batch_l, "used_learned": bool(out.used_learned),
                "validation_distortion": {"plain": out.val_plain, "learned": out.val_learned},
                "test_distortion": {"plain": float(plain.mean()), "learned": float(learned.mean())},
                "test_distortion_raw": {"plain": float((plain * norms_a).mean()),
                                        "learned": float((learned * norms_a).mean())},
                "sketch_solve_ratio_minus_1": {"plain": float((rho_p - 1).mean()), "learned": float((rho_l - 1).mean()),
                                               "plain_max": float((rho_p - 1).max()),
                                               "learned_max": float((rho_l - 1).max())},
                "lstsq_1e-6": {"plain": solves(None), "learned": solves(out.learned)},
            }
            del mats, tr_m, va_m, te_m, rhs
            torch.cuda.empty_cache()

    # ------------------------------------------------------------ oracle on the host
    if not args.no_cpu:
        import oracle as O

        log("timing the oracle on the host (same sparse workload, 2 repetitions)")
        reps = 2
        t0 = time.perf_counter()
        for _ in range(reps):
            O.sketch_csr(A.n, A.d, A.row_ptr, A.col_idx, A.val, seed, t)
        el = (time.perf_counter() - t0) / reps
        result["cpu_baseline"] = {"value": nnz / el, "unit": "nnz/s", "cores": 1, "kind": "oracle",
                                  "sample": f"full sparse workload (nnz={nnz}), {reps} repetitions of the NumPy "
                                            "float64 oracle sketch, single thread",
                                  "host_cpus": os.cpu_count()}
        if args.only is None and not args.no_extras:
            result["cpu_baseline"]["rows"] = oracle_rows(log)
            # the same samples with BLAS free to use every host core (the
            # headline sketch has no multithreaded NumPy path: its figure
            # holds for any core count)
            result["cpu_baseline"]["rows_all_cores"] = oracle_rows(log, threads=None)
            result["cpu_baseline"]["rows_all_cores"]["cores"] = int(os.environ.get("OMP_NUM_THREADS") or os.cpu_count())
        if small_run is not None:
            # the small regression's sketch-and-solve on the GPU against the
            # oracle's on the same seeded input: residual ratios to the exact
            # least-squares residual
            A1, b1, x1h = small_run
            Ad1 = O.MatrixOp(A1).dense()
            xs1 = O.lstsq_exact(Ad1, b1)
            xo1 = O.sketch_and_solve(A1, b1, seed, 4000)[0]
            rg, ro = O.residual_ratio(Ad1, b1, x1h, xs1), O.residual_ratio(Ad1, b1, xo1, xs1)
            result["cpu_baseline"]["parity"] = {
                "lstsq_small": {"rho_minus_1_gpu": rg - 1.0, "rho_minus_1_oracle": ro - 1.0, "abs_diff": abs(rg - ro),
                                "x_rel_diff": float(np.linalg.norm(x1h - xo1) / np.linalg.norm(xo1)),
                                "x_rel_err_gpu": float(np.linalg.norm(x1h - xs1) / np.linalg.norm(xs1))}}
    print(json.dumps(result), flush=True)


if __name__ == "__main__":
    main()
