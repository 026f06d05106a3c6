"""Benchmark: H^2-ULV factor + solve at N = 2^20 on one MI355X.

One step = h2_factor + h2_solve (the parallel substitution as the
preconditioner of CG against the FP64 H^2 operator, down to a relative
residual of 1e-8) on a resident H^2 matrix of 2^20 points; the H^2
construction runs once before the timed region.  The default run times the
target path (rank-predicted basis buffers; the near-pair, diagonal and
far-coupling transforms on FP32 copies of their operands in HBM, multiplied on
the BF16 matrix cores with each operand split into BF16 high and low parts
(three products per product, FP32 accumulation); the Schur update on FP32
MFMA; the substitution reading BF16 copies of the factors, with FP64
products and sums; Cholesky factors, root, H^2 matvec and refinement in
FP64) next to the plain FP64 path and
prints one JSON line with both.

    python bench.py [--steps K] [--warmup W] [--gpus 1] [--path target|plain|custom]
"""
from __future__ import annotations

import argparse
import json
import math
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

FP64_PEAK_TFLOPS = 78.6      # MI355X dense FP64 (vector = matrix)
# The pair-transform GEMM by precision: kernel, dense matrix peak of the
# instruction it runs, and matrix-core flops executed per algorithmic flop
# (split BF16 does three BF16 products per product).
PAIR_KERNEL = {0: ("gemm_f64_pair_kernel", FP64_PEAK_TFLOPS, 1),
               1: ("gemm_f32io_pair_kernel", 157.3, 1),
               2: ("gemm_bf16s_pair_kernel", 2500.0, 1),
               3: ("gemm_bf16s_pair_kernel", 2500.0, 3)}
HBM_PEAK_GBS = 8000.0

# HBM bytes per launch measured with rocprofv3 --pmc FETCH_SIZE and, in a
# second run, WRITE_SIZE on this workload (the default target path, one factor
# + one solve), each scaled by the counter's reading for a plain 1 GiB device
# copy (FETCH_SIZE reads half of the bytes moved: factor 2.0; WRITE_SIZE
# factor 1.0).  Valid only for the sources they were taken on (the kernel and
# the planner that shapes its launches): a changed source reports null.
GATHER_SRC = ['paper_2502_02395_amd/csrc/k_gather.hip', 'paper_2502_02395_amd/csrc/gather_plan.cpp',
              'paper_2502_02395_amd/csrc/h2_internal.hpp']
MEASURED_TRAFFIC = {
    "gv16_kernel<bf16>": {"src": GATHER_SRC, "sha256": "cfd79b81529fae76baeb9a8fb9eb92a39b5c7c791f0d54b12b3b4f182eb2e13e",
                          "bytes_per_launch": 0.3867e9 + 0.0114e9},
    "gchunk_kernel<f32> (PCG products)": {"src": GATHER_SRC, "sha256": "cfd79b81529fae76baeb9a8fb9eb92a39b5c7c791f0d54b12b3b4f182eb2e13e",
                                          "bytes_per_launch": 22.6678e9 + 0.6242e9},
    "gchunk_kernel<f64>": {"src": GATHER_SRC, "sha256": "cfd79b81529fae76baeb9a8fb9eb92a39b5c7c791f0d54b12b3b4f182eb2e13e",
                           "bytes_per_launch": 0.4720e9 + 0.0069e9},
    "greduce_kernel": {"src": GATHER_SRC, "sha256": "cfd79b81529fae76baeb9a8fb9eb92a39b5c7c791f0d54b12b3b4f182eb2e13e",
                       "bytes_per_launch": 0.0171e9 + 0.0013e9},
}


def measured_traffic(kernel: str):
    import hashlib
    m = MEASURED_TRAFFIC.get(kernel)
    if m is None:
        return None
    h = hashlib.sha256()
    for src in m["src"]:
        with open(os.path.join(ROOT, src), "rb") as f:
            h.update(f.read())
    return m["bytes_per_launch"] if h.hexdigest() == m["sha256"] else None


PHASES = ["basis_qr", "diag_transform", "rr_cholesky_inverse", "v_schur", "near_pair_transform",
          "far_coupling", "merge", "root", "solve_copies"]


def factor_roofline(st: dict, t_phase: list, t_factor: float, prec: int) -> dict:
    """Precision-weighted roofline of the factorization: the time each phase's
    canonical flops would take at the dense peak of the matrix instruction
    that runs them (FP64 78.6 TF; FP32 157.3 TF; BF16 2500 TF, a third of it
    for split BF16, which issues three products per product), summed over the
    phases, divided by the measured factor time; per phase the same ratio."""
    f64, f32 = FP64_PEAK_TFLOPS * 1e12, 157.3e12
    tr = {0: f64, 1: f32, 2: 2500e12, 3: 2500e12 / 3}[prec]
    schur = f64 if prec == 0 else f32
    peak = [f64, tr, f64, None, tr, tr, None, f64, None]
    total = 0.0
    phases = {}
    for q, name in enumerate(PHASES):
        fl = st["flops_factor_phase"][q]
        if fl <= 0:
            continue
        if q == 3:  # V and L(s) in FP64, the Schur update on the reduced GEMMs
            ideal = (fl - st["flops_schur"]) / f64 + st["flops_schur"] / schur
        else:
            ideal = fl / peak[q]
        total += ideal
        t = t_phase[q]
        phases[name] = {"gflop": fl / 1e9, "s": t,
                        "tflops": fl / t / 1e12 if t > 0 else None,
                        "frac": ideal / t if t > 0 else None}
    return {"bound": "mfma", "ideal_s": total, "measured_s": t_factor,
            "frac": total / t_factor if t_factor > 0 else None, "phases": phases}


def matern_status(h2, n: int) -> dict:
    """The rank-predictor configuration's kernel (Matern-3/2, l = 0.2, 1e-4
    nugget, leaf 256, eps 1e-6, 512-point samples) at n points, built and
    factored on the FP64 path: the status of each call, and where a Cholesky
    breakdown happened."""
    import torch
    import workloads as W
    p = W.matern_cube(n=n, leaf=256, eps=1e-6, s=512)
    out = {"workload": "matern_cube", "n": p.n, "leaf": p.leaf, "eps": p.eps, "s": 512,
           "kernel": "matern32 l=0.2 nugget=1e-4"}
    try:
        H = h2.build(p.points, p.kernel, p.leaf, p.eta, p.eps, p.perm(), s_far=p.s_far,
                     s_near=p.s_near)
    except h2.H2Error as e:
        out.update({"stage": "build", "status": h2._status_str(e.status), "where": e.where})
        return out
    s = h2.load().h2_factor(H._h, h2._stream(None))
    st = H.stats()
    out.update({"stage": "factor", "status": h2._status_str(s),
                "where": {"fail_level": st["fail_level"], "fail_box": st["fail_box"]}
                if s == h2.ERR_NOT_SPD else None})
    H.close()
    torch.cuda.empty_cache()
    return out


def workload(n: int, kernel: str, eps: float, leaf: int, s: int, nrhs: int = 1):
    import workloads as W
    if kernel == "gaussian_batch":
        return W.gaussian_batch(n_inst=64, leaf=leaf, eps=eps, s=s)
    if kernel == "yukawa":
        return W.yukawa_cube(n=n, leaf=leaf, eps=eps, nrhs=nrhs, s=s)
    if kernel == "laplace_sphere":
        return W.laplace_sphere(n=n, leaf=leaf, eps=eps, nrhs=nrhs, s=s)
    if kernel == "laplace":
        return W.laplace_cube(n=n, leaf=leaf, eps=eps, s=s)
    if kernel == "matern":
        return W.matern_cube(n=n, leaf=leaf, eps=eps, s=s)
    if kernel == "yukawa_drift":
        return W.yukawa_drift_cube(n=n, leaf=leaf, eps=eps, beta=0.5, nrhs=nrhs, s=s)
    raise SystemExit(f"unknown kernel {kernel}")


def cpu_baseline(kernel: str, eps: float, leaf: int, s: int, n_sample: int) -> dict:
    """Time the oracle's factor + solve on a bounded sample of the same workload
    (same kernel, leaf, eps, sampling, point distribution; N = n_sample)."""
    import numpy as np
    from oracle import construct, flops, ulv
    try:
        from threadpoolctl import threadpool_info
        cores = max([t.get("num_threads", 1) for t in threadpool_info()] + [1])
    except Exception:
        cores = len(os.sched_getaffinity(0))
    p = workload(n_sample, kernel, eps, leaf, s)
    h2 = construct.construct(p.points, p.kernel, p.leaf, p.eta, p.eps, p.perm(), p.s_far, p.s_near)
    t0 = time.perf_counter()
    fac = ulv.factor(h2)
    t1 = time.perf_counter()
    b = p.b()
    x, hist = ulv.refine(fac, b, 1e-8, 50)
    t2 = time.perf_counter()
    ff, fs = flops.count_h2(h2, nrhs=1)
    total = ff + fs * len(hist)
    return {"value": total / (t2 - t0) / 1e12, "unit": "TFLOP/s", "cores": int(cores),
            "kind": "oracle",
            "sample": f"{kernel} cube N={n_sample} leaf={leaf} eps={eps} s={s}: oracle factor "
                      f"{t1 - t0:.1f}s + solve/refine {t2 - t1:.1f}s ({len(hist) - 1} refinement "
                      f"steps, residual {hist[-1]:.1e}); canonical flops {total:.3e}"}


def train_rank_model(a, h2):
    """Train the rank predictor on three smaller seeded builds of the same
    workload (2^16 points each); untimed."""
    import workloads as W
    from paper_2502_02395_amd import rank_model
    train_ps = []
    for sd in (100, 101, 102):
        q = workload(1 << 16, a.kernel, a.eps, a.leaf, a.s)
        q.points = W.cube_points(1 << 16, 3, sd)
        train_ps.append(q)
    X, y = rank_model.collect(train_ps)
    model, hist = rank_model.train(X, y, steps=2000, lr=3e-3)
    print(f"[bench] rank model trained on {len(y)} boxes, loss {hist[0]:.3f} -> {hist[-1]:.4f}",
          file=sys.stderr, flush=True)
    return model


def run_path(a, h2, prec: int, sprec: int, model, label: str, mvprec: int = 0) -> dict:
    """Build once (untimed), W warm-up steps, then time K steps of factor +
    solve with the inputs resident in HBM."""
    import torch
    nrhs = getattr(a, "nrhs", 1)
    p = workload(a.n, a.kernel, a.eps, a.leaf, a.s, nrhs)
    t0 = time.perf_counter()
    if a.kernel == "gaussian_batch":
        import numpy as np
        H = h2.build_batched([q.points for q in p], [q.kernel for q in p], a.leaf, 1.0, a.eps,
                             perms=[q.perm() for q in p], s_far=a.s, s_near=a.s, gemm_prec=prec,
                             ir_max_iter=50, ir_tol=a.tol, use_pcg=True, timing=True,
                             use_graph=a.graph, solve_prec=sprec)
        bnp = np.concatenate([q.b() for q in p], axis=0)
        n_total = sum(q.n for q in p)
    else:
        H = h2.build(p.points, p.kernel, p.leaf, p.eta, p.eps, p.perm(), s_far=a.s,
                     s_near=a.s_near, ir_max_iter=100, ir_tol=a.tol, timing=True,
                     gemm_prec=prec, rank_model=model, use_graph=a.graph,
                     use_pcg=not a.stationary, solve_prec=sprec, matvec_prec=mvprec)
        bnp = p.b()
        n_total = p.n
    t_build = time.perf_counter() - t0
    b = torch.from_numpy(bnp).cuda()
    cols_b = b.t().contiguous()
    cols_x = torch.empty_like(cols_b)
    print(f"[bench] {label}: built N={n_total} in {t_build:.1f}s: {H.stats()['levels']} levels",
          file=sys.stderr, flush=True)
    for w in range(a.warmup):
        H.factor()
        s = H.solve_into(cols_b, cols_x)
        if s != h2.OK:
            raise h2.H2Error(s, "h2_solve")
        st = H.stats()
        print(f"[bench] {label} warmup {w}: factor {st['t_factor']:.3f}s solve "
              f"{st['t_solve']:.3f}s ({st['ir_iters']} iterations, residual "
              f"{st['ir_residual']:.1e})", file=sys.stderr, flush=True)
    torch.cuda.synchronize()
    K = a.steps
    t_fac = t_sol = t_pair = 0.0
    t_phase = [0.0] * 9
    t_g, b_g, n_g = [0.0] * 4, [0.0] * 4, [0] * 4
    iters = fp64_mv = 0
    res = 0.0
    t0 = time.perf_counter()
    for k in range(K):
        H.factor()
        st = H.stats()
        t_fac += st["t_factor"]
        t_pair += st["t_pair_gemm"]
        t_phase = [x + y for x, y in zip(t_phase, st["t_factor_phase"])]
        s = H.solve_into(cols_b, cols_x)
        if s != h2.OK:
            raise h2.H2Error(s, "h2_solve")
        st = H.stats()
        t_sol += st["t_solve"]
        for q in range(3):
            t_g[q] += st["t_gather"][q]
            b_g[q] += st["bytes_gather"][q]
            n_g[q] += st["gather_launches"][q]
        t_g[3] += st["t_gather_mv32"]
        b_g[3] += st["bytes_gather_mv32"]
        n_g[3] += st["gather_launches_mv32"]
        iters += st["ir_iters"]
        fp64_mv += st["ir_fp64_matvecs"]
        res = max(res, st["ir_residual"])
    torch.cuda.synchronize()
    dt = time.perf_counter() - t0
    st = H.stats()
    H.close()
    torch.cuda.empty_cache()
    flops_step = st["flops_factor"] + st["flops_solve"] * nrhs * (1 + iters / K)
    # Kernels of the timed steps with their work per launch over their average
    # launch time (HIP events on the launch stream), largest total time first:
    # the neighbour gathers of the substitution and the matvec (HBM-bound; FP64
    # blocks and FP32 copies are separate instances) and the near-pair
    # transform GEMMs of the factorization (MFMA-bound).  A captured
    # factorization is not timed per launch.
    cands = []
    if t_pair > 0:
        tf = st["flops_pair_gemm"] * K / t_pair / 1e12
        kname, peak, mult = PAIR_KERNEL[prec]
        cands.append({"bound": "mfma", "kernel": kname, "achieved": tf * mult,
                      "peak": peak, "unit": "TFLOP/s", "frac": tf * mult / peak,
                      "algorithmic_tflops": tf, "mfma_flops_per_flop": mult,
                      "traffic": None, "launches": st["pair_launches"] * K,
                      "avg_launch_ms": 1e3 * t_pair / K / max(st["pair_launches"], 1),
                      "total_s": t_pair})
    # one right-hand side on BF16 copies: the 16-byte-load chunks (gv16_kernel)
    copies = "gv16_kernel<bf16>" if sprec == h2.PREC_BF16 else "gchunk_kernel<f32>"
    for q, kname in ((0, "gchunk_kernel<f64>"), (1, copies), (2, "greduce_kernel"),
                     (3, "gchunk_kernel<f32> (PCG products)")):
        if n_g[q] == 0:
            continue
        gbs = b_g[q] / max(t_g[q], 1e-30) / 1e9
        cands.append({"bound": "hbm", "kernel": kname, "achieved": gbs, "peak": HBM_PEAK_GBS,
                      "unit": "GB/s", "frac": gbs / HBM_PEAK_GBS,
                      "traffic": None, "launches": n_g[q],
                      "avg_launch_ms": 1e3 * t_g[q] / n_g[q], "bytes_per_launch": b_g[q] / n_g[q],
                      "total_s": t_g[q]})
    cands.sort(key=lambda d: -d["total_s"])
    return {
        "value": flops_step * K / dt / 1e12, "ms_per_step": 1e3 * dt / K, "n_total": n_total,
        "factor_s": t_fac / K, "solve_s": t_sol / K, "ir_iters": iters / K, "residual": res,
        "fp64_matvecs": fp64_mv / K,
        "build_s": t_build, "stats": st, "cands": cands,
        "factor_phase_s": dict(zip(PHASES, [round(x / K, 5) for x in t_phase])),
        "factor_roofline": factor_roofline(st, [x / K for x in t_phase], t_fac / K, prec),
        # the solve's gathers: algorithmic bytes (every stored block and
        # vector slice once per pass) over the whole solve's time
        "solve_roofline": {"bound": "hbm", "gather_bytes": sum(b_g) / K,
                           "s": t_sol / K,
                           "achieved": sum(b_g) / max(t_sol, 1e-30) / 1e9,
                           "peak": HBM_PEAK_GBS, "unit": "GB/s",
                           "frac": sum(b_g) / max(t_sol, 1e-30) / 1e9 / HBM_PEAK_GBS},
    }


def run_graph(a, h2, model) -> dict:
    """The target path's settings with the factorization and the solve's
    substitutions and products captured in hipGraphs (use_graph) and no
    per-launch timing: K steps of factor + solve after W warm-up steps
    (the first of which captures)."""
    import torch
    p = workload(a.n, a.kernel, a.eps, a.leaf, a.s, 1)
    H = h2.build(p.points, p.kernel, p.leaf, p.eta, p.eps, p.perm(), s_far=a.s, s_near=a.s_near,
                 ir_max_iter=100, ir_tol=a.tol, gemm_prec=h2.PREC_BF16X3, rank_model=model,
                 use_graph=True, use_pcg=True, solve_prec=h2.PREC_BF16,
                 matvec_prec=h2.PREC_FP32)
    b = torch.from_numpy(p.b()).cuda()
    cols_b = b.t().contiguous()
    cols_x = torch.empty_like(cols_b)
    for _ in range(max(a.warmup, 1)):
        H.factor()
        if H.solve_into(cols_b, cols_x) != h2.OK:
            raise h2.H2Error(h2.ERR_NOCONV, "h2_solve")
    torch.cuda.synchronize()
    K = a.steps
    iters = 0
    res = 0.0
    t0 = time.perf_counter()
    for _ in range(K):
        H.factor()
        s = H.solve_into(cols_b, cols_x)
        if s != h2.OK:
            raise h2.H2Error(s, "h2_solve")
        st = H.stats()
        iters += st["ir_iters"]
        res = max(res, st["ir_residual"])
    torch.cuda.synchronize()
    dt = time.perf_counter() - t0
    st = H.stats()
    H.close()
    torch.cuda.empty_cache()
    flops_step = st["flops_factor"] + st["flops_solve"] * (1 + iters / K)
    return {"value": flops_step * K / dt / 1e12, "unit": "TFLOP/s", "ms_per_step": 1e3 * dt / K,
            "ir_iters": iters / K, "residual": res, "steps": K,
            "graph": "factor and solve captured", "launch_timing": False}


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=3)
    ap.add_argument("--warmup", type=int, default=1)
    ap.add_argument("--n", type=int, default=1 << 20)
    ap.add_argument("--kernel", default="yukawa",
                    help="yukawa (default) | laplace | laplace_sphere | matern | gaussian_batch "
                         "(64 instances) | yukawa_drift (non-symmetric: the LU variant, "
                         "stationary refinement, FP64)")
    ap.add_argument("--nrhs", type=int, default=1, help="right-hand sides per solve")
    ap.add_argument("--path", default="target", choices=["target", "plain", "custom"],
                    help="target: rank-predicted buffers, split-BF16 transform GEMMs on FP32 "
                         "copies, packed BF16 copies for the substitution and PCG products on "
                         "FP32 copies of the near blocks and couplings (stopped by the FP64 "
                         "operator's residual), timed next to the plain FP64 path (default); "
                         "plain: the FP64 path only; custom: --prec / --solve-prec / --mv-prec / "
                         "--rank-model as given")
    ap.add_argument("--prec", default="fp64", choices=["fp64", "fp32", "bf16", "bf16x3"],
                    help="custom path: precision of the basis-transform and Schur-update GEMMs")
    ap.add_argument("--mv-prec", default="fp64", choices=["fp64", "fp32"],
                    help="custom path: precision of the near blocks and couplings PCG's "
                         "products read (the residual that stops it is the FP64 operator's)")
    ap.add_argument("--solve-prec", default="fp64", choices=["fp64", "fp32", "bf16"],
                    help="custom path: precision of the factor copies the substitution reads "
                         "(the H^2 matvec, the refinement and all arithmetic stay FP64)")
    ap.add_argument("--rank-model", action="store_true",
                    help="custom path: train the rank predictor on smaller seeded builds first "
                         "(untimed) and size the basis buffers with it")
    ap.add_argument("--graph", action="store_true", help="capture the factorization in a hipGraph")
    ap.add_argument("--stationary", action="store_true",
                    help="stationary iterative refinement instead of PCG")
    ap.add_argument("--eps", type=float, default=1e-6)
    ap.add_argument("--leaf", type=int, default=256)
    ap.add_argument("--s", type=int, default=512)
    ap.add_argument("--s-near", type=int, default=0,
                    help="near-field sample size (0: the same as --s)")
    ap.add_argument("--tol", type=float, default=1e-8)
    ap.add_argument("--cpu-sample", type=int, default=16384)
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--no-extras", action="store_true",
                    help="skip the batched-Gaussian timing and the Matern status run")
    ap.add_argument("--calib-copy", action="store_true",
                    help="first run one plain 1 GiB device-to-device copy (the reference for "
                         "FETCH_SIZE / WRITE_SIZE counters)")
    a = ap.parse_args()
    if a.s_near <= 0:
        a.s_near = a.s
    if a.kernel == "yukawa_drift":
        # the LU variant refines by stationary iterations and takes no BF16
        # substitution copies: the target path's settings do not apply, so it
        # defaults to the FP64 path (--path custom --prec bf16x3 --solve-prec
        # fp32 for the precision split)
        if a.path == "target":
            a.path = "plain"
        a.stationary = True
    if a.gpus != 1 or int(os.environ.get("WORLD_SIZE", "1")) != 1:
        print("bench.py runs on one GPU only: the library implements the single-GPU H^2-ULV "
              "path; a distribution over several GPUs is not implemented.", file=sys.stderr)
        sys.exit(2)

    import torch
    from paper_2502_02395_amd import h2
    torch.cuda.set_device(0)
    if a.calib_copy:
        src = torch.ones(1 << 27, dtype=torch.float64, device="cuda")
        dst = torch.empty_like(src)
        dst.copy_(src)
        torch.cuda.synchronize()
        del src, dst
    P = {"fp64": h2.PREC_FP64, "fp32": h2.PREC_FP32, "bf16": h2.PREC_BF16,
         "bf16x3": h2.PREC_BF16X3}
    plain = None
    if a.path == "custom":
        model = train_rank_model(a, h2) if a.rank_model else None
        setting = (a.prec, a.solve_prec, a.rank_model, a.mv_prec)
        r = run_path(a, h2, P[a.prec], P[a.solve_prec], model, "custom", P[a.mv_prec])
    elif a.path == "plain":
        setting = ("fp64", "fp64", False, "fp64")
        r = run_path(a, h2, h2.PREC_FP64, h2.PREC_FP64, None, "plain")
    else:
        plain = run_path(a, h2, h2.PREC_FP64, h2.PREC_FP64, None, "plain fp64")
        model = train_rank_model(a, h2) if a.kernel != "gaussian_batch" else None
        setting = ("bf16x3", "bf16", model is not None, "fp32")
        r = run_path(a, h2, h2.PREC_BF16X3, h2.PREC_BF16, model, "target", h2.PREC_FP32)
    if a.path == "target" and a.kernel == "yukawa" and a.n == 1 << 20:
        for d in r["cands"]:  # traffic was measured on this workload and path
            d["traffic"] = measured_traffic(d["kernel"])
    st = r["stats"]
    K = a.steps
    mixed = setting[0] != "fp64" or setting[1] != "fp64"
    out = {
        "metric": "H2-ULV factor+solve TFLOP/s at N=2^20 (rel. residual <= 1e-8 vs FP64 H2 operator)",
        "value": r["value"], "unit": "TFLOP/s", "n_gpus": 1, "steps": K, "warmup": a.warmup,
        "ms_per_step": r["ms_per_step"], "higher_is_better": True, "scaling": "weak",
        "vs_baseline": None,
        "dtype": {"fp64": "f64+f32" if mixed else "f64", "fp32": "f64+f32", "bf16": "f64+bf16",
                  "bf16x3": "f64+bf16x3"}[setting[0]],
        "data": "synthetic",
        "config": {"workload": a.kernel if a.kernel in ("gaussian_batch", "laplace_sphere")
                   else f"{a.kernel}_cube",
                   "path": a.path, "n": r["n_total"],
                   "dim": 2 if a.kernel == "gaussian_batch" else 3, "leaf": a.leaf,
                   "eta": 1.0, "eps": a.eps, "s_far": a.s, "s_near": a.s_near, "nrhs": a.nrhs,
                   "gemm_prec": setting[0], "solve_prec": setting[1], "rank_model": setting[2],
                   "matvec_prec": setting[3],
                   "graph": a.graph, "rank_fallbacks": st["rank_fallbacks"],
                   "basis_bytes": st["bytes_basis"], "autotuned_lists": st["tuned_lists"],
                   "tile_choice": st["tuned_cfg_hist"], "ir_tol": a.tol, "levels": st["levels"],
                   "root_n": st["root_n"], "max_rank": st["max_rank_seen"],
                   "near_pairs": st["near_pairs"]},
        "factor_s": r["factor_s"], "factor_phase_s": r["factor_phase_s"],
        "factor_roofline": r["factor_roofline"], "solve_roofline": r["solve_roofline"],
        "solve_s": r["solve_s"], "ir_iters": r["ir_iters"], "residual": r["residual"],
        "fp64_matvecs": r["fp64_matvecs"],
        "build_s": r["build_s"], "build_id_s": st["t_build_id"],
        "flops_factor": st["flops_factor"],
        "flops_solve": st["flops_solve"],
        "roofline": r["cands"][0] if r["cands"] else None,
        "roofline_other": r["cands"][1:],
    }
    if plain is not None:
        out["plain_fp64"] = {"value": plain["value"], "ms_per_step": plain["ms_per_step"],
                             "factor_s": plain["factor_s"], "solve_s": plain["solve_s"],
                             "ir_iters": plain["ir_iters"], "residual": plain["residual"],
                             "basis_bytes": plain["stats"]["bytes_basis"],
                             "build_s": plain["build_s"],
                             "build_id_s": plain["stats"]["t_build_id"],
                             "roofline": plain["cands"][0] if plain["cands"] else None}
        out["speedup_vs_plain_fp64"] = plain["ms_per_step"] / r["ms_per_step"]
    if a.path == "target" and a.kernel == "yukawa" and a.n == 1 << 20 and not a.no_extras:
        # the same path with captured factorization and solves, without
        # per-launch timing (beside the timed headline)
        print("[bench] target path, captured", file=sys.stderr, flush=True)
        try:
            out["target_graph"] = run_graph(a, h2, model)
        except h2.H2Error as e:
            out["target_graph"] = {"status": str(e)}
        # the batched configuration (64 independent 2-D Gaussian systems, one
        # handle, factorization captured in a hipGraph; FP64 transforms: these
        # covariance matrices break down under FP32 ones) and the status of
        # the Matern configuration, beside the headline
        import copy
        import torch
        b = copy.copy(a)
        b.kernel, b.leaf, b.eps, b.s, b.s_near, b.graph = "gaussian_batch", 128, 1e-9, 512, 512, True
        b.steps, b.warmup = min(a.steps, 10), 1
        print("[bench] batched Gaussian instances", file=sys.stderr, flush=True)
        try:
            g = run_path(b, h2, h2.PREC_FP64, h2.PREC_FP64, None, "batched")
            out["batched_gaussian"] = {
                "instances": 64, "n_total": g["n_total"], "leaf": 128, "eps": 1e-9, "s": 512,
                "gemm_prec": "fp64", "solve_prec": "fp64", "graph": True, "steps": b.steps,
                "value": g["value"], "unit": "TFLOP/s", "ms_per_step": g["ms_per_step"],
                "factor_s": g["factor_s"], "solve_s": g["solve_s"], "ir_iters": g["ir_iters"],
                "residual": g["residual"]}
        except h2.H2Error as e:
            out["batched_gaussian"] = {"instances": 64, "status": str(e)}
        torch.cuda.empty_cache()
        # the sphere configuration (Laplace, N=65536 on the unit sphere, leaf
        # 256, eps 1e-8, 16 right-hand sides, FP64) and the mixed-precision
        # cube (Yukawa, N=262144, leaf 256, eps 1e-8, 4 right-hand sides,
        # refined to 1e-10 against the FP64 H^2 operator) on reduced-precision
        # transforms
        extra = [("sphere_16rhs", "laplace_sphere", 1 << 16, 16, h2.PREC_FP64, h2.PREC_FP64, 1e-8),
                 ("mixed_4rhs_bf16x3", "yukawa", 1 << 18, 4, h2.PREC_BF16X3, h2.PREC_BF16, 1e-10),
                 ("mixed_4rhs_bf16", "yukawa", 1 << 18, 4, h2.PREC_BF16, h2.PREC_FP32, 1e-10)]
        names = {h2.PREC_FP64: "fp64", h2.PREC_FP32: "fp32", h2.PREC_BF16: "bf16",
                 h2.PREC_BF16X3: "bf16x3"}
        for key, kern, n, nrhs, gp, sp, tol in extra:
            c = copy.copy(a)
            c.kernel, c.n, c.nrhs, c.leaf, c.eps, c.s, c.s_near, c.tol = kern, n, nrhs, 256, 1e-8, 256, 256, tol
            c.steps, c.warmup, c.graph = min(a.steps, 3), 1, False
            print(f"[bench] {key}", file=sys.stderr, flush=True)
            try:
                g = run_path(c, h2, gp, sp, None, key)
                out[key] = {"workload": kern, "n": n, "nrhs": nrhs, "leaf": 256, "eps": 1e-8,
                            "s": 256, "gemm_prec": names[gp], "solve_prec": names[sp],
                            "ir_tol": tol, "steps": c.steps, "value": g["value"],
                            "unit": "TFLOP/s", "ms_per_step": g["ms_per_step"],
                            "factor_s": g["factor_s"], "solve_s": g["solve_s"],
                            "ir_iters": g["ir_iters"], "residual": g["residual"],
                            "build_s": g["build_s"], "max_rank": g["stats"]["max_rank_seen"]}
            except h2.H2Error as e:
                out[key] = {"workload": kern, "n": n, "nrhs": nrhs, "status": str(e)}
            torch.cuda.empty_cache()
        # the LU variant: the non-symmetric drift kernel (beta 0.5) on the
        # cube, N=262144, leaf 256, eps 1e-6, 512-point samples, stationary
        # refinement to 1e-8 against the FP64 H^2 operator; FP64, and with
        # split-BF16 transforms and FP32 substitution copies
        for key, gp, sp in (("lu_drift", h2.PREC_FP64, h2.PREC_FP64),
                            ("lu_drift_bf16x3", h2.PREC_BF16X3, h2.PREC_FP32)):
            c = copy.copy(a)
            c.kernel, c.n, c.nrhs, c.leaf, c.eps, c.s, c.s_near, c.tol = "yukawa_drift", 1 << 18, 1, 256, 1e-6, 512, 512, 1e-8
            c.steps, c.warmup, c.graph, c.stationary = min(a.steps, 3), 1, False, True
            print(f"[bench] {key}", file=sys.stderr, flush=True)
            try:
                g = run_path(c, h2, gp, sp, None, key)
                out[key] = {"workload": "yukawa_drift_cube", "beta": 0.5, "n": c.n, "nrhs": 1,
                            "leaf": 256, "eps": 1e-6, "s": 512, "gemm_prec": names[gp],
                            "solve_prec": names[sp], "refinement": "stationary", "ir_tol": 1e-8,
                            "steps": c.steps, "value": g["value"], "unit": "TFLOP/s",
                            "ms_per_step": g["ms_per_step"], "factor_s": g["factor_s"],
                            "solve_s": g["solve_s"], "ir_iters": g["ir_iters"],
                            "residual": g["residual"], "build_s": g["build_s"],
                            "max_rank": g["stats"]["max_rank_seen"],
                            "lu_variant": g["stats"]["lu_variant"],
                            "factor_phase_s": g["factor_phase_s"]}
            except h2.H2Error as e:
                out[key] = {"workload": "yukawa_drift_cube", "n": c.n, "status": str(e)}
            torch.cuda.empty_cache()
        print("[bench] Matern configuration status", file=sys.stderr, flush=True)
        out["matern_status"] = []
        for n in (1 << 20, 1 << 18):  # the configuration, and a size that fits
            try:
                out["matern_status"].append(matern_status(h2, n))
            except h2.H2Error as e:
                out["matern_status"].append({"workload": "matern_cube", "n": n, "status": str(e)})
            torch.cuda.empty_cache()
    if not a.no_cpu_baseline and a.kernel != "gaussian_batch":
        print("[bench] timing the CPU oracle on a bounded sample", file=sys.stderr, flush=True)
        out["cpu_baseline"] = cpu_baseline(a.kernel, a.eps, a.leaf, a.s, a.cpu_sample)
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
