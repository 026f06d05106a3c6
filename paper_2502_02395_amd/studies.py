"""Single-node studies on synthetic geometry, after the paper's Section 6
scaling and parameter studies (the sphere-surface family of Section 6.2;
the paper's plotted values are not available as numbers, so these are
measurements of this library only):

  scaling  -- build, factor and solve time, factor TFLOP/s and the number of
              near (dense, non-zero) and far blocks vs N (O(N) behaviour);
  eta      -- the flop counts of the construction's pre-factorization and
              of the factorization (Fig. 17), near / far blocks, ranks and
              times vs the admissibility eta at a fixed N;
  hss      -- HSS (eta = 0, weak admissibility) vs H^2 (eta = 1) at fixed
              ranks without far-field sampling (Figs. 18-19): the unrefined
              solve's error against the dense solve, and time to solution;
  prefactor -- the pre-factorization of the construction (Section 3.5):
              exact near-sample solve vs Gauss-Seidel sweeps, on the Yukawa
              cube of the headline configuration (build time, ranks, PCG
              iterations and residual).

    python -m paper_2502_02395_amd.studies [scaling|eta|hss|prefactor|all] [--max-n N]

Every line printed is one JSON record.  The dense reference of the hss
study is the FP64 solve of the kernel matrix formed with plain torch
operations on the GPU (N = 8192), not the library.
"""
from __future__ import annotations

import argparse
import json
import sys
import time


def _run(h2, p, gemm_prec, solve_prec, nrhs=1, refine=True, gs_sweeps=0):
    import numpy as np
    import torch
    t0 = time.perf_counter()
    kw = dict(s_far=p.s_far, s_near=p.s_near, gemm_prec=gemm_prec, solve_prec=solve_prec,
              gs_sweeps=gs_sweeps)
    if refine:
        kw.update(ir_max_iter=100, ir_tol=1e-8, use_pcg=True)
    H = h2.build(p.points, p.kernel, p.leaf, p.eta, p.eps, p.perm(), **kw)
    t_build = time.perf_counter() - t0
    b = torch.from_numpy(p.b()[:, :nrhs].copy()).cuda()
    H.factor()          # warm-up (first-use costs)
    H.solve(b)
    torch.cuda.synchronize()
    H.factor()
    x = H.solve(b)
    torch.cuda.synchronize()
    st = H.stats()
    _, ranks, ms, _ = H.structure()
    rec = {"n": p.n, "leaf": p.leaf, "eta": p.eta, "eps": p.eps, "levels": st["levels"],
           "near_pairs": st["near_pairs"], "far_pairs": st["far_pairs"],
           "leaf_near_blocks": st["leaf_near_blocks"], "max_rank": int(ranks.max()),
           "mean_rank": float(ranks.mean()), "root_n": st["root_n"],
           "build_s": t_build, "factor_s": st["t_factor"], "solve_s": st["t_solve"],
           "flops_factor": st["flops_factor"],
           "factor_tflops": st["flops_factor"] / max(st["t_factor"], 1e-12) / 1e12,
           "ir_iters": st["ir_iters"], "residual": st["ir_residual"]}
    return H, b, x, rec


def scaling(h2, max_n: int, prec):
    import workloads as W
    n = 1 << 14
    while n <= max_n:
        p = W.laplace_sphere(n=n, leaf=256, eps=1e-8, nrhs=1)
        H, _, _, rec = _run(h2, p, prec, prec)
        H.close()
        rec["study"] = "scaling"
        print(json.dumps(rec), flush=True)
        n *= 2


def eta_sweep(h2, n: int, prec):
    """Fig. 17: FP64 operation counts of the construction's pre-factorization
    (Section 3.5) and of the ULV factorization vs eta; the counts come from
    the build, the times from a factor + solve where the factorization holds."""
    import workloads as W
    for eta in (0.0, 0.5, 1.0, 1.5, 2.0, 3.0):
        p = W.laplace_sphere(n=n, leaf=256, eps=1e-8, eta=eta, nrhs=1)
        H = h2.build(p.points, p.kernel, p.leaf, p.eta, p.eps, p.perm(), s_far=p.s_far,
                     s_near=p.s_near, gemm_prec=prec, solve_prec=prec, ir_max_iter=100,
                     ir_tol=1e-8, use_pcg=True)
        st = H.stats()
        rec = {"study": "eta", "n": p.n, "leaf": p.leaf, "eta": eta, "eps": p.eps,
               "s": p.s_far, "near_pairs": st["near_pairs"], "far_pairs": st["far_pairs"],
               "leaf_near_blocks": st["leaf_near_blocks"], "max_rank": st["max_rank_seen"],
               "flops_prefactor": st["flops_prefactor"], "flops_factor": st["flops_factor"],
               "prefactor_share": st["flops_prefactor"] /
               (st["flops_prefactor"] + st["flops_factor"]), "build_s": st["t_build"]}
        try:
            import torch
            b = torch.from_numpy(p.b()).cuda()
            H.factor()
            H.solve(b)
            H.factor()
            H.solve(b)
            st = H.stats()
            rec.update({"factor_s": st["t_factor"], "solve_s": st["t_solve"],
                        "ir_iters": st["ir_iters"], "residual": st["ir_residual"]})
        except h2.H2Error as e:  # e.g. a Cholesky breakdown: recorded, not fatal
            rec["error"] = str(e)
        H.close()
        print(json.dumps(rec), flush=True)


def hss_vs_h2(h2, ranks=(25, 50, 100, 200, 400)):
    """Figs. 18-19: HSS (eta = 0) vs H^2 (eta = 1) at fixed ranks, N = 8192,
    leaf 512, every far-field point used (no far sampling; near samples of
    2048 points): the unrefined solve's error against the dense FP64 solve,
    and the time to solution (factor + solve)."""
    import torch
    import workloads as W
    p0 = W.laplace_sphere(n=8192, leaf=512, eps=0.0, eta=1.0, nrhs=1, s=-1)
    X = torch.from_numpy(p0.points).cuda()
    A = 1.0 / (torch.cdist(X, X) + p0.kernel.delta)
    b = torch.from_numpy(p0.b()).cuda()
    xd = torch.linalg.solve(A, b)
    del A
    torch.cuda.empty_cache()
    for eta in (0.0, 1.0):
        for r in ranks:
            rec = {"study": "hss" if eta == 0.0 else "h2", "n": p0.n, "leaf": 512, "eta": eta,
                   "max_rank": r, "s_far": -1, "s_near": 2048}
            try:
                H = h2.build(p0.points, p0.kernel, 512, eta, 0.0, p0.perm(), s_far=-1,
                             s_near=2048, max_rank=r)
                st = H.stats()
                rec.update({"max_rank_seen": st["max_rank_seen"], "root_n": st["root_n"],
                            "near_pairs": st["near_pairs"], "far_pairs": st["far_pairs"],
                            "flops_factor": st["flops_factor"], "build_s": st["t_build"]})
                H.factor()
                x = H.solve(b)
                H.factor()
                x = H.solve(b)
                torch.cuda.synchronize()
                st = H.stats()
                rec.update({"factor_s": st["t_factor"], "solve_s": st["t_solve"],
                            "time_to_solution_s": st["t_factor"] + st["t_solve"],
                            "rel_err_vs_dense": float(torch.linalg.norm(x - xd) /
                                                      torch.linalg.norm(xd))})
                H.close()
            except h2.H2Error as e:
                rec["error"] = str(e)
            print(json.dumps(rec), flush=True)


def prefactor(h2, n: int):
    import workloads as W
    for sweeps in (0, 1, 2, 4):
        p = W.yukawa_cube(n=n, leaf=256, eps=1e-6, nrhs=1, s=512)
        try:
            H, _, _, rec = _run(h2, p, h2.PREC_FP32, h2.PREC_FP32, gs_sweeps=sweeps)
            H.close()
        except h2.H2Error as e:
            rec = {"n": p.n, "error": str(e)}
        rec["study"] = "prefactor"
        rec["gs_sweeps"] = sweeps
        print(json.dumps(rec), flush=True)


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("study", nargs="?", default="all",
                    choices=["scaling", "eta", "hss", "prefactor", "all"])
    ap.add_argument("--max-n", type=int, default=1 << 19)
    ap.add_argument("--eta-n", type=int, default=1 << 18)
    ap.add_argument("--prec", default="fp32", choices=["fp64", "fp32"],
                    help="transform and substitution precision of the scaling and eta runs")
    a = ap.parse_args()
    import torch
    from paper_2502_02395_amd import h2
    torch.cuda.set_device(0)
    prec = h2.PREC_FP32 if a.prec == "fp32" else h2.PREC_FP64
    if a.study in ("scaling", "all"):
        scaling(h2, a.max_n, prec)
    if a.study in ("eta", "all"):
        eta_sweep(h2, a.eta_n, prec)
    if a.study in ("hss", "all"):
        hss_vs_h2(h2)
    if a.study in ("prefactor", "all"):
        prefactor(h2, 1 << 20)


if __name__ == "__main__":
    sys.exit(main())
