"""Benchmark: Newton-GMRES time-to-1e-8 (mixed precision and FP64) on one MI355X.

A step is one complete mixed-precision solve of the CNP DG system on the
16^3-hex, p = 2, three-ion cube (vortex flow, Pe = 1e3) from the paper's
initial guess to ||R|| <= 1e-8 ||R_0||: residual, block assembly, BILU(0)
factorisation of every multigrid level of the concentration blocks and their
Galerkin operators, the potential multigrid set-up, FGMRES with the
block-triangular preconditioner (one geometric-multigrid V-cycle per
concentration block with ILU(0) smoothing, the potential V-cycle, coupling
applies; Sec. 4.1's second approach, `--conc-pc bilu` for its first) and FP32
Jacobian applies under FP64 residuals and refinement, backtracking line
search.  The seeded synthetic inputs are resident on the GPU before timing
starts.

One JSON line is printed.  Besides the contract fields it carries the FP64
time-to-solution on the same input, the adjoint-gradient time, the
Jacobian-apply bandwidth on the largest channel (128x32x16 hexes, p = 3,
12.6M DOFs), mixed and FP64 time-to-solution on the two channels (64x16x8 and
128x32x16 hexes, p = 3) with an adjoint on the larger, the two
concentration-block preconditioners (block ILU(0) and geometric multigrid) on
the p = 1 channel of the same size (256x64x32 hexes), the roofline of the
dominant kernel of the timed solve and the CPU oracle baseline.
"""
from __future__ import annotations

import argparse
import hashlib
import json
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

PEAK_HBM_GBS = 8000.0          # MI355X HBM3E
PEAK_FP32_TFLOPS = 157.3       # vector FP32 (published; counts packed FP32 FMAs)
PEAK_FP32_UNPACKED_TFLOPS = 78.6  # 256 CUs x 64 lanes x 2 flops x 2.4 GHz (packed FP32 disabled at compile time)
PEAK_FP64_TFLOPS = 78.6        # vector FP64
METRIC = "Newton-GMRES time-to-1e-8 (FP64 vs mixed); Jacobian-apply HBM GB/s"
REPS = 5  # repetitions behind every median of the extra legs


def parse():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=5)
    ap.add_argument("--warmup", type=int, default=1)
    ap.add_argument("--workload", default="cfg2")
    ap.add_argument("--apply-workload", default="cfg5")
    ap.add_argument("--no-cpu", action="store_true", help="skip the CPU oracle baseline")
    ap.add_argument("--no-extra", action="store_true",
                    help="skip the FP64, adjoint, large-apply and channel-solve legs")
    ap.add_argument("--only-apply", action="store_true", help="run only the large Jacobian-apply leg")
    ap.add_argument("--only-gmg", action="store_true",
                    help="run only the concentration-preconditioner comparison on the p = 1 channel")
    ap.add_argument("--conc-pc", default="gmg", choices=("gmg", "bilu"),
                    help="concentration-block preconditioner of the timed solve (Sec. 4.1): one geometric-"
                         "multigrid V-cycle with one ILU(0) smoothing step per side, or one block-ILU(0) solve")
    ap.add_argument("--apply-variants", default="",
                    help="comma-separated launch variants of the Jacobian apply to time (A/B), then exit")
    return ap.parse_args()


def log(msg):
    print(msg, file=sys.stderr, flush=True)


# ---- algorithmic byte and flop counts -------------------------------------------
def _couplings(cfg):
    """(elements, block size, lower-neighbour couplings) of the element graph."""
    import numpy as np
    n = np.array(cfg.n[: cfg.dim])
    E = int(np.prod(n))
    nb = (cfg.p + 1) ** cfg.dim
    n_low = int(sum(E // n[a] * (n[a] - 1) for a in range(cfg.dim)))
    return E, nb, n_low


def ilu_sweep_bytes(cfg, word, backward=False):
    """Algorithmic HBM bytes of one BILU(0) sweep over all concentration blocks
    (one launch of the dataflow sweep): forward, every element reads its D^-1
    block, the scaled coupling block of each lower neighbour, its right-hand
    side and the lower neighbours' solution values, and writes its solution;
    backward, the upper coupling blocks, the forward result and the upper
    neighbours' values."""
    E, nb, n_low = _couplings(cfg)
    blocks = n_low if backward else E + n_low
    per_field = (blocks * nb * nb + (2 * E + n_low) * nb) * word
    return float((cfg.m - 1) * per_field)


def _levels(cfg):
    return int(sum(cfg.n[: cfg.dim])) - cfg.dim + 1


def ilu_factor_bytes(cfg):
    """Algorithmic HBM bytes of one launch of the BILU(0) factorisation (one
    hyperplane level), averaged over the levels: every element reads its
    diagonal and coupling blocks (FP64) and, for the Schur update, the scaled
    upper block of each lower neighbour; it writes D^-1 and its scaled
    coupling blocks in FP64 and FP32 (both concentration fields)."""
    E, nb, n_low = _couplings(cfg)
    reads = (E + 2 * n_low + n_low) * nb * nb * 8
    writes = (E + 2 * n_low) * nb * nb * (8 + 4)
    return float((cfg.m - 1) * (reads + writes)) / _levels(cfg)


def ilu_factor_flops(cfg):
    """FP64 operations of one launch of the factorisation, averaged over the
    levels: per element a Schur product per lower neighbour, the inversion of
    D_i (Gauss-Jordan, 2 n_b^3) and the scaling of every coupling block, each
    2 n_b^3."""
    E, nb, n_low = _couplings(cfg)
    return float((cfg.m - 1) * (n_low + E + 2 * n_low) * 2 * nb ** 3) / _levels(cfg)


def cheb_blk_bytes(cfg, word):
    """Algorithmic HBM bytes per launch of the fused Chebyshev step on the
    element-block level, averaged over the four launches of one V-cycle: the
    first (zero initial guess) reads D^-1 and the right-hand side and writes
    x; the other three read every block of the potential block row (diagonal
    and couplings) plus D^-1 and their vectors once (14 vectors of N_f values
    over the four launches)."""
    E, nb, n_low = _couplings(cfg)
    blocks = E * nb * nb + 3 * (2 * E + 2 * n_low) * nb * nb
    vectors = 14 * E * nb
    return float((blocks + vectors) * word) / 4.0


def japply_bytes(N, word):
    """Algorithmic bytes of one Jacobian apply: the input vector and the
    linearisation state are read once and the output written once."""
    return 3 * N * word


def japply_flops(cfg):
    """Floating-point operations of the sum-factorised contractions of one
    Jacobian apply as the kernel performs them (2 per multiply-add): the state
    is tabulated at the quadrature points once per linearisation, so per
    element one interpolation of the input and one integration; per element
    face two trace evaluations of the input (own and neighbour) and one face
    integration.  The pointwise flux arithmetic is not counted."""
    import numpy as np
    d, p, m = cfg.dim, cfg.p, cfg.m
    nn, nq = p + 1, p + 2
    E = int(np.prod(cfg.n[: d]))
    if d == 3:
        vol = m * (2 * nn ** 3 * nq + 3 * nn ** 2 * nq ** 2 + 4 * nn * nq ** 3)
        trace = m * (nn ** 3 + 2 * nn * nn * nq + 2 * nq * nq * nn)
        finteg = m * (2 * nn * nq * nq + 2 * nn * nn * nq + nn ** 3)
    else:
        vol = m * (2 * nn * nn * nq + 3 * nn * nq * nq)
        trace = m * (nn * nn + 2 * nn * nq)
        finteg = m * (2 * nn * nq + nn * nn)
    per_elem = 2 * vol + 2 * d * (2 * trace + finteg)
    return 2.0 * per_elem * E


def source_hash(*names):
    h = hashlib.sha256()
    for n in names:
        with open(os.path.join(ROOT, "paper_2112_09271_amd", "csrc", n), "rb") as f:
            h.update(f.read())
    return h.hexdigest()[:16]


def profile_ranking(workload):
    """The dominant kernel family of this workload's timed solve by total kernel
    time in the committed rocprofv3 statistics, with its average duration."""
    path = os.path.join(ROOT, "profiles", "dominant_kernels.json")
    try:
        with open(path) as f:
            return json.load(f).get(workload)
    except (OSError, ValueError):
        return None


def measured_traffic(kernel_key, src_hash):
    """HBM bytes per launch from the committed rocprofv3 counter summary, or
    None when it is missing or was taken on different kernel sources."""
    path = os.path.join(ROOT, "profiles", "hbm_traffic.json")
    try:
        with open(path) as f:
            rec = json.load(f).get(kernel_key)
    except (OSError, ValueError):
        return None
    if not rec or rec.get("source_hash") != src_hash:
        return None
    return rec.get("bytes_per_launch")


# ---- legs ---------------------------------------------------------------------------
def cpu_baseline(gpu_same_input_s):
    """The oracle (NumPy/SciPy, SuperLU) solving the same physics on a bounded
    sample: the 4^3-element cube (1/64 of the elements; the 16^3 cube's direct
    solves do not finish in minutes), to the same 1e-8, with all host threads;
    the GPU's mixed solve of that same sample is reported beside it."""
    from threadpoolctl import threadpool_info

    from oracle import solve as osolve
    from oracle.dg import DG
    from oracle.problem import Problem as OProblem
    from workload import boundary_data, get_config
    cfg = get_config("cfg2t")
    od = DG(OProblem(cfg, boundary_data(cfg)))
    t0 = time.perf_counter()
    x, hist = osolve.newton(od, tol=1e-8)
    dt = time.perf_counter() - t0
    threads = max([i.get("num_threads", 1) for i in threadpool_info()] + [1])
    return {"value": dt, "unit": "s", "cores": threads, "kind": "oracle",
            "sample": f"oracle Newton + SuperLU to 1e-8 on the same physics with 4^3 elements "
                      f"({od.N} DOFs, 1/64 of the workload's elements; {len(hist) - 1} Newton steps); "
                      "SuperLU factorisation is single-threaded, BLAS parts use the listed threads",
            "gpu_mixed_same_input_s": gpu_same_input_s,
            "oracle_over_gpu_same_input": dt / gpu_same_input_s if gpu_same_input_s else None}


def oracle_operator_timings(names=("cfg2", "cfg3", "cfg5"), reps=3):
    """The oracle's vectorised residual and Jacobian apply (NumPy, full tabulated
    basis matrices) on the bench's operator inputs, median of `reps` after one
    warm-up, with one BLAS thread and with all host threads."""
    from threadpoolctl import threadpool_info, threadpool_limits

    from oracle.dg import DG
    from oracle.problem import Problem as OProblem
    from workload import boundary_data, get_config, random_state, random_vector
    import numpy as np
    allt = max([i.get("num_threads", 1) for i in threadpool_info()] + [1])
    out = {"cores_all": allt, "cpu": _cpu_model()}
    for name in names:
        cfg = get_config(name)
        od = DG(OProblem(cfg, boundary_data(cfg)))
        x, v = random_state(cfg), random_vector(cfg)
        rec = {"dofs": od.N}
        for label, lim in (("1_thread", 1), ("all_threads", allt)):
            with threadpool_limits(limits=lim):
                for what, fn in (("residual_s", lambda: od.residual(x)), ("jac_apply_s", lambda: od.jac_apply(x, v))):
                    fn()
                    ts = []
                    for _ in range(reps):
                        t0 = time.perf_counter()
                        fn()
                        ts.append(time.perf_counter() - t0)
                    rec[f"{what}_{label}"] = float(np.median(ts))
        out[name] = rec
        log(f"[bench] oracle {name}: residual {rec['residual_s_1_thread']:.2f}/{rec['residual_s_all_threads']:.2f} s, "
            f"J apply {rec['jac_apply_s_1_thread']:.2f}/{rec['jac_apply_s_all_threads']:.2f} s (1/all threads)")
        del od
    return out


def _cpu_model():
    try:
        with open("/proc/cpuinfo") as f:
            for line in f:
                if line.startswith("model name"):
                    return line.split(":", 1)[1].strip()
    except OSError:
        pass
    return None


def apply_bandwidth(name, reps=20):
    """Jacobian apply (FP32 and FP64) on the largest channel, timed with HIP
    events on the stream the kernels run on, rotating 4 input/output pairs."""
    import torch

    from paper_2112_09271_amd.dgnp import DGNP_F32, DGNP_F64, DGNP_STATE_APPLY_ONLY, Problem
    from workload import boundary_data, get_config, random_state, random_vector
    cfg = get_config(name)
    prob = Problem(cfg, boundary_data(cfg))
    x = torch.as_tensor(random_state(cfg), device="cuda")
    out = {"workload": f"{cfg.name}: {cfg.note}", "dofs": prob.N}
    for prec, tag, word, dt_ in ((DGNP_F32, "f32", 4, torch.float32), (DGNP_F64, "f64", 8, torch.float64)):
        prob.set_state(x, prec=prec | DGNP_STATE_APPLY_ONLY)
        vs = [torch.as_tensor(random_vector(cfg, 100 + i), device="cuda").to(dt_) for i in range(4)]
        ys = [torch.empty_like(v) for v in vs]
        from paper_2112_09271_amd import dgnp as D
        st = torch.cuda.current_stream().cuda_stream
        for i in range(3):
            D.dgnp_jacobian_apply(prob.ctx, vs[i % 4].data_ptr(), ys[i % 4].data_ptr(), prec, 0, st)
        e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        torch.cuda.synchronize()
        e0.record()
        for i in range(reps):
            D.dgnp_jacobian_apply(prob.ctx, vs[i % 4].data_ptr(), ys[i % 4].data_ptr(), prec, 0, st)
        e1.record()
        torch.cuda.synchronize()
        sec = e0.elapsed_time(e1) * 1e-3 / reps
        gbs = japply_bytes(prob.N, word) / sec / 1e9
        tfl = japply_flops(cfg) / sec / 1e12
        out[tag] = {"us_per_apply": 1e6 * sec, "GBps": gbs, "hbm_frac": gbs / PEAK_HBM_GBS,
                    "contraction_TFLOPs": tfl,
                    "alu_frac": tfl / (PEAK_FP32_TFLOPS if word == 4 else PEAK_FP64_TFLOPS)}
        if word == 4:  # without packed FP32 instructions one lane retires one FP32 FMA per cycle
            out[tag]["alu_frac_unpacked_issue"] = tfl / PEAK_FP32_UNPACKED_TFLOPS
        log(f"[bench] J apply {tag} on {cfg.name}: {1e6 * sec:.1f} us, {gbs:.0f} GB/s, {tfl:.2f} TFLOP/s")
        # the coupling block of Eq. P2 (potential rows, concentration input)
        ycs = [torch.empty(prob.Nf, dtype=dt_, device="cuda") for _ in range(4)]
        for i in range(3):
            D.dgnp_coupling_apply(prob.ctx, vs[i % 4].data_ptr(), ycs[i % 4].data_ptr(), prec, st)
        torch.cuda.synchronize()
        e0.record()
        for i in range(reps):
            D.dgnp_coupling_apply(prob.ctx, vs[i % 4].data_ptr(), ycs[i % 4].data_ptr(), prec, st)
        e1.record()
        torch.cuda.synchronize()
        csec = e0.elapsed_time(e1) * 1e-3 / reps
        out[tag]["coupling_us_per_apply"] = 1e6 * csec
        out[tag]["coupling_over_full_apply"] = csec / sec
    prob.close()
    return out


def channel_solves(names):
    """Time-to-solution on the channel configurations: mixed and FP64 solves from
    the initial guess to 1e-8 (medians of REPS runs after one untimed run of each), their agreement,
    on the largest one a mixed-precision adjoint gradient, and the mixed solve
    with the other potential-block multigrids."""
    import torch

    from paper_2112_09271_amd.dgnp import DGNP_F32, DGNP_F64, DGNP_PHIMG_P, DGNP_PHIMG_Q1, Problem
    from workload import boundary_data, get_config
    out = {}
    for name in names:
        cfg = get_config(name)
        prob = Problem(cfg, boundary_data(cfg))
        rec = {"workload": f"{cfg.name}: {cfg.note}", "dofs": prob.N}

        def run(prec):
            torch.cuda.synchronize()
            t0 = time.perf_counter()
            x, st = prob.solve(rtol=cfg.newton_tol, prec=prec)
            torch.cuda.synchronize()
            if st.status != 0:
                raise RuntimeError(f"{name} solve failed with status {st.status}")
            return x, st, time.perf_counter() - t0

        import numpy as np
        run(DGNP_F32)
        runs32 = [run(DGNP_F32) for _ in range(REPS)]
        x32, st32 = runs32[-1][0], runs32[-1][1]
        t32 = float(np.median([r[2] for r in runs32]))
        del runs32[:-1]
        run(DGNP_F64)
        runs64 = [run(DGNP_F64) for _ in range(REPS)]
        x64, st64 = runs64[-1][0], runs64[-1][1]
        t64 = float(np.median([r[2] for r in runs64]))
        del runs64
        rec.update({"mixed_s": t32, "fp64_s": t64, "mixed_speedup_vs_fp64": t64 / t32,
                    "newton_its": st32.newton_its, "fgmres_its_mixed": st32.lin_its_total,
                    "fgmres_its_fp64": st64.lin_its_total, "setup_s_mixed": st32.t_setup,
                    "krylov_s_mixed": st32.t_krylov,
                    "mixed_vs_fp64_rel_l2": (x64 - x32).norm().item() / x64.norm().item()})
        if name == names[-1]:
            ta = []
            for _ in range(3):
                torch.cuda.synchronize()
                t0 = time.perf_counter()
                prob.adjoint(x32, prec=DGNP_F32, rtol=1e-8)
                torch.cuda.synchronize()
                ta.append(time.perf_counter() - t0)
            rec["adjoint_s"] = float(np.median(ta))
        log(f"[bench] {name}: mixed {t32:.3f}s fp64 {t64:.3f}s ({st32.lin_its_total} / {st64.lin_its_total} its)")
        prob.close()
        del x64
        torch.cuda.empty_cache()
        # the same mixed solve with the other potential multigrids (the default at
        # p = 3 is p-multigrid with the Galerkin p = 1 level)
        rec["phi_mg"] = "PG (p-multigrid, Galerkin p = 1 level)" if cfg.p >= 3 else "Q1"
        rec["alternatives"] = {}
        for label, mode in (("Q1", DGNP_PHIMG_Q1), ("P", DGNP_PHIMG_P)):
            if label == "Q1" and cfg.p < 3:
                continue
            prob = Problem(cfg, boundary_data(cfg), phi_mg=mode)
            run(DGNP_F32)
            xp, stp, tp = run(DGNP_F32)
            rec["alternatives"][label] = {
                "mixed_s": tp, "fgmres_its": stp.lin_its_total, "setup_s": stp.t_setup, "krylov_s": stp.t_krylov,
                "vs_default_rel_l2": (xp - x32).norm().item() / x32.norm().item()}
            log(f"[bench] {name}: phi_mg {label} mixed {tp:.3f}s ({stp.lin_its_total} its)")
            prob.close()
            del xp
            torch.cuda.empty_cache()
        del x32
        out[name] = rec
    return out


def conc_pc_solves(names, reps=3):
    """The p = 1 channel with the two concentration-block preconditioners of
    Sec. 4.1: one block-ILU(0) solve (the one-subdomain ASM) against one
    geometric-multigrid V-cycle (1 and 2 ILU(0) Richardson steps per side);
    mixed-precision time-to-1e-8 (median of `reps` after one untimed run),
    iterations, set-up / Krylov split and agreement with the BILU solution."""
    import numpy as np
    import torch

    from paper_2112_09271_amd.dgnp import DGNP_CPC_GMG, DGNP_F32, Problem
    from workload import boundary_data, get_config
    out = {}
    for name in names:
        cfg = get_config(name)
        data = boundary_data(cfg)
        rec = {"workload": f"{cfg.name}: {cfg.note}"}
        x_ref = None
        for label, kw in (("bilu", {}), ("gmg_nu1", {"conc_pc": DGNP_CPC_GMG, "gmg_nu": 1}),
                          ("gmg_nu2", {"conc_pc": DGNP_CPC_GMG, "gmg_nu": 2})):
            prob = Problem(cfg, data, **kw)
            rec["dofs"] = prob.N

            def run():
                torch.cuda.synchronize()
                t0 = time.perf_counter()
                x, st = prob.solve(rtol=cfg.newton_tol, prec=DGNP_F32)
                torch.cuda.synchronize()
                if st.status != 0:
                    raise RuntimeError(f"{name} {label} solve failed with status {st.status}")
                return x, st, time.perf_counter() - t0

            run()
            runs = [run() for _ in range(reps)]
            x, st = runs[-1][0], runs[-1][1]
            r = {"mixed_s": float(np.median([q[2] for q in runs])), "newton_its": st.newton_its,
                 "fgmres_its": st.lin_its_total, "setup_s": st.t_setup, "krylov_s": st.t_krylov}
            if x_ref is None:
                x_ref = x.clone()
            else:
                r["vs_bilu_rel_l2"] = (x - x_ref).norm().item() / x_ref.norm().item()
            rec[label] = r
            log(f"[bench] {name} {label}: mixed {r['mixed_s']:.3f}s ({st.lin_its_total} its)")
            del runs, x
            prob.close()
            torch.cuda.empty_cache()
        rec["gmg_nu1_speedup_vs_bilu"] = rec["bilu"]["mixed_s"] / rec["gmg_nu1"]["mixed_s"]
        out[name] = rec
    return out


def copy_bandwidth(mib=512, reps=20):
    """GB/s (read + write bytes) of a device-to-device copy of `mib` MiB, timed
    with events over `reps` copies after one untimed copy."""
    import torch
    n = mib * (1 << 20) // 4
    a = torch.ones(n, dtype=torch.float32, device="cuda")
    b = torch.empty_like(a)
    b.copy_(a)
    e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    torch.cuda.synchronize()
    e0.record()
    for _ in range(reps):
        b.copy_(a)
    e1.record()
    torch.cuda.synchronize()
    sec = e0.elapsed_time(e1) / 1e3 / reps
    del a, b
    return 2.0 * n * 4 / sec / 1e9


def main():
    args = parse()
    if args.gpus != 1:
        print(f"bench.py measures one GPU only (asked for --gpus {args.gpus}): the library has no "
              "multi-GPU path; run with --gpus 1", file=sys.stderr)
        sys.exit(2)
    import numpy as np
    import torch

    from paper_2112_09271_amd.dgnp import DGNP_CPC_GMG, DGNP_F32, DGNP_F64, Problem
    from workload import boundary_data, get_config

    torch.cuda.set_device(0)
    if args.only_apply:
        print(json.dumps({"jacobian_apply": apply_bandwidth(args.apply_workload)}), flush=True)
        return
    if args.only_gmg:
        print(json.dumps({"concentration_preconditioners": conc_pc_solves(["ch256p1"])}), flush=True)
        return
    if args.apply_variants:
        res = {}
        for wl in args.apply_workload.split(","):
            for var in args.apply_variants.split(","):
                os.environ["DGNP_JAC_VARIANT"] = var
                res[f"{wl}:{var}"] = apply_bandwidth(wl)
        print(json.dumps({"jacobian_apply_variants": res}), flush=True)
        return
    cfg = get_config(args.workload)
    pc_kw = {"conc_pc": DGNP_CPC_GMG, "gmg_nu": 1} if args.conc_pc == "gmg" else {}
    pc_name = "GMG V-cycle, 1 ILU(0) step per side" if args.conc_pc == "gmg" else "BILU(0)"
    prob = Problem(cfg, boundary_data(cfg), **pc_kw)
    log(f"[bench] workload {cfg.name}: {cfg.note}, N = {prob.N} DOFs, concentration preconditioner {pc_name}")

    def solve(prec):
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        x, st = prob.solve(rtol=cfg.newton_tol, prec=prec)
        torch.cuda.synchronize()
        dt = time.perf_counter() - t0
        if st.status != 0:
            raise RuntimeError(f"solve failed with status {st.status}")
        return x, st, dt

    for i in range(args.warmup):
        _, st, dt = solve(DGNP_F32)
        log(f"[bench] warmup {i}: {dt:.3f}s newton {st.newton_its} fgmres {st.lin_its_total}")
    times = []
    for i in range(args.steps):
        x32, st32, dt = solve(DGNP_F32)
        times.append(dt)
        log(f"[bench] step {i}: {dt:.3f}s newton {st32.newton_its} fgmres {st32.lin_its_total} "
            f"setup {st32.t_setup:.3f}s krylov {st32.t_krylov:.3f}s")
    t_mixed = float(np.mean(times))

    # one more solve with per-kernel HIP events (not part of `value`): the library
    # records an event pair around every kernel of the timed regions on its stream
    prob.profile(True)
    solve(DGNP_F32)
    kern = prob.timers()
    prob.profile(False)
    # roofline of the dominant kernel.  The family is the one with the largest
    # total kernel time in the committed rocprofv3 statistics of this solve
    # (profiles/dominant_kernels.json, written from the kernel-trace summary);
    # its average launch duration is measured here with the library's per-launch
    # HIP events on its own stream (they include the dispatch gap that the
    # profiler's durations exclude, so the fraction is slightly low).
    models = {
        "cheb_blk_f32": (cheb_blk_bytes(cfg, 4),
                         "k_cheb_blk<float> (fused Chebyshev step of the potential smoother on the element blocks)"),
        "ilu_fwd_f32": (ilu_sweep_bytes(cfg, 4),
                        "k_ilu_dfp<fwd> (dataflow BILU(0) forward sweep, both concentration blocks)"),
        "ilu_bwd_f32": (ilu_sweep_bytes(cfg, 4, backward=True),
                        "k_ilu_dfp<bwd> (dataflow BILU(0) backward sweep, both concentration blocks)"),
        "jac_apply_f32": (float(japply_bytes(prob.N, 4)), "k_jlin<float> (Jacobian apply, tabulated state)"),
        "ilu_factor": (ilu_factor_bytes(cfg),
                       "k_ilu_factor (BILU(0) factorisation of the fine concentration blocks, one hyperplane "
                       "level per launch)"),
    }
    present = {k: v for k, v in kern.items() if k in models}
    ranking = profile_ranking(cfg.name + ("_bilu" if args.conc_pc == "bilu" else ""))
    if ranking and ranking.get("family") in present:
        dom, chosen_by = ranking["family"], "largest total kernel time in the rocprofv3 statistics of this solve"
    else:
        dom = max(present.items(), key=lambda kv: kv[1][0])[0]
        chosen_by = "largest event-timed total (no rocprofv3 ranking for this workload)"
    tot, launches = kern[dom]
    avg = tot / launches
    per_launch_bytes, kname = models[dom]
    achieved = per_launch_bytes / avg / 1e9
    # counter-measured HBM bytes per launch (profiles/hbm_traffic.json), per workload
    keys = {"cfg2": {"cheb_blk_f32": "k_cheb_blk_f32_cfg2", "ilu_fwd_f32": "k_ilu_dfp_fwd_cfg2",
                     "ilu_bwd_f32": "k_ilu_dfp_bwd_cfg2", "jac_apply_f32": "k_jlin_f32_cfg2",
                     "ilu_factor": "k_ilu_factor_fine_cfg2"},
            "cfg5": {"ilu_fwd_f32": "k_ilu_dfl_fwd_cfg5", "ilu_bwd_f32": "k_ilu_dfl_bwd_cfg5",
                     "jac_apply_f32": "k_jlin_f32_cfg5", "ilu_factor": "k_ilu_factor_cfg5"}}.get(cfg.name, {})
    srcs = ("kernels_jac.hip", "dg_device.hpp", "pointwise.hpp") if dom == "jac_apply_f32" else ("kernels_block.hip",)
    copy_gbs = copy_bandwidth()
    roofline = {"kernel": kname, "bound": "hbm", "achieved": achieved, "peak": PEAK_HBM_GBS, "unit": "GB/s",
                "frac": achieved / PEAK_HBM_GBS, "avg_launch_us": 1e6 * avg, "launches": launches,
                "bytes_per_launch": per_launch_bytes, "chosen_by": chosen_by,
                "traffic": measured_traffic(keys[dom], source_hash(*srcs)) if dom in keys else None,
                # context, not the peak: what a plain device-to-device copy sustains here
                "copy_GBps": copy_gbs, "frac_of_copy": achieved / copy_gbs if copy_gbs else None}
    if ranking and ranking.get("family") == dom and ranking.get("avg_us"):
        # the same kernel's average duration in the committed profile, for comparison
        roofline["rocprof_avg_launch_us"] = ranking["avg_us"]
        roofline["frac_rocprof"] = per_launch_bytes / (1e-6 * ranking["avg_us"]) / 1e9 / PEAK_HBM_GBS
    if dom == "ilu_factor":
        # its block products run on the FP64 matrix cores: their fraction too
        # (the memory roof binds first at the speed of light: bytes / 8 TB/s
        # exceeds flops / 78.6 TFLOP/s)
        fl = ilu_factor_flops(cfg)
        roofline["flops_per_launch"] = fl
        roofline["fp64_mfma_TFLOPs"] = fl / avg / 1e12
        roofline["fp64_mfma_frac"] = fl / avg / 1e12 / PEAK_FP64_TFLOPS
    log(f"[bench] dominant kernel {dom}: {tot:.3f}s in {launches} launches, {1e6 * avg:.2f} us/launch, "
        f"{achieved:.0f} GB/s")
    others = {}
    for k in models:
        if k in kern and k != dom:
            t, n_ = kern[k]
            others[k] = {"avg_launch_us": 1e6 * t / n_, "GBps": models[k][0] / (t / n_) / 1e9}

    out = {
        "metric": METRIC,
        "value": t_mixed,
        "unit": "s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": 1e3 * t_mixed,
        "higher_is_better": False,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f32 apply+preconditioner, f64 residual/Arnoldi/refinement",
        "data": "synthetic (seeded inflow data U[0.5,1.5], random-free solve)",
        "config": {"workload": f"{cfg.name}: {cfg.note}", "elements": list(cfg.n), "order": cfg.p,
                   "ions": cfg.m, "dofs": prob.N, "newton_rtol": cfg.newton_tol,
                   "newton_its": st32.newton_its, "fgmres_its": st32.lin_its_total,
                   "concentration_preconditioner": pc_name},
        "roofline": roofline,
        "other_kernels": others,
        "kernel_seconds_per_solve": {k: round(v[0], 6) for k, v in kern.items()},
    }
    out["median_step_s"] = float(np.median(times))
    if not args.no_extra:
        solve(DGNP_F64)
        r64 = [solve(DGNP_F64) for _ in range(REPS)]
        x64, st64 = r64[-1][0], r64[-1][1]
        t64 = float(np.median([r[2] for r in r64]))
        del r64
        out["fp64_time_s"] = t64
        out["mixed_speedup_vs_fp64"] = t64 / t_mixed
        out["mixed_vs_fp64_rel_l2"] = (x64 - x32).norm().item() / x64.norm().item()
        ta = []
        for _ in range(REPS):
            torch.cuda.synchronize()
            t0 = time.perf_counter()
            J, dg, dpe, lam, ast = prob.adjoint(x32, prec=DGNP_F32, rtol=1e-8)
            torch.cuda.synchronize()
            ta.append(time.perf_counter() - t0)
        out["adjoint_time_s"] = float(np.median(ta))
        log(f"[bench] fp64 {t64:.3f}s, adjoint {out['adjoint_time_s']:.3f}s")
        prob.close()
        if pc_kw:
            # the same solves with one block-ILU(0) solve per concentration block
            pb = Problem(cfg, boundary_data(cfg))
            rec = {}
            for tag, prec in (("mixed_s", DGNP_F32), ("fp64_s", DGNP_F64)):
                solve_with = [None]

                def run_b():
                    torch.cuda.synchronize()
                    t0 = time.perf_counter()
                    x, st = pb.solve(rtol=cfg.newton_tol, prec=prec)
                    torch.cuda.synchronize()
                    if st.status != 0:
                        raise RuntimeError(f"BILU solve failed with status {st.status}")
                    solve_with[0] = st
                    return time.perf_counter() - t0

                run_b()
                rec[tag] = float(np.median([run_b() for _ in range(REPS)]))
                rec["fgmres_its" if prec == DGNP_F32 else "fgmres_its_fp64"] = solve_with[0].lin_its_total
            pb.close()
            out["bilu_concentration_preconditioner"] = rec
            log(f"[bench] BILU(0): mixed {rec['mixed_s']:.4f}s, fp64 {rec['fp64_s']:.4f}s")
        ja = apply_bandwidth(args.apply_workload)
        ja["traffic_f32"] = measured_traffic("k_jlin_f32_cfg5", source_hash("kernels_jac.hip", "dg_device.hpp",
                                                                            "pointwise.hpp"))
        out["jacobian_apply"] = ja
        out["channel_solves"] = channel_solves(["cfg3", "cfg5"])
        out["concentration_preconditioners"] = conc_pc_solves(["ch256p1"])
    if not args.no_cpu:
        # the GPU's mixed solve of the oracle's sample input, beside the oracle
        small = get_config("cfg2t")
        sp = Problem(small, boundary_data(small))
        sp.solve(rtol=small.newton_tol, prec=DGNP_F32)
        ts = []
        for _ in range(3):
            torch.cuda.synchronize()
            t0 = time.perf_counter()
            sp.solve(rtol=small.newton_tol, prec=DGNP_F32)
            torch.cuda.synchronize()
            ts.append(time.perf_counter() - t0)
        sp.close()
        cb = cpu_baseline(float(np.median(ts)))
        log(f"[bench] cpu oracle: {cb['value']:.2f}s ({cb['sample']}); GPU on the same input {np.median(ts):.4f}s")
        out["cpu_baseline"] = cb
        if not args.no_extra:
            out["oracle_operator_timings"] = oracle_operator_timings()
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
