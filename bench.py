"""Throughput of the matrix-element hot path on one MI355X.

Workload: g g -> t tbar g g at sqrt(s) = 13 TeV, 2^20 seeded RAMBO points
(seed 2), float64 momenta resident in HBM.  One step = one evaluation of
|M|^2 for every point (all helicities, diagrams and colour sums).

Prints one JSON line.  `value` is the float64 form's MEs/s; the mixed form
(float32 amplitudes + float16 hi/lo MFMA colour sum + float64 rerun of flagged
events) and the surrogate form (network trained on exact labels, two-stage
unweighting) are reported under "forms".  `roofline` is the dominant float64
kernel, timed with HIP events on its launch stream; `cpu_baseline` is the CPU
oracle on a bounded sample of the same points.
"""
from __future__ import annotations

import argparse
import hashlib
import json
import math
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

PEAK = {"fp64": 78.6, "fp32": 157.3, "bf16_mfma": 2500.0}  # MI355X, TFLOP/s (dense)


def log(msg):
    print(f"[bench] {msg}", file=sys.stderr, flush=True)


def timed(fn, steps, stream):
    """Average kernel-side time of fn() over `steps` calls (HIP events on `stream`) and wall time."""
    import torch

    e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    torch.cuda.synchronize()
    w0 = time.perf_counter()
    e0.record(stream)
    for _ in range(steps):
        fn()
    e1.record(stream)
    torch.cuda.synchronize()
    wall = (time.perf_counter() - w0) / steps
    return e0.elapsed_time(e1) / steps * 1e-3, wall


def kernel_sources_digest(process):
    """Digest of the sources that make up the float64 kernel of `process`."""
    h = hashlib.sha256()
    csrc = os.path.join(ROOT, "paper_2503_21935_amd", "csrc")
    for f in ("me_vertex.h", "me_process.h", "me_kernels.h", "me_launch.h", "me_lds.h", "me_coop.h", "me_qew.h",
              os.path.join("gen", f"proc_{process}.h")):
        p = os.path.join(csrc, f)
        if os.path.exists(p):
            h.update(open(p, "rb").read())
    return h.hexdigest()[:16]


def traffic_from_profile(process, kernel):
    """HBM bytes per launch from the committed counter summary, or None when the
    kernel's sources changed after the counters were taken."""
    path = os.path.join(ROOT, "profiles", "counters.json")
    if not os.path.exists(path):
        return None
    rec = json.load(open(path)).get(kernel)
    if not rec or rec.get("sources") != kernel_sources_digest(process):
        return None
    return rec["fetch_kib"] * rec["fetch_factor"] * 1024 + rec["write_kib"] * rec["write_factor"] * 1024


def bench_fp64(m, mom, out, args, stream):
    for _ in range(args.warmup):
        m.eval(mom, out=out, stream=stream)
    return timed(lambda: m.eval(mom, out=out, stream=stream), args.steps, stream)


def bench_process(me, proc, nevt, seed, steps, stream, check=8, tol=None):
    """Float64 throughput of another process at its own workload size, with a
    few events checked against the oracle."""
    import numpy as np
    import torch

    import oracle
    from inputs import process_points

    mom_np = process_points(proc, nevt, seed, precise=True)
    mom = torch.from_numpy(mom_np).cuda()
    m = me.MatrixElement(proc)
    info = m.info()
    out = torch.empty(nevt, dtype=torch.float64, device=mom.device)
    m.eval(mom, out=out, stream=stream)
    k_s, wall = timed(lambda: m.eval(mom, out=out, stream=stream), steps, stream)
    res = out.cpu().numpy()
    idx = np.sort(np.random.default_rng(5).choice(nevt, check, replace=False))
    ref = oracle.me2(proc, mom_np[idx])
    rel = np.abs(res[idx] / ref - 1)
    mixed = None
    if m.info()["ncol"] > 1 and tol:
        m.set_precision(me.ME_MIXED, tol)
        m.eval(mom, out=out, stream=stream)
        mk_s, mwall = timed(lambda: m.eval(mom, out=out, stream=stream), steps, stream)
        nfb = m.fallback_count()
        mres = out.cpu().numpy()
        mixed = {"MEs_per_s": nevt / mwall, "ms_per_step": mwall * 1e3, "tolerance": tol,
                 "fallback_fraction": nfb / nevt, "max_rel_err_vs_oracle": float(np.abs(mres[idx] / ref - 1).max())}
        m.set_precision(me.ME_FP64, tol)
    m.close()
    achieved = info["flops_per_event"] * nevt / k_s / 1e12
    kernel = {"gg_ttggg": f"k_me_gg_coop<proc_{proc}>", "ee_mumu": "k_me_ee<proc_ee_mumu>"}.get(
        proc, f"k_me_qew<proc_{proc}>" if proc.startswith("gux_") else f"k_me_gg<proc_{proc}>")
    return {"workload": f"{proc}, {nevt} RAMBO points seed {seed}", "MEs_per_s": nevt / wall, "kernel": kernel,
            "traffic": traffic_from_profile(proc, kernel),
            "kernel_ms": k_s * 1e3, "flops_per_event": info["flops_per_event"],
            "achieved_tflops": achieved, "frac_of_fp64_peak": achieved / PEAK["fp64"],
            "max_rel_dev_vs_oracle": float(rel.max()), "checked_events": check, "mixed": mixed}


def nevt_sweep(me, proc, seed, lanes_list, logs, stream):
    """MEs/s of the float64 kernel against the number of events per launch, for
    the automatic lane count (0: enough lanes per event to put 2^16 lanes in
    flight), one lane per event and helicity-parallel launches (2^k lanes per
    event)."""
    import torch

    from inputs import process_points

    nmax = 1 << max(logs)
    mom_all = torch.from_numpy(process_points(proc, nmax, seed, precise=False)).cuda()
    m = me.MatrixElement(proc)
    rows = []
    for lanes in lanes_list:
        m.set_helicity_lanes(lanes)
        for lg in logs:
            n = 1 << lg
            mom = mom_all[:n]
            out = torch.empty(n, dtype=torch.float64, device=mom.device)
            reps = max(3, min(200, (1 << 22) // n))
            m.eval(mom, out=out, stream=stream)
            k_s, _ = timed(lambda: m.eval(mom, out=out, stream=stream), reps, stream)
            rows.append({"lanes_per_event": lanes, "nevt": n, "kernel_ms": k_s * 1e3, "MEs_per_s": n / k_s})
        log(f"sweep {proc} lanes {lanes}: " + ", ".join(f"2^{lg} {r['MEs_per_s']:.2e}"
                                                       for lg, r in zip(logs, rows[-len(logs):])))
    m.close()
    return {"process": proc, "timing": "HIP events on the launch stream, average per launch", "points": rows}


def bench_phase_space(me, stream, n, host_s):
    """GPU phase-space sampling (Philox4x32-10 + RAMBO) of the benchmark's
    workload: 2^20 g g -> t tbar g g points; bound by the HBM write of the
    momenta and weights (192 + 8 bytes per point)."""
    import torch

    masses = [173.0, 173.0, 0.0, 0.0]
    mom = torch.empty((n, 6, 4), dtype=torch.float64, device="cuda")
    wt = torch.empty(n, dtype=torch.float64, device="cuda")
    me.ps_rambo(13000.0, masses, 2, 0, n, mom, wt, stream)
    k_s, _ = timed(lambda: me.ps_rambo(13000.0, masses, 2, 0, n, mom, wt, stream), 20, stream)
    nbytes = n * (6 * 4 * 8 + 8)
    return {"workload": f"{n} g g -> t tbar g g points, sqrt(s) = 13 TeV", "kernel": "k_ps_rambo<4>",
            "points_per_s": n / k_s, "kernel_ms": k_s * 1e3,
            "roofline": {"bound": "hbm", "achieved": nbytes / k_s / 1e9, "peak": 8000.0, "unit": "GB/s",
                         "frac": nbytes / k_s / 1e9 / 8000.0, "bytes_per_point": 200,
                         "note": "the output bytes against HBM; the kernel is bound by its float64 arithmetic "
                                 "(Philox, logarithms, square roots, the massive rescaling), counted in "
                                 "profiles/ps_rambo_2p20.md"},
            "host_numpy_rambo_s_same_size": host_s}


def bench_ps_multichannel(me, stream, n, steps):
    """Multi-channel phase space for the DY+3j subprocess g ubar -> tau+ tau-
    g g ubar at sqrt(s) = 13 TeV (2^20 points; flat, Z Breit-Wigner and photon
    1/M^2 channels on the tau-pair mass, window 50 GeV .. sqrt(s)): sampler
    throughput, then the integral of |M|^2 with the generator cuts on the
    partons, estimated from the same number of flat RAMBO points and of
    multi-channel points.  Reported per sampler: the estimate, its relative
    standard error, the effective sample fraction (sum f)^2 / (N sum f^2) and
    the unweighting efficiency mean(f) / max(f) of f = w |M|^2."""
    import numpy as np
    import torch

    from inputs import gluon_cuts

    proc, roots, nf, pair, window = "gux_taptamggux", 13000.0, 5, (0, 1), (50.0, 13000.0)
    mz, wz = me.DEFAULT_MASSES[0], me.DEFAULT_MASSES[1]  # the matrix element's Z mass and width
    alpha = (0.3, 0.4, 0.3)
    mom = torch.empty((n, nf + 2, 4), dtype=torch.float64, device="cuda")
    wt = torch.empty(n, dtype=torch.float64, device="cuda")
    ch = torch.empty(n, dtype=torch.int32, device="cuda")

    def sample(seed):
        me.ps_multichannel(roots, nf, pair, window, mz, wz, alpha, seed, 0, n, mom, wt, ch, stream)

    sample(6)
    k_s, _ = timed(lambda: sample(6), steps, stream)
    nbytes = n * ((nf + 2) * 4 * 8 + 8 + 4)
    m = me.MatrixElement(proc)
    me2 = torch.empty(n, dtype=torch.float64, device="cuda")
    stats = {}
    for name in ("flat", "multichannel"):
        if name == "flat":
            me.ps_rambo(roots, [0.0] * nf, 6, 0, n, mom, wt, stream)
        else:
            sample(6)
        m.eval(mom, out=me2, stream=stream)
        mom_np = mom.cpu().numpy()
        P = mom_np[:, 2 + pair[0]] + mom_np[:, 2 + pair[1]]
        mll2 = P[:, 0] ** 2 - (P[:, 1:] ** 2).sum(-1)
        ok = gluon_cuts(mom_np) & (mll2 >= window[0] ** 2)
        f = np.where(ok, wt.cpu().numpy() * me2.cpu().numpy(), 0.0)
        mean = f.mean()
        near_z = ok & (np.abs(np.sqrt(np.maximum(mll2, 0.0)) - mz) < 10.0)
        stats[name] = {"estimate": float(mean), "rel_std_error": float(f.std() / (mean * np.sqrt(n))),
                       "effective_sample_fraction": float(f.sum() ** 2 / (n * (f ** 2).sum())),
                       "unweighting_efficiency": float(mean / f.max()), "points_passing_cuts": int(ok.sum()),
                       "points_within_10_GeV_of_MZ": int(near_z.sum()),
                       "share_of_estimate_within_10_GeV_of_MZ": float(f[near_z].sum() / f.sum())}
        if name == "multichannel":
            stats[name]["channel_counts"] = np.bincount(ch.cpu().numpy(), minlength=3).tolist()
    m.close()
    fl, mc = stats["flat"], stats["multichannel"]
    return {"workload": f"{n} {proc} points, sqrt(s) = 13 TeV, pair-mass window {window[0]:g} GeV .. sqrt(s), "
                        f"alpha {alpha}", "kernel": f"k_ps_mc<{nf}>", "points_per_s": n / k_s,
            "kernel_ms": k_s * 1e3,
            "roofline": {"bound": "hbm", "achieved": nbytes / k_s / 1e9, "peak": 8000.0, "unit": "GB/s",
                         "frac": nbytes / k_s / 1e9 / 8000.0, "bytes_per_point": nbytes // n,
                         "note": "the output bytes against HBM; the kernel is bound by its float64 "
                                 "transcendental functions, counted in profiles/ps_multichannel_dy3j_2p20.md"},
            "flat": fl, "multichannel": mc,
            "variance_gain": (fl["rel_std_error"] / mc["rel_std_error"]) ** 2,
            "estimates_differ_by_sigma": float(abs(fl["estimate"] - mc["estimate"]) / np.hypot(
                fl["rel_std_error"] * fl["estimate"], mc["rel_std_error"] * mc["estimate"]))}


def bench_colour_forms(me, stream, cases):
    """Float64 kernel time with the colour sum on the VALU (symmetric form) and
    as a float64 MFMA GEMM over block pairs (me_set_colour_form)."""
    import torch

    from inputs import process_points

    out = {}
    for proc, n, seed, steps in cases:
        mom = torch.from_numpy(process_points(proc, n, seed, precise=False)).cuda()
        res = torch.empty(n, dtype=torch.float64, device="cuda")
        m = me.MatrixElement(proc)
        row = {"nevt": n}
        vals = {}
        for name, form in (("valu", me.ME_COLOUR_VALU), ("mfma", me.ME_COLOUR_MFMA)):
            m.set_colour_form(form)
            m.eval(mom, out=res, stream=stream)
            k_s, _ = timed(lambda: m.eval(mom, out=res, stream=stream), steps, stream)
            vals[name] = res.clone()
            row[f"{name}_kernel_ms"] = k_s * 1e3
            row[f"{name}_MEs_per_s"] = n / k_s
        row["max_rel_diff_between_forms"] = float(((vals["mfma"] / vals["valu"]) - 1).abs().max())
        m.close()
        out[proc] = row
        log(f"colour forms {proc}: {row}")
    return out


def bench_multichannel(me, stream, mom, proc, steps):
    """|M|^2 with the single-diagram weight of each event's channel (channels
    drawn uniformly, mixed within every wave), against the plain float64 kernel
    on the same points; a few events checked against the oracle's diagrams."""
    import numpy as np
    import torch

    import oracle

    m = me.MatrixElement(proc)
    nchan = len(m.channels())
    n = mom.shape[0]
    chan = torch.from_numpy(np.random.default_rng(8).integers(0, nchan, size=n).astype(np.int32)).cuda()
    out = torch.empty(n, dtype=torch.float64, device="cuda")
    alpha = torch.empty(n, dtype=torch.float64, device="cuda")
    me.me_eval_multichannel(m.ctx, mom, chan, n, out, alpha, stream)
    k_s, wall = timed(lambda: me.me_eval_multichannel(m.ctx, mom, chan, n, out, alpha, stream), steps, stream)
    idx = np.arange(0, n, n // 8)
    descs, sums = oracle.diagram_sums(proc, mom[idx].cpu().numpy())
    col = {d: i for i, d in enumerate(descs)}
    gd = m.channels()
    ch = chan[idx].cpu().numpy()
    ref = np.array([sums[j, col[gd[c]]] / sums[j].sum() for j, c in enumerate(ch)])
    dev = float(np.max(np.abs(alpha[idx].cpu().numpy() / ref - 1)))
    m.close()
    return {"process": proc, "nevt": n, "channels": nchan, "kernel": f"k_me_gg_mc<proc_{proc}_mc>",
            "MEs_per_s": n / k_s, "kernel_ms": k_s * 1e3, "max_rel_dev_alpha_vs_oracle": dev, "checked_events": len(idx)}


def parity_adjudication(proc, mom_np, got, ref, tol=1e-12):
    """Events beyond tol against the float64 oracle, re-evaluated with the
    __float128 oracle: their deviation from the quad result and the spread of
    the quad result under 2^-52 relative perturbations of the input momenta."""
    import numpy as np

    import oracle

    rel = np.abs(got / ref - 1)
    bad = np.nonzero(rel > tol)[0]
    out = {"events": int(len(got)), "beyond_1e-12_vs_double_oracle": int(bad.size),
           "max_rel_dev_vs_double_oracle": float(rel.max())}
    if bad.size:
        q0 = oracle.me2(proc, mom_np[bad], quad=True)
        rng = np.random.default_rng(1)
        spread = np.zeros(bad.size)
        for _ in range(16):
            pert = mom_np[bad] * (1 + rng.choice([-1.0, 1.0], size=mom_np[bad].shape) * 2.0 ** -52)
            spread = np.maximum(spread, np.abs(oracle.me2(proc, pert, quad=True) / q0 - 1))
        rq = np.abs(got[bad] / q0 - 1)
        ok = (rq <= tol) | (rq <= 10 * spread)
        out.update({"their_max_rel_dev_vs_quad_oracle": float(rq.max()),
                    "their_max_input_rounding_spread": float(spread.max()),
                    "within_1e-12_of_quad_or_10x_spread": int(ok.sum())})
    return out


def cpu_model():
    try:
        for line in open("/proc/cpuinfo"):
            if line.startswith("model name"):
                return line.split(":", 1)[1].strip()
    except OSError:
        pass
    return "unknown"


def omp_threads(n=None):
    """Set (n given) or read the OpenMP thread count of the oracle's runtime."""
    import ctypes

    try:
        gomp = ctypes.CDLL("libgomp.so.1")
    except OSError:
        return None
    if n is not None:
        gomp.omp_set_num_threads(int(n))
    return int(gomp.omp_get_max_threads())


def bench_mixed(me, m, mom, mom_np, args, stream):
    import numpy as np
    import torch

    import oracle

    m.set_precision(me.ME_MIXED, args.tol)
    out = torch.empty(mom.shape[0], dtype=torch.float64, device=mom.device)
    for _ in range(args.warmup):
        m.eval(mom, out=out, stream=stream)
    k_s, wall = timed(lambda: m.eval(mom, out=out, stream=stream), args.steps, stream)
    nfb = m.fallback_count()
    res = out.cpu().numpy()
    raw, est, flag = m.eval_mixed_diag(mom, stream=stream)
    diag_s, _ = timed(lambda: m.eval_mixed_diag(mom, stream=stream), 3, stream)
    torch.cuda.synchronize()
    raw = raw.cpu().numpy()
    idx = np.sort(np.random.default_rng(3).choice(len(res), args.check, replace=False))
    ref = oracle.me2(args.process, mom_np[idx])
    rel = np.abs(res[idx] / ref - 1)
    rel_raw = np.abs(raw[idx] / ref - 1)
    m.set_precision(me.ME_FP64, args.tol)
    n = mom.shape[0]
    info = m.info()
    # composite bound: amplitudes at the float32 vector peak, colour form (dense
    # quadratic form, 4 ncol^2 + 4 ncol per event and helicity) at the FP16 MFMA peak
    f_col = info["nhel_good"] * (4 * info["ncol"] ** 2 + 4 * info["ncol"])
    f_amp = info["flops_per_event"] - info["nhel_good"] * info["flops_colour_per_hel"]
    t_min = n * (f_amp / (PEAK["fp32"] * 1e12) + f_col / (PEAK["bf16_mfma"] * 1e12))
    return {
        "MEs_per_s": n / wall, "ms_per_step": wall * 1e3, "tolerance": args.tol,
        "roofline": {"bound": "composite: fp32 vector (amplitudes) + fp16 mfma (colour)",
                     "t_min_ms": t_min * 1e3, "mixed_kernel_ms": diag_s * 1e3, "frac": t_min / diag_s,
                     "frac_incl_rerun": t_min / k_s,
                     "flops_amplitudes_per_event": f_amp, "flops_colour_per_event": f_col},
        "fallback_fraction": nfb / n,
        "mixed_kernel_ms_without_rerun": diag_s * 1e3,
        "max_rel_err_vs_oracle": float(rel.max()),
        "float32_form_rel_err": {"p50": float(np.median(rel_raw)), "p99.9": float(np.quantile(rel_raw, 0.999)),
                                 "max": float(rel_raw.max())},
        "checked_events": int(args.check),
    }


def unweighting_scan(me, ctx, net, mu_t, wu_t, uu_t, nu, mu, sig, s_c, wex_c, me2_all, one_s, stream,
                     quantiles=(0.99, 0.999, 0.9999), nboot=200):
    """N_eff of both unweightings and the cost gain per effective event at several
    quantiles of the calibration sample for the reduced maxima, with a Poisson
    bootstrap over the unweighting sample's points (each point drawn k ~ Poisson(1)
    times, the same k for both unweightings) at each quantile: median and the
    16th / 84th percentiles.  The two-stage cost is timed at each quantile; the
    exact-only cost (every point's |M|^2) is the main run's."""
    import torch

    dev = mu_t.device
    pos = s_c > 0
    wex = me2_all * wu_t
    out_idx = torch.empty(nu, dtype=torch.int32, device=dev)
    out_w = torch.empty(nu, dtype=torch.float64, device=dev)
    cnt = torch.zeros(2, dtype=torch.int32, device=dev)
    gen = torch.Generator(device=dev)
    res = []
    for q in quantiles:
        s_max = float(torch.quantile(s_c[pos].float(), q))
        r_max = float(torch.quantile((wex_c[pos] / s_c[pos]).float(), q))
        w_max = float(torch.quantile(wex_c[pos].float(), q))
        def run2():
            me.unweight_two_stage(ctx.ctx, net.h, mu_t, wu_t, nu, uu_t, mu, sig, s_max, r_max, out_idx, out_w, cnt,
                                  stream)

        run2()
        _, t2 = timed(run2, 1, stream)
        n2 = int(cnt[1])
        # per-point weights of the two samples (zero where not accepted)
        w2 = torch.zeros(nu, dtype=torch.float64, device=dev)
        w2[out_idx[:n2].long()] = out_w[:n2]
        acc1 = uu_t[:, 0] < torch.clamp(wex / w_max, max=1.0)
        w1 = torch.where(acc1, torch.clamp(wex / w_max, min=1.0), torch.zeros_like(wex))

        def neff(w, k=None):
            if k is not None:
                return float((k * w).sum() ** 2 / (k * w * w).sum().clamp_min(1e-300))
            return float(w.sum() ** 2 / (w * w).sum().clamp_min(1e-300))

        n_e1, n_e2 = neff(w1), neff(w2)
        gen.manual_seed(int(q * 1e6))
        gains = []
        for _ in range(nboot):
            k = torch.poisson(torch.ones(nu, dtype=torch.float64, device=dev), generator=gen)
            b1, b2 = neff(w1, k), neff(w2, k)
            gains.append((one_s / max(b1, 1e-30)) / (t2 / max(b2, 1e-30)))
        gains.sort()
        res.append({"quantile": q, "n_eff_two_stage": n_e2, "n_eff_exact_only": n_e1,
                    "accepted_two_stage": n2, "accepted_exact_only": int(acc1.sum()),
                    "two_stage_s": t2, "exact_calls_per_point": int(cnt[0]) / nu,
                    "gain": (one_s / max(n_e1, 1e-30)) / (t2 / max(n_e2, 1e-30)),
                    "gain_boot_p16_p50_p84": [gains[int(0.16 * nboot)], gains[nboot // 2], gains[int(0.84 * nboot)]]})
    main = min(res, key=lambda r: abs(r["quantile"] - 0.999))
    return {"scan": res, "bootstrap": {"quantile": main["quantile"], "p16_p50_p84": main["gain_boot_p16_p50_p84"],
                                       "replicates": nboot}}


def bench_surrogate(me, args, stream):
    import torch

    from inputs import gluon_cuts, process_points, uniforms

    dev = torch.device("cuda:0")
    proc = args.process
    t0 = time.time()
    mom_tr = process_points(proc, args.n_train, 4, precise=False)
    mom_tr = mom_tr[gluon_cuts(mom_tr)]
    log(f"surrogate: {len(mom_tr)} training points after cuts ({time.time() - t0:.1f}s)")
    ctx = me.MatrixElement(proc)
    mt = torch.from_numpy(mom_tr).to(dev)
    del mom_tr
    lab = ctx.eval(mt)  # labels from the exact float64 kernel
    x = me.features(mt)
    del mt
    lnl = torch.log(lab)
    mu, sig = float(lnl.mean()), float(lnl.std())
    t = ((lnl - mu) / sig).float()
    n = t.shape[0]
    n_val = n // 10
    n_fit = (n - n_val) // args.batch * args.batch
    net = me.Surrogate(seed=1004)
    loss = torch.zeros(1, dtype=torch.float32, device=dev)
    steps_per_epoch = n_fit // args.batch
    total = steps_per_epoch * args.epochs
    # warm-up outside the timed region: the first device randperm and the
    # first launch of the training kernel carry one-time set-up costs
    gw = torch.Generator(device=dev)
    gw.manual_seed(1)
    wperm = (torch.randperm(n_fit, generator=gw, device=dev) + n_val).to(torch.int32)
    net_w = me.Surrogate(seed=1)
    net_w.train_steps(x, t, wperm[:2 * args.batch], args.batch, torch.full((2,), args.lr, device=dev), None, stream)
    torch.cuda.synchronize()
    net_w.close()
    del wperm
    tt0 = time.perf_counter()
    gperm = torch.Generator(device=dev)
    gperm.manual_seed(7)
    # cosine learning rates of every step, one device array
    lr_all = torch.tensor([0.5 * args.lr * (1 + math.cos(math.pi * st / total)) for st in range(total)],
                          dtype=torch.float32, device=dev)
    for ep in range(args.epochs):
        # the epoch's sample order, drawn on the device
        perm = (torch.randperm(n_fit, generator=gperm, device=dev) + n_val).to(torch.int32)
        # the epoch's steps in one call (one cooperative launch)
        net.train_steps(x, t, perm, args.batch, lr_all[ep * steps_per_epoch:(ep + 1) * steps_per_epoch], None,
                        stream)
    torch.cuda.synchronize()
    train_s = time.perf_counter() - tt0
    log(f"surrogate: {args.epochs} epochs of {steps_per_epoch} steps in {train_s:.3f} s")
    # the same step as one call per step, and as the layered GEMM path, on
    # separate networks, for comparison
    idx_l = perm[:args.batch]
    net_c = me.Surrogate(seed=1004)
    net_c.train_step(x, t, idx_l, args.lr, loss, stream)
    percall_s, _ = timed(lambda: net_c.train_step(x, t, idx_l, args.lr, loss, stream), 100, stream)
    net_c.close()
    net_l = me.Surrogate(seed=1004)
    net_l.set_fused_step(False)
    net_l.train_step(x, t, idx_l, args.lr, loss, stream)
    layered_s, _ = timed(lambda: net_l.train_step(x, t, idx_l, args.lr, loss, stream), 100, stream)
    net_l.close()
    yv = net.forward(x[:n_val])
    val_mse = float(torch.mean((yv - t[:n_val]) ** 2))
    yall = torch.empty(n, dtype=torch.float32, device=dev)
    inf_s, _ = timed(lambda: me.mlp_forward(net.h, x, n, yall, stream), 3, stream)
    del x, t, lab, lnl, yall
    # s_max and r_max from an independent calibration sample (seed 6)
    mom_c, w_c = process_points(proc, args.n_calib, 6, return_weight=True, precise=False)
    w_c = w_c * gluon_cuts(mom_c)
    mc = torch.from_numpy(mom_c).to(dev)
    wc_t = torch.from_numpy(w_c).to(dev)
    yc = net.forward(me.features(mc)).double()
    s_c = torch.exp(sig * yc + mu) * wc_t
    wex_c = ctx.eval(mc) * wc_t
    # Reduced maxima (a quantile of the calibration sample): flat phase space puts
    # single points many orders above the bulk; points above a maximum are kept
    # with weight > 1, so both unweightings stay unbiased.
    pos = s_c > 0
    q = args.max_quantile
    s_max = float(torch.quantile(s_c[pos].float(), q))
    r_max = float(torch.quantile((wex_c[pos] / s_c[pos]).float(), q))
    w_max = float(torch.quantile(wex_c[pos].float(), q))
    del mc, mom_c
    # unweighting sample (seed 5): two-stage, then exact-only on the same points
    mom_u, w_u = process_points(proc, args.n_unweight, 5, return_weight=True, precise=False)
    w_u = w_u * gluon_cuts(mom_u)
    nu = len(mom_u)
    u = uniforms(nu, 2, 55)
    mu_t = torch.from_numpy(mom_u).to(dev)
    wu_t = torch.from_numpy(w_u).to(dev)
    uu_t = torch.from_numpy(u).to(dev)
    del mom_u
    out_idx = torch.empty(nu, dtype=torch.int32, device=dev)
    out_w = torch.empty(nu, dtype=torch.float64, device=dev)
    cnt = torch.zeros(2, dtype=torch.int32, device=dev)

    def two_stage():
        me.unweight_two_stage(ctx.ctx, net.h, mu_t, wu_t, nu, uu_t, mu, sig, s_max, r_max, out_idx, out_w, cnt,
                              stream)

    two_stage()
    _, two_s = timed(two_stage, 1, stream)
    n1, n2 = [int(v) for v in cnt.cpu()]
    wsel = out_w[:n2]
    neff2 = float(wsel.sum() ** 2 / (wsel ** 2).sum()) if n2 else 0.0
    me2_all = torch.empty(nu, dtype=torch.float64, device=dev)
    one = {}

    def exact_only():
        ctx.eval(mu_t, out=me2_all, stream=stream)
        wex = me2_all * wu_t
        one["acc"] = uu_t[:, 0] < torch.clamp(wex / w_max, max=1.0)
        one["wt"] = torch.clamp(wex / w_max, min=1.0)

    exact_only()
    _, one_s = timed(exact_only, 1, stream)
    sel1 = one["wt"][one["acc"]]
    neff1 = float(sel1.sum() ** 2 / (sel1 ** 2).sum()) if sel1.numel() else 0.0
    mlp_flops = 2 * (24 * 256 + 3 * 256 * 256 + 256)
    gain = (one_s / max(neff1, 1e-30)) / (two_s / max(neff2, 1e-30))
    scan = unweighting_scan(me, ctx, net, mu_t, wu_t, uu_t, nu, mu, sig, s_c, wex_c, me2_all, one_s, stream)
    ctx.close()
    net.close()
    train_rate = total * args.batch / train_s
    return {
        "train_samples_per_s": train_rate, "train_epochs": args.epochs, "train_batch": args.batch,
        "train_step": "one cooperative launch per epoch (per step: forward, backward, batch sums, Adam)",
        "train_samples_per_s_one_call_per_step": args.batch / percall_s,
        "train_samples_per_s_layered_kernels": args.batch / layered_s,
        "train_tflops": 3 * mlp_flops * train_rate / 1e12,
        "train_frac_of_bf16_mfma_peak": 3 * mlp_flops * train_rate / 1e12 / PEAK["bf16_mfma"],
        "train_points": int(n_fit), "val_mse_standardised_log_me2": val_mse,
        "inference_samples_per_s": n / inf_s,
        "inference_tflops": mlp_flops * n / inf_s / 1e12,
        "inference_frac_of_bf16_mfma_peak": mlp_flops * n / inf_s / 1e12 / PEAK["bf16_mfma"],
        "unweighting_points": nu, "unweighting_points_per_s": nu / two_s,
        "stage1_kept": n1, "exact_calls_per_point": n1 / nu, "accepted": n2, "n_eff": neff2,
        "exact_only": {"points_per_s": nu / one_s, "accepted": int(one["acc"].sum()), "n_eff": neff1},
        "gain_cost_per_effective_event": gain,
        "gain_bootstrap": scan["bootstrap"],
        "max_quantile_scan": scan["scan"],
        "s_max": s_max, "r_max": r_max, "w_max": w_max, "max_quantile": args.max_quantile,
        "cuts": "gluon pT > 20 GeV, |eta| < 5, Delta R > 0.4",
    }


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=20)
    ap.add_argument("--warmup", type=int, default=3)
    ap.add_argument("--nevt", type=int, default=1 << 20)
    ap.add_argument("--process", default="gg_ttgg")
    ap.add_argument("--seed", type=int, default=2)
    ap.add_argument("--tol", type=float, default=1e-5, help="mixed form: per-event relative tolerance")
    ap.add_argument("--check", type=int, default=2048, help="mixed form: events checked against the oracle")
    ap.add_argument("--cpu-sample", type=int, default=1 << 16, help="events for the CPU oracle baseline")
    ap.add_argument("--forms", default="fp64,mixed,surrogate,gg_ttggg,dy3j,configs,sweep,ps,psmc,colour,mc",
                    help="gg_ttggg: also time the float64 kernel of g g -> t tbar g g g (2^18 points, seed 3); "
                         "dy3j: g ubar -> tau+ tau- g g ubar, the DY+3j subprocess (2^20 points, seed 4); "
                         "configs: e+e- -> mu+mu- (16384 points, seed 0) and g g -> t tbar (2^20, seed 1); "
                         "sweep: events per launch 2^10..2^20 at 1, 4, 16, 64 lanes per event; "
                         "ps: the GPU phase-space sampler on the benchmark's workload; "
                         "psmc: multi-channel phase space for the DY+3j subprocess, and its variance against flat; "
                         "colour: float64 kernels with the colour sum on the VALU and on the matrix cores; "
                         "mc: the multi-channel form (single-diagram weights)")
    ap.add_argument("--cpu-sample-1t", type=int, default=4096, help="events for the single-thread oracle figure")
    ap.add_argument("--n-train", type=int, default=1 << 22)
    ap.add_argument("--n-calib", type=int, default=1 << 20)
    ap.add_argument("--n-unweight", type=int, default=1 << 22)
    ap.add_argument("--epochs", type=int, default=8)
    ap.add_argument("--batch", type=int, default=4096)
    ap.add_argument("--lr", type=float, default=1e-3)
    ap.add_argument("--max-quantile", type=float, default=0.999,
                    help="unweighting maxima: this quantile of the calibration sample")
    ap.add_argument("--no-cpu", action="store_true")
    ap.add_argument("--copy-calibration", type=int, default=0, metavar="MIB",
                    help="first run a plain device-to-device copy of this many MiB (a reference kernel of "
                         "known traffic for the HBM byte counters)")
    args = ap.parse_args()
    if args.gpus != 1:
        print(json.dumps({"error": "this build runs on one GPU; --gpus must be 1"}))
        sys.exit(2)
    forms = set(args.forms.split(","))

    import numpy as np
    import torch

    import paper_2503_21935_amd as me
    from inputs import process_points

    dev = torch.device("cuda:0")
    torch.cuda.set_device(dev)
    stream = torch.cuda.current_stream()
    if args.copy_calibration:
        nb = args.copy_calibration << 20
        a = torch.ones(nb // 8, dtype=torch.float64, device=dev)
        b = torch.empty_like(a)
        b.copy_(a)
        torch.cuda.synchronize()
        log(f"copy calibration: {nb} bytes read, {nb} bytes written")
        del a, b
    t0 = time.time()
    mom_np = process_points(args.process, args.nevt, args.seed)
    host_gen_s = time.time() - t0
    log(f"generated {args.nevt} points on the host in {host_gen_s:.1f}s")
    mom = torch.from_numpy(mom_np).to(dev)
    out = torch.empty(args.nevt, dtype=torch.float64, device=dev)
    m = me.MatrixElement(args.process)
    info = m.info()

    k_s, wall = bench_fp64(m, mom, out, args, stream)
    res = out.cpu().numpy()
    assert np.all(np.isfinite(res)), "non-finite results"
    value = args.nevt / wall
    flops_evt = info["flops_per_event"]
    achieved = flops_evt * args.nevt / k_s / 1e12
    kernel = f"k_me_gg<proc_{args.process}>"
    traffic = traffic_from_profile(args.process, kernel)
    log(f"fp64: {value:.3e} MEs/s, kernel {k_s * 1e3:.2f} ms")

    line = {
        "metric": "matrix elements/sec, gg->ttgg 1 GPU: FP64 (value) vs mixed vs surrogate (forms)",
        "value": value,
        "unit": "MEs/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": wall * 1e3,
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f64",
        "data": "synthetic: seeded RAMBO points, sqrt(s)=13 TeV",
        "config": {"workload": f"{args.process} |M|^2, {args.nevt} RAMBO points seed {args.seed}, "
                               f"{info['nhel_good']} helicities, {info['ndiag']} diagrams, "
                               f"{info['ncol']}x{info['ncol']} colour matrix",
                   "nevt": args.nevt, "parallelism": "single GPU, one event per lane"},
        "roofline": {"bound": "alu", "achieved": achieved, "peak": PEAK["fp64"], "unit": "TFLOP/s",
                     "frac": achieved / PEAK["fp64"], "traffic": traffic,
                     "kernel": kernel, "flops_per_event": flops_evt, "kernel_ms": k_s * 1e3},
        "forms": {"fp64": {"MEs_per_s": value, "ms_per_step": wall * 1e3}},
    }
    if "mixed" in forms:
        line["forms"]["mixed"] = bench_mixed(me, m, mom, mom_np, args, stream)
        log(f"mixed: {line['forms']['mixed']['MEs_per_s']:.3e} MEs/s")
    m.close()
    if "surrogate" in forms:
        del mom
        line["forms"]["surrogate"] = bench_surrogate(me, args, stream)
        log(f"surrogate: {line['forms']['surrogate']}")

    line["processes"] = {}
    if "gg_ttggg" in forms:
        line["processes"]["gg_ttggg"] = bench_process(me, "gg_ttggg", 1 << 18, 3, max(2, args.steps // 5), stream,
                                                      tol=args.tol if "mixed" in forms else None)
        log(f"gg_ttggg: {line['processes']['gg_ttggg']}")
    if "dy3j" in forms:
        # the paper's DY+3j subprocess (Sec. 3), a quark line + lepton pair
        line["processes"]["gux_taptamggux"] = bench_process(me, "gux_taptamggux", 1 << 20, 4, args.steps, stream,
                                                            check=64)
        log(f"dy3j: {line['processes']['gux_taptamggux']['MEs_per_s']:.3e} MEs/s")
    if "configs" in forms:
        line["processes"]["ee_mumu"] = bench_process(me, "ee_mumu", 16384, 0, args.steps, stream, check=64)
        line["processes"]["gg_tt"] = bench_process(me, "gg_tt", 1 << 20, 1, args.steps, stream, check=64)
        log(f"configs: ee_mumu {line['processes']['ee_mumu']['MEs_per_s']:.3e}, "
            f"gg_tt {line['processes']['gg_tt']['MEs_per_s']:.3e} MEs/s")
    if "colour" in forms:
        line["colour_forms"] = bench_colour_forms(me, stream, [("gg_ttgg", args.nevt, args.seed, 5),
                                                                ("gg_ttggg", 1 << 18, 3, 2)])
    if "mc" in forms:
        line["multichannel"] = bench_multichannel(me, stream, mom if "surrogate" not in forms else
                                                  torch.from_numpy(mom_np).to(dev), args.process, 5)
        log(f"multichannel: {line['multichannel']}")
    if "ps" in forms:
        line["phase_space"] = bench_phase_space(me, stream, args.nevt, host_gen_s)
        log(f"phase space: {line['phase_space']['points_per_s']:.3e} points/s")
    if "psmc" in forms:
        line["phase_space_multichannel"] = bench_ps_multichannel(me, stream, 1 << 20, 20)
        log(f"multi-channel phase space: {line['phase_space_multichannel']}")
    if "sweep" in forms:
        line["nevt_sweep"] = nevt_sweep(me, args.process, args.seed, [0, 1, 4, 16, 64], list(range(10, 21, 2)), stream)

    if not args.no_cpu:
        import oracle

        n = min(args.cpu_sample, args.nevt)
        threads = omp_threads()
        c0 = time.perf_counter()
        ref = oracle.me2(args.process, mom_np[:n])
        cpu_s = time.perf_counter() - c0
        n1 = min(args.cpu_sample_1t, n)
        omp_threads(1)
        c0 = time.perf_counter()
        oracle.me2(args.process, mom_np[:n1])
        cpu1_s = time.perf_counter() - c0
        omp_threads(threads)
        line["cpu_baseline"] = {"value": n / cpu_s, "unit": "MEs/s", "cores": threads, "kind": "oracle",
                                "sample": f"first {n} of the {args.nevt} points, float64 oracle "
                                          f"(colour-ordered Berends-Giele, OpenMP over events), {cpu_s:.1f} s",
                                "single_thread_MEs_per_s": n1 / cpu1_s,
                                "single_thread_sample": f"first {n1} points, {cpu1_s:.1f} s",
                                "cpu_model": cpu_model(), "host_cpus_visible": os.cpu_count()}
        line["fp64_parity_on_cpu_sample"] = parity_adjudication(args.process, mom_np[:n], res[:n], ref)
    print(json.dumps(line), flush=True)


if __name__ == "__main__":
    main()
