"""Throughput of the fast high-dimensional filter on one MI355X.

One step = one whole call of Algorithm 1 on the 2048x2048 RGB bilateral
workload (sigma_s = 5, S = 15, sigma_r = 0.12, K = 32, guide = image):
bisecting K-means of the guide, the K x K solve, weights and coefficients, the
4K row-filtered planes and the column pass with the recombination.  Inputs
are resident in HBM before the timed region.

Prints one JSON line.  `value` is the forward throughput (Mpix/s) of that
workload; beside it:
  * the spread of single steps (p10 / p50 / p90), the stage split, and the
    rooflines of the three largest kernels (row pass, column pass, the
    clustering's assignment step), each from its HIP-event time on the
    library's stream and its algorithmic FLOPs or bytes per launch;
  * quality: PSNR of eq. (21) against the GPU brute force of eqs. (1)-(2) and
    max-abs against the FP64 oracle fed the GPU's centers, next to every
    Mpix/s figure;
  * the other workloads: 256x256 RGB, forward + adjoint at 2048x2048, the
    512x512x32 hyperspectral image (FP32 and BF16 contractions, with the K
    sweep for the equal-PSNR comparison), nonlocal means at 1024x1024 (FP32,
    FP16, hard variant, K sweep), the ragged batch of 16 images (forward and
    forward + adjoint, HBM fraction), the window forms, the approximation
    error, the per-pixel least squares of eq. (10) against the surrogate
    eq. (11), the 3-D domain;
  * the FP64 CPU oracle timed on the host (cpu_baseline).

`--only LEG,...` runs the named legs only (for profiling); `--copy-calibration`
runs a plain device copy of known size (the reference for scaling rocprofv3's
FETCH_SIZE / WRITE_SIZE counters).
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

METRIC = "Mpix/s (fwd; fwd+bwd) at stated PSNR vs brute force, BF16 vs FP32 form"
HBM_PEAK_GBS = 8000.0        # MI355X HBM3E, published
FP32_VECTOR_PEAK = 157.3     # TFLOP/s, MI355X published FP32 vector (packed FMA)

# HBM bytes per launch at the 2048x2048 workload from rocprofv3 --pmc:
# FETCH_SIZE x 2.0 + WRITE_SIZE x 1.0 (KiB per dispatch, scaled by what the
# counters read for a 1 GiB device copy: 524,302 KiB fetched, 1,048,576 KiB
# written), for the kernels as they are in this tree (the assignment step:
# the mean over all of a call's launches); None where the counters have not
# been taken for the current version of the kernel.
MEASURED_TRAFFIC = {"row": 2246282317, "col": 2620828902, "lloyd": 40184826}

LEGS = ("c1", "quality", "c0", "fwd_bwd", "forms", "nlm", "batch", "window", "approx_error", "exact_ls", "volume",
        "cpu")


def parse():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=20)
    ap.add_argument("--warmup", type=int, default=3)
    ap.add_argument("--no-cpu", action="store_true", help="skip the CPU oracle leg")
    ap.add_argument("--quick", action="store_true", help="the 2048x2048 forward timing only")
    ap.add_argument("--only", default="", help="comma-separated legs to run (of: " + ", ".join(LEGS) + ")")
    ap.add_argument("--no-sweep", action="store_true", help="skip the K sweeps of the forms and nlm legs")
    ap.add_argument("--copy-calibration", type=int, default=0, metavar="MIB",
                    help="run a device copy of MIB MiB three times and exit")
    return ap.parse_args()


def psnr(a, b):
    """Eq. (21): -10 log10 of the channel-summed squared error per pixel."""
    d = (a.double() - b.double())
    mse = float((d * d).sum()) / (a.shape[-1] * a.shape[-2])
    return float("inf") if mse == 0 else -10.0 * math.log10(mse)


def timed(torch, fn, reps):
    """Median wall time (ms) of fn() over reps, synchronised around each call."""
    ts = []
    for _ in range(reps):
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        fn()
        torch.cuda.synchronize()
        ts.append((time.perf_counter() - t0) * 1000.0)
    ts.sort()
    return ts[len(ts) // 2]


def quantiles(ts):
    ts = sorted(ts)
    q = lambda p: ts[min(len(ts) - 1, max(0, int(round(p * (len(ts) - 1)))))]
    return {"p10": round(q(0.1), 4), "p50": round(q(0.5), 4), "p90": round(q(0.9), 4)}


def copy_calibration(mib):
    import torch
    n = mib * (1 << 20) // 4
    src = torch.rand(n, device="cuda")
    dst = torch.empty_like(src)
    for _ in range(3):
        dst.copy_(src)
    torch.cuda.synchronize()
    print(json.dumps({"copy_bytes_read": n * 4, "copy_bytes_written": n * 4, "reps": 3}))


def cache_read_rate(torch):
    """GB/s of a plain read (torch sum) of a 128 MiB buffer that stays in the
    256 MB last-level cache between repetitions: the rate the clustering's
    cache-resident assignment steps are measured against beside HBM."""
    x = torch.rand(32 << 20, device="cuda")
    for _ in range(3):
        x.sum()
    torch.cuda.synchronize()
    reps = 20
    t0 = time.perf_counter()
    for _ in range(reps):
        x.sum()
    torch.cuda.synchronize()
    return round(x.numel() * 4 * reps / (time.perf_counter() - t0) / 1e9, 1)


def pass_models(n, rho, K, S, box=False):
    """Algorithmic FLOPs and bytes per output pixel of the two convolution
    passes (FP32), split as the design splits the work of Algorithm 1.
    Whole forward: 4K rho + 2K^2 + Kn + 2K(n+1) + n + F_conv, with the
    convolutions F_conv = 4K(n+1)(2S+1) (two passes of 2S+1 taps, a multiply
    and an add each; 4K(n+1) for the box as running sums) and the exponentials
    (2K) not counted.  Row pass: distances and weights (4K rho), c = A^+ b
    (2K^2), c_l [f, 1] (Kn) and half of F_conv; column pass: the
    recombination (2K(n+1)), the division (n) and the other half.  Bytes: the
    row pass reads f and the guide and writes K(n+1) planes; the column pass
    reads the planes and the guide and writes g_hat."""
    conv_half = 2 * K * (n + 1) * (1 if box else (2 * S + 1))
    return {"row": (4 * (n + rho + K * (n + 1)), 4 * K * rho + 2 * K * K + K * n + conv_half),
            "col": (4 * (K * (n + 1) + rho + n), 2 * K * (n + 1) + n + conv_half)}


def o2_whole(oracle, np, f, g, cen, ss, sr, S, spatial):
    """The oracle's eqs. (13)-(16) over the whole image (separable FP64 window
    sums) with the GPU's centers; returns g, r_hat, and the magnitude sums."""
    c = np.asarray(cen, np.float64)
    P, _, _ = oracle.pinv(oracle.kernel_matrix(c, sr))
    ref, rden, _, mv, mr = oracle.fast_filter(f, g, c, P, ss, sr, S, spatial, conv_method="separable",
                                              return_terms=True)
    return ref, rden, mr


def maxabs_whole(oracle, np, out, f, g, cen, ss, sr, S, spatial):
    """Max-abs against the oracle, condition aware: over the pixels with
    |r_hat| >= 1e-2, and the count of the others (near a zero of the unguarded
    r_hat no finite-precision evaluation fixes g_hat = v / r_hat)."""
    t0 = time.perf_counter()
    ref, rden, _ = o2_whole(oracle, np, f, g, cen, ss, sr, S, spatial)
    o = out.cpu().numpy().astype(np.float64)
    well = np.abs(rden) >= 1e-2
    e = float(np.abs(o - ref)[:, well].max()) if well.any() else float("nan")
    return {"max_abs_vs_oracle": float(f"{e:.3e}"), "oracle_pixels": int(well.size),
            "pixels_abs_r_hat_below_1e-2": int((~well).sum()), "oracle_s": round(time.perf_counter() - t0, 1)}


def maxabs_sampled(oracle, np, out, f, g, cen, ss, sr, S, spatial, count, seed):
    """Max-abs against the oracle's direct per-pixel window sums at `count`
    random pixels plus the four corners."""
    H, W = f.shape[1:]
    rng = np.random.default_rng(seed)
    ys = np.concatenate([rng.integers(0, H, count), [0, 0, H - 1, H - 1]])
    xs = np.concatenate([rng.integers(0, W, count), [0, W - 1, 0, W - 1]])
    c = np.asarray(cen, np.float64)
    P, _, _ = oracle.pinv(oracle.kernel_matrix(c, sr))
    ref, _ = oracle.fast_filter_at(f, g, c, P, ss, sr, ys, xs, S=S, spatial=spatial)
    o = out.cpu().numpy()
    return float(f"{float(np.abs(o[:, ys, xs].T - ref).max()):.3e}")


def den_stats(info):
    return {k: info[k] for k in ("den_min", "den_nonpos", "den_small", "nonfinite")}


# ---------------------------------------------------------------------------
# legs

def leg_c1(torch, fhd, x, cfg, args):
    """The timed steps (value), their spread, stage split and rooflines."""
    H, W, n, K, S = cfg["H"], cfg["W"], cfg["n"], cfg["K"], cfg["S"]
    ss, sr = cfg["sigma_s"], cfg["sigma_r"]

    def step():
        return fhd.filter(x, sigma_s=ss, sigma_r=sr, K=K, radius=S)

    for _ in range(args.warmup):
        step()
    torch.cuda.synchronize()
    fhd.timing_enable(0, True)
    fhd.timing_read(0)
    fhd.timing_units(0)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for _ in range(args.steps):
        step()
    torch.cuda.synchronize()
    dt = time.perf_counter() - t0
    stages = fhd.timing_read(0)
    units = fhd.timing_units(0)
    fhd.timing_enable(0, False)
    # the spread of single steps (each synchronised), after the timed region
    single = []
    for _ in range(args.steps):
        torch.cuda.synchronize()
        t1 = time.perf_counter()
        step()
        torch.cuda.synchronize()
        single.append((time.perf_counter() - t1) * 1000.0)
    N = H * W
    avg = {s: (ms / cnt if cnt else 0.0) for s, (ms, cnt) in stages.items()}
    models = pass_models(n, n, K, S)
    rl = {}
    for k in ("row", "col"):
        bpx, fpx = models[k]
        sec = avg[k] * 1e-3
        gbs, tfs = bpx * N / sec / 1e9, fpx * N / sec / 1e12
        if k == "row":   # VALU-bound: FIR taps and c = A^+ b
            rl[k] = {"bound": "alu", "achieved": round(tfs, 2), "peak": FP32_VECTOR_PEAK, "unit": "TFLOP/s",
                     "frac": round(tfs / FP32_VECTOR_PEAK, 4)}
        else:
            rl[k] = {"bound": "hbm", "achieved": round(gbs, 1), "peak": HBM_PEAK_GBS, "unit": "GB/s",
                     "frac": round(gbs / HBM_PEAK_GBS, 4)}
        rl[k].update({"traffic": MEASURED_TRAFFIC.get(k), "kernel": f"{k} pass", "flops_per_px": fpx,
                      "bytes_per_px": bpx, "flops_per_launch": fpx * N, "bytes_per_launch": bpx * N,
                      "hbm_gbs": round(gbs, 1), "hbm_frac": round(gbs / HBM_PEAK_GBS, 4),
                      "avg_ms": round(avg[k], 4), "launches": stages[k][1],
                      "ms_per_step": round(stages[k][0] / args.steps, 4)})
    # the clustering's assignment step: 4 rho bytes per point of the jobs it
    # streams (the points of every job that has not stopped)
    nl = stages["lloyd"][1]
    if nl:
        b_launch = 4 * n * units["lloyd"] / nl
        gbs = b_launch / (avg["lloyd"] * 1e-3) / 1e9
        rl["lloyd"] = {"bound": "hbm", "achieved": round(gbs, 1), "peak": HBM_PEAK_GBS, "unit": "GB/s",
                       "frac": round(gbs / HBM_PEAK_GBS, 4), "traffic": MEASURED_TRAFFIC.get("lloyd"),
                       "kernel": "km_lloyd (2-means assignment step)", "bytes_per_point": 4 * n,
                       "bytes_per_launch": round(b_launch), "points_per_launch": round(units["lloyd"] / nl),
                       "avg_ms": round(avg["lloyd"], 4), "launches": nl,
                       "ms_per_step": round(stages["lloyd"][0] / args.steps, 4)}
    dom = max(rl, key=lambda k: rl[k]["ms_per_step"])
    res = {
        "value": round(N * args.steps / dt / 1e6, 2),
        "ms_per_step": round(dt * 1000.0 / args.steps, 4),
        "step_ms_spread": quantiles(single),
        "stage_ms": {s: round(avg[s] * (stages[s][1] / args.steps), 4) for s in avg if stages[s][1]},
        "roofline": dict(rl[dom], dominant_by="GPU time per step among the row pass, the column pass and "
                                              "the assignment steps"),
        "rooflines": rl,
    }
    return res


def leg_quality(torch, fhd, oracle, np, x, f, cfg):
    H, W, K, S, ss, sr = cfg["H"], cfg["W"], cfg["K"], cfg["S"], cfg["sigma_s"], cfg["sigma_r"]
    N = H * W
    brute = fhd.bruteforce(x, sigma_s=ss, sigma_r=sr, radius=S)
    ms_brute = timed(torch, lambda: fhd.bruteforce(x, sigma_s=ss, sigma_r=sr, radius=S), 5)
    o, cen, info = fhd.filter(x, sigma_s=ss, sigma_r=sr, K=K, radius=S, return_centers=True, info=True)
    q = {"psnr_vs_brute_db": round(psnr(o, brute), 2), **den_stats(info),
         "brute_force_mpix_s": round(N / ms_brute / 1e3, 1), "brute_force_ms": round(ms_brute, 3)}
    q.update(maxabs_whole(oracle, np, o, f, f, cen.numpy(), ss, sr, S, "gaussian"))
    return q


def leg_c0(torch, fhd, oracle, np, synth):
    c = synth.WORKLOADS["bf_rgb_256"]
    f = synth.workload_input("bf_rgb_256")
    x = torch.from_numpy(f).cuda()
    kw = dict(sigma_s=c["sigma_s"], sigma_r=c["sigma_r"], K=c["K"], radius=c["S"])
    run = lambda: fhd.filter(x, **kw)
    o, cen, info = fhd.filter(x, return_centers=True, info=True, **kw)
    ts = [timed(torch, run, 1) for _ in range(20)]
    brute = fhd.bruteforce(x, sigma_s=c["sigma_s"], sigma_r=c["sigma_r"], radius=c["S"])
    N = c["H"] * c["W"]
    leg = {"workload": "bf_rgb_256: 256x256 RGB bilateral, sigma_s 3 (S 9), sigma_r 0.1, K 16, FP32",
           "mpix_s": round(N / quantiles(ts)["p50"] / 1e3, 2), "ms": quantiles(ts),
           "psnr_vs_brute_db": round(psnr(o, brute), 2), **den_stats(info)}
    leg.update(maxabs_whole(oracle, np, o, f, f, cen.numpy(), c["sigma_s"], c["sigma_r"], c["S"], "gaussian"))
    return leg


def leg_fwd_bwd(torch, fhd, np, x, f, cfg, steps):
    K, S, ss, sr = cfg["K"], cfg["S"], cfg["sigma_s"], cfg["sigma_r"]
    N = cfg["H"] * cfg["W"]
    G = torch.from_numpy(np.random.default_rng(7).standard_normal(f.shape).astype(np.float32)).cuda()
    # the forward call keeps its row-filtered planes and coefficients for the adjoint
    sv = fhd.saved_buffer(cfg["n"], cfg["n"], cfg["H"], cfg["W"], K, sigma_s=ss, sigma_r=sr, radius=S)

    def fb():
        o, d, c = fhd.filter(x, sigma_s=ss, sigma_r=sr, K=K, radius=S, return_den=True, return_centers=True,
                             saved=sv)
        fhd.filter_backward(x, x, c, o, d, G, sigma_s=ss, sigma_r=sr, radius=S, saved=sv)

    fb()
    ms = timed(torch, fb, max(3, steps // 4))
    return {"mpix_s": round(N / ms / 1e3, 2), "ms_per_step": round(ms, 3),
            "saved_bytes": sv.numel(),
            "note": "one forward call (keeping its intermediates for the adjoint) plus one adjoint call "
                    "(dL/df, dL/dguide, dL/dsigma_r), same workload"}


def equal_psnr(sweep, form, ref_form, K_ref):
    """Mpix/s of `form` interpolated (linearly in PSNR between adjacent K) at
    the PSNR `ref_form` reaches at K_ref; None if `form` never reaches it."""
    target = sweep[ref_form][f"K{K_ref}"]["psnr_vs_brute_db"]
    pts = sorted(((v["psnr_vs_brute_db"], v["mpix_s"], int(k[1:])) for k, v in sweep[form].items()),
                 key=lambda t: t[2])
    for (p0, m0, k0), (p1, m1, k1) in zip(pts, pts[1:]):
        if p0 <= target <= p1 and p1 > p0:
            w = (target - p0) / (p1 - p0)
            return {"psnr_db": target, "mpix_s": round(m0 + w * (m1 - m0), 2), "between_K": [k0, k1]}
    for p, m, k in pts:
        if p == target:
            return {"psnr_db": target, "mpix_s": m, "between_K": [k, k]}
    return {"psnr_db": target, "mpix_s": None, "note": f"{form} never reaches it over the sweep"}


def leg_forms(torch, fhd, oracle, np, synth, sweep_on=True):
    c2 = synth.WORKLOADS["bf_hyper_512x32"]
    f = synth.workload_input("bf_hyper_512x32")
    h = torch.from_numpy(f).cuda()
    base = dict(sigma_s=c2["sigma_s"], sigma_r=c2["sigma_r"], radius=c2["S"])
    ref = fhd.bruteforce(h, **base)
    ms_b = timed(torch, lambda: fhd.bruteforce(h, **base), 3)
    N = c2["H"] * c2["W"]
    leg = {"workload": "hyper_512: 512x512x32 bands, guide = image, sigma_s 4 (S 12), sigma_r 0.2, K 64",
           "brute_force_mpix_s": round(N / ms_b / 1e3, 1)}
    outs = {}
    for form in ("fp32", "bf16"):
        run = lambda: fhd.filter(h, K=c2["K"], contract=form, **base)
        o, cen, info = fhd.filter(h, K=c2["K"], contract=form, return_centers=True, info=True, **base)
        outs[form] = o
        ms = timed(torch, run, 5)
        leg[form] = {"mpix_s": round(N / ms / 1e3, 2), "psnr_vs_brute_db": round(psnr(o, ref), 2),
                     "max_abs_vs_oracle_sampled": maxabs_sampled(oracle, np, o, f, f, cen.numpy(), c2["sigma_s"],
                                                                 c2["sigma_r"], c2["S"], "gaussian", 256, 41),
                     **den_stats(info)}
    leg["bf16_vs_fp32_max_abs"] = float((outs["bf16"] - outs["fp32"]).abs().max())
    if not sweep_on:
        return leg
    sweep = {}
    for form in ("fp32", "bf16"):
        sweep[form] = {}
        for K in (8, 16, 32, 48, 64, 96, 128):
            run = lambda: fhd.filter(h, K=K, contract=form, **base)
            o = run()
            ms = timed(torch, run, 3)
            sweep[form][f"K{K}"] = {"mpix_s": round(N / ms / 1e3, 2), "psnr_vs_brute_db": round(psnr(o, ref), 2)}
    leg["K_sweep"] = sweep
    leg["bf16_at_fp32_psnr_K64"] = equal_psnr(sweep, "bf16", "fp32", 64)
    return leg


def leg_nlm(torch, fhd, oracle, np, synth, sweep_on=True):
    """Nonlocal means on the 1024x1024 workload: the patch-PCA guide, then the
    filter with FP32 and FP16 distance contractions and the hard variant;
    PSNR against the GPU brute force on the same guide and, for denoising,
    against the clean image; max-abs against the oracle fed the GPU's guide
    and centers; K sweep of both forms."""
    c3 = synth.WORKLOADS["nlm_rgb_1024"]
    noisy, clean = synth.workload_input("nlm_rgb_1024")
    x = torch.from_numpy(noisy).cuda()
    cl = torch.from_numpy(clean).cuda()
    N = c3["H"] * c3["W"]
    g = fhd.nlm_guide(x, patch=c3["patch"], dims=c3["dims"])
    ms_guide = timed(torch, lambda: fhd.nlm_guide(x, patch=c3["patch"], dims=c3["dims"]), 3)
    kw = dict(sigma_r=c3["sigma_r"], spatial="box", radius=c3["S"])
    ref = fhd.bruteforce(x, g, **kw)
    ms_b = timed(torch, lambda: fhd.bruteforce(x, g, **kw), 3)
    gh = g.cpu().numpy()
    leg = {"workload": "nlm_rgb_1024: 1024x1024 RGB, noise 0.1, 5x5x3 patches -> 16-d PCA guide, "
                       "box 21x21, sigma_r 0.1 sqrt(75), K 32",
           "guide_ms": round(ms_guide, 3), "brute_force_mpix_s": round(N / ms_b / 1e3, 1),
           "noisy_psnr_vs_clean_db": round(psnr(x, cl), 2)}
    for form, coef in (("fp32", "lsq"), ("fp16", "lsq"), ("fp32", "hard")):
        run = lambda: fhd.filter(x, g, K=c3["K"], contract=form, coef=coef, **kw)
        o, cen, info = fhd.filter(x, g, K=c3["K"], contract=form, coef=coef, return_centers=True, info=True, **kw)
        ms = timed(torch, run, 5)
        e = (o - ref).abs().amax(0)
        ent = {"mpix_s": round(N / ms / 1e3, 2), "mpix_s_with_guide": round(N / (ms + ms_guide) / 1e3, 2),
               "psnr_vs_brute_db": round(psnr(o, ref), 2), "median_abs_err_vs_brute": float(e.median()),
               "denoised_psnr_vs_clean_db": round(psnr(o, cl), 2), **den_stats(info)}
        if coef == "lsq":
            ent.update(maxabs_whole(oracle, np, o, noisy, gh, cen.numpy(), None, c3["sigma_r"], c3["S"], "box"))
        leg[form if coef == "lsq" else "hard_fp32"] = ent
    if not sweep_on:
        return leg
    sweep = {}
    for form in ("fp32", "fp16"):
        sweep[form] = {}
        for K in (8, 16, 32, 48, 64):
            run = lambda: fhd.filter(x, g, K=K, contract=form, **kw)
            o = run()
            ms = timed(torch, run, 3)
            sweep[form][f"K{K}"] = {"mpix_s": round(N / ms / 1e3, 2), "psnr_vs_brute_db": round(psnr(o, ref), 2)}
    leg["K_sweep"] = sweep
    leg["fp16_at_fp32_psnr_K32"] = equal_psnr(sweep, "fp16", "fp32", 32)
    return leg


def leg_batch(torch, np, fhd, oracle, synth):
    """The ragged batch of 16 RGB images (384x384 .. 768x1024): one batched
    forward call, then forward plus the batched adjoint (image, guide and
    sigma_r gradients).  HBM fraction from the algorithmic bytes per pixel of
    the two-pass design (forward 4 [2n + 2 rho + 2K(n+1)], adjoint
    4 [4K(n+1) + 2K + 7n + 5 rho + 2])."""
    c4 = synth.WORKLOADS["bf_rgb_batch16"]
    imgs_np = synth.workload_input("bf_rgb_batch16")
    imgs = [torch.from_numpy(a).cuda() for a in imgs_np]
    flat, sizes = fhd.pack_batch(imgs)
    n, K, S = c4["n"], c4["K"], c4["S"]
    N = sum(h * w for h, w in sizes)
    kw = dict(sigma_s=c4["sigma_s"], sigma_r=c4["sigma_r"], radius=S)
    G = torch.from_numpy(np.random.default_rng(11).standard_normal(flat.numel()).astype(np.float32)).cuda()
    sv = fhd.saved_buffer(n, n, [h for h, _ in sizes], [w for _, w in sizes], K, **kw)

    def fwd():
        return fhd.filter_batch(flat, sizes, n, K=K, return_den=True, **kw)

    def fb():
        # the forward call keeps its intermediates for the adjoint
        out, den, cen, keff = fhd.filter_batch(flat, sizes, n, K=K, return_den=True, saved=sv, **kw)
        fhd.filter_batch_backward(flat, sizes, n, cen, keff, out, den, G, saved=sv, **kw)

    fb()
    ms_f = timed(torch, fwd, 5)
    ms_fb = timed(torch, fb, 5)
    out, den, cen, keff = fwd()
    worst, o = 0.0, 0
    for b, (h, w) in enumerate(sizes):
        ob = out[o * n:(o + h * w) * n].reshape(n, h, w)
        o += h * w
        worst = max(worst, maxabs_sampled(oracle, np, ob, imgs_np[b], imgs_np[b], cen[b, :keff[b]].numpy(),
                                          c4["sigma_s"], c4["sigma_r"], S, "gaussian", 16, 100 + b))
    rho = n
    bf = 4 * (2 * n + 2 * rho + 2 * K * (n + 1))
    bb = 4 * (4 * K * (n + 1) + 2 * K + 7 * n + 5 * rho + 2)
    gbs = (bf + bb) * N / (ms_fb * 1e-3) / 1e9
    return {"workload": "bf_rgb_batch16: 16 RGB images 384x384 .. 768x1024, sigma_s 3 (S 9), "
                        "sigma_r 0.1, K 32",
            "pixels": N, "fwd_mpix_s": round(N / ms_f / 1e3, 2), "fwd_ms": round(ms_f, 3),
            "fwd_bwd_mpix_s": round(N / ms_fb / 1e3, 2), "fwd_bwd_ms": round(ms_fb, 3),
            "fwd_bwd_model_bytes_per_px": bf + bb, "fwd_bwd_hbm_gbs": round(gbs, 1), "saved_bytes": sv.numel(),
            "fwd_bwd_hbm_frac": round(gbs / HBM_PEAK_GBS, 4),
            "max_abs_vs_oracle_sampled": worst}


def leg_window(torch, fhd, x, sr, K):
    """The 2048x2048 RGB workload over sigma_s 2 .. 20 (the paper's sweep of
    the spatial scale): the fast filter with the truncated-Gaussian FIR
    window (S = 3 sigma_s) and with the recursive Gaussian (the paper's O(1)
    convolution), each with its Mpix/s and PSNR against the GPU brute force
    of the truncated window, and that brute force's own Mpix/s: where the
    clustered filter overtakes the direct sum on this GPU."""
    N = x.shape[1] * x.shape[2]
    leg = {"workload": "bf_rgb_2048, sigma_r 0.12, K 32: window forms and the brute force over sigma_s"}
    for ss in (2.0, 3.0, 5.0, 8.0, 12.0, 20.0):
        S = int(round(3 * ss))
        bf = lambda: fhd.bruteforce(x, sigma_s=ss, sigma_r=sr, radius=S)
        brute = bf()
        ms_b = timed(torch, bf, 3)
        ent = {"brute_force": {"mpix_s": round(N / ms_b / 1e3, 2), "ms": round(ms_b, 3)}}
        for name, kw in (("fir", dict(spatial="gaussian", radius=S)), ("recursive", dict(spatial="young"))):
            run = lambda: fhd.filter(x, sigma_s=ss, sigma_r=sr, K=K, **kw)
            o = run()
            ms = timed(torch, run, 5)
            ent[name] = {"mpix_s": round(N / ms / 1e3, 2), "ms": round(ms, 3),
                         "psnr_vs_brute_db": round(psnr(o, brute), 2)}
        leg[f"sigma_s_{int(ss)}_S{S}"] = ent
    return leg


def leg_approx_error(torch, fhd, synth):
    """E_ls (eq. (10) at c = A^+ b, averaged over the pixels: the least-squares
    error of Sec. II-A, not the clustering error E_K of eq. (20)) against K for a
    3-dimensional and a 32-dimensional guide, clusters from the library's own
    bisecting K-means: the fall of the approximation error with K."""
    legs = {}
    for name, K_list in (("bf_rgb_256", (4, 8, 16, 32, 64)), ("bf_hyper_512x32", (8, 16, 32, 64))):
        c = synth.WORKLOADS[name]
        g = torch.from_numpy(synth.workload_input(name)).cuda()
        row = {"guide": f"{name}: rho {g.shape[0]}, sigma_r {c['sigma_r']}, window {2 * c['S'] + 1}^2"}
        for K in K_list:
            cen, _ = fhd.cluster(g, K)
            run = lambda: fhd.approx_error(g, cen, sigma_r=c["sigma_r"], radius=c["S"], spatial="box",
                                           per_pixel=False)
            _, Els = run()
            ms = timed(torch, run, 2)
            row[f"K{K}"] = {"E_ls": float(f"{Els:.4e}"), "K_eff": int(cen.shape[0]), "ms": round(ms, 2)}
        legs[name] = row
    return legs


def leg_exact_ls(torch, fhd, synth):
    """Sec. II-A's comparison of the per-pixel fit eq. (10) with the surrogate
    eq. (11), in the setting of the paper's grayscale study (256 x 256, sigma_s
    2, sigma_r 20/255, K 4) and on the 256 x 256 RGB workload (K 16, S 9): time
    and PSNR against the brute force of the filter with each set of
    coefficients, the objective of eq. (10) averaged over the pixels at each
    minimiser, and how far the surrogate's coefficients lie from the exact
    ones (median and 90th percentile over the pixels of |A^+ b - c*| / |c*|,
    and of both norms)."""
    legs = {}
    gray = synth.voronoi_rgb(256, 256, 24, 0.05, 1301)[:1].copy()
    c0 = synth.WORKLOADS["bf_rgb_256"]
    cases = (("gray_256", "256x256 grayscale (one Voronoi channel, noise 0.05), sigma_s 2 (S 6), sigma_r 20/255, "
                          "K 4", gray, 4, 2.0, 20.0 / 255.0, None),
             ("bf_rgb_256", "256x256 RGB, sigma_s 3 (S 9), sigma_r 0.1, K 16", synth.workload_input("bf_rgb_256"),
              c0["K"], c0["sigma_s"], c0["sigma_r"], c0["S"]))
    for name, desc, img, K, ss, sr, S in cases:
        x = torch.from_numpy(img).cuda()
        cen, _ = fhd.cluster(x, K)
        kw = dict(sigma_s=ss, sigma_r=sr, radius=S)
        ref = fhd.bruteforce(x, x, **kw)
        row = {"workload": desc, "K_eff": int(cen.shape[0]),
               "brute_force_ms": round(timed(torch, lambda: fhd.bruteforce(x, x, **kw), 3), 3)}
        for coef, key in (("lsq", "eq11_surrogate"), ("exact", "eq10_exact")):
            run = lambda: fhd.filter_centers(x, x, cen, coef=coef, **kw)
            o = run()
            row[key] = {"ms": round(timed(torch, run, 3), 3), "psnr_vs_brute_db": round(psnr(o, ref), 2)}
        cf, o10, o11 = fhd.exact_ls(x, cen, sigma_r=sr, sigma_s=ss, radius=S)
        row["eq10_objective_mean"] = {"at_exact": float(f"{float(o10.double().mean()):.4e}"),
                                      "at_surrogate": float(f"{float(o11.double().mean()):.4e}")}
        row["exact_ls_ms"] = round(timed(torch, lambda: fhd.exact_ls(x, cen, sigma_r=sr, sigma_s=ss, radius=S,
                                                                     obj=False, obj11=False), 3), 3)
        # the surrogate's coefficients A^+ b(i), formed here for the comparison
        _, P, _, _ = fhd.pinv(cen, sr)
        X = x.reshape(x.shape[0], -1).t().double()
        mu = torch.as_tensor(cen, dtype=torch.float64, device=x.device)
        B = torch.exp(-((X[:, None, :] - mu[None, :, :]) ** 2).sum(-1) / (2.0 * sr * sr))
        Cs = B @ P.to(x.device).t()
        Ce = cf.reshape(cf.shape[0], -1).t().double()
        rel = (Cs - Ce).norm(dim=1) / Ce.norm(dim=1).clamp_min(1e-30)
        qs = torch.tensor([0.5, 0.9], device=x.device)
        q = torch.quantile(rel.float(), qs)
        ne, ns = torch.quantile(Ce.norm(dim=1).float(), qs), torch.quantile(Cs.norm(dim=1).float(), qs)
        row["coef_rel_diff"] = {"median": float(f"{float(q[0]):.3e}"), "p90": float(f"{float(q[1]):.3e}")}
        # the minimum-norm fit of eq. (10) keeps every singular direction above
        # the pseudo-inverse's tolerance; in near-flat windows the K basis
        # functions are nearly dependent over the samples and its coefficients
        # grow large while the fit itself changes little
        row["coef_norm"] = {"exact_median": float(f"{float(ne[0]):.3e}"), "exact_p90": float(f"{float(ne[1]):.3e}"),
                            "surrogate_median": float(f"{float(ns[0]):.3e}"),
                            "surrogate_p90": float(f"{float(ns[1]):.3e}")}
        legs[name] = row
    return legs


def leg_volume(torch, fhd, synth):
    """Algorithm 1 on a 3-D domain: a 64 x 256 x 256 three-component vector
    field (as many voxels as the 2048^2 image has pixels), window [-6,6]^3
    (sigma_s 2), sigma_r 0.12, K 32; Mvox/s and the stage split."""
    v = torch.from_numpy(synth.voronoi_volume(64, 256, 256, 256, 0.05, 1005)).cuda()
    run = lambda: fhd.filter_volume(v, sigma_s=2.0, sigma_r=0.12, K=32)
    run()
    ms = timed(torch, run, 5)
    fhd.timing_enable(0, True)
    fhd.timing_read(0)
    run()
    st = fhd.timing_read(0)
    fhd.timing_enable(0, False)
    N = v.shape[1] * v.shape[2] * v.shape[3]
    out = run()
    brute = lambda: fhd.bruteforce_volume(v, sigma_s=2.0, sigma_r=0.12)
    ref = brute()
    ms_b = timed(torch, brute, 2)
    return {"workload": "volume_64x256x256: 3-component 3-D Voronoi field, noise 0.05, sigma_s 2 (S 6), "
                        "sigma_r 0.12, K 32",
            "mvox_s": round(N / ms / 1e3, 1), "ms": round(ms, 3),
            "stage_ms": {k: round(t, 3) for k, (t, nl) in st.items() if nl},
            "psnr_vs_brute_db": round(-10.0 * math.log10(float(((out.double() - ref.double()) ** 2).sum()) / N), 2),
            "brute_force_mvox_s": round(N / ms_b / 1e3, 1)}


def cpu_model():
    try:
        for line in open("/proc/cpuinfo"):
            if line.startswith("model name"):
                return line.split(":", 1)[1].strip()
    except OSError:
        pass
    return "unknown"


def leg_cpu(np, synth, f, cfg):
    """The FP64 oracle on the host: Algorithm 1 end to end (O-2) on the whole
    2048x2048 image (the value), the brute force of eqs. (1)-(2) (O-1) on a
    512x512 crop of it, and both on the 256x256 workload with one thread."""
    import oracle
    threads = oracle.threads()
    t0 = time.perf_counter()
    res = oracle.fhd_filter(f, f, cfg["sigma_s"], cfg["sigma_r"], cfg["K"], S=cfg["S"], conv_method="separable")
    t_o2 = time.perf_counter() - t0
    # split: the clustering (NumPy, one thread) against the rest
    t0 = time.perf_counter()
    oracle.fhd_filter(f, f, cfg["sigma_s"], cfg["sigma_r"], cfg["K"], S=cfg["S"], conv_method="separable",
                      centers=res.centers)
    t_rest = time.perf_counter() - t0
    N = cfg["H"] * cfg["W"]
    crop = np.ascontiguousarray(f[:, :512, :512])
    t0 = time.perf_counter()
    oracle.bruteforce(crop, crop, cfg["sigma_s"], cfg["sigma_r"], S=cfg["S"])
    t_o1 = time.perf_counter() - t0
    c0 = synth.WORKLOADS["bf_rgb_256"]
    f0 = synth.workload_input("bf_rgb_256")
    prev = oracle.set_threads(1)
    try:
        t0 = time.perf_counter()
        oracle.fhd_filter(f0, f0, c0["sigma_s"], c0["sigma_r"], c0["K"], S=c0["S"], conv_method="separable")
        t_c0_o2 = time.perf_counter() - t0
        t0 = time.perf_counter()
        oracle.bruteforce(f0, f0, c0["sigma_s"], c0["sigma_r"], S=c0["S"])
        t_c0_o1 = time.perf_counter() - t0
    finally:
        oracle.set_threads(prev)
    return {"value": round(N / t_o2 / 1e6, 4), "unit": "Mpix/s", "cores": threads, "kind": "oracle",
            "sample": f"FP64 oracle O-2, the whole of Algorithm 1 on the whole 2048x2048 image of the same "
                      f"input and parameters ({t_o2:.1f} s): bisecting K-means in NumPy on one thread "
                      f"({t_o2 - t_rest:.1f} s), the K x K solve, weights and the separable convolutions in C "
                      f"with OpenMP on {threads} threads ({t_rest:.1f} s)",
            "cpu_model": cpu_model(), "threads_by_stage": {"clustering": 1, "solve_weights_convolutions": threads},
            "o1_brute_force": {"mpix_s": round(512 * 512 / t_o1 / 1e6, 4), "threads": threads,
                               "sample": f"eqs. (1)-(2) on the 512x512 top-left crop, S 15 ({t_o1:.2f} s)"},
            "one_thread_bf_rgb_256": {"o2_mpix_s": round(256 * 256 / t_c0_o2 / 1e6, 4),
                                      "o1_mpix_s": round(256 * 256 / t_c0_o1 / 1e6, 4),
                                      "o2_s": round(t_c0_o2, 2), "o1_s": round(t_c0_o1, 2)}}


def main():
    args = parse()
    if args.gpus != 1:
        print(f"bench.py measures one GPU only: the library has no multi-GPU path "
              f"(asked for --gpus {args.gpus})", file=sys.stderr)
        sys.exit(2)
    if args.copy_calibration:
        copy_calibration(args.copy_calibration)
        return
    import numpy as np
    import torch

    import paper_1811_02363_amd as fhd
    import synth

    only = set(x for x in args.only.split(",") if x)
    bad = only - set(LEGS)
    if bad:
        print(f"unknown legs {sorted(bad)}; legs are {LEGS}", file=sys.stderr)
        sys.exit(2)

    def want(leg):
        if only:
            return leg in only
        if args.quick:
            return leg == "c1"
        return leg != "cpu" or not args.no_cpu

    cfg = synth.WORKLOADS["bf_rgb_2048"]
    f = synth.workload_input("bf_rgb_2048")
    x = torch.from_numpy(f).cuda()
    torch.cuda.synchronize()
    res = {"metric": METRIC, "value": None, "unit": "Mpix/s", "n_gpus": 1, "steps": args.steps,
           "warmup": args.warmup, "ms_per_step": None, "higher_is_better": True, "scaling": "weak",
           "vs_baseline": None, "dtype": "f32", "data": "synthetic",
           "config": {"workload": "bf_rgb_2048: 2048x2048 RGB bilateral, guide = image, "
                                  "sigma_s 5 (S 15), sigma_r 0.12, K 32, forward, FP32 form",
                      "H": cfg["H"], "W": cfg["W"], "n": cfg["n"], "rho": cfg["n"], "K": cfg["K"], "S": cfg["S"],
                      "sigma_s": cfg["sigma_s"], "sigma_r": cfg["sigma_r"]}}
    oracle = None
    if any(want(k) for k in ("quality", "c0", "forms", "nlm", "batch")):
        import oracle
    t_start = time.perf_counter()

    def run(leg, key, fn):
        if not want(leg):
            return
        t0 = time.perf_counter()
        out = fn()
        if key is None:
            res.update(out)
        else:
            res[key] = out
        print(f"bench: {leg} done in {time.perf_counter() - t0:.1f} s "
              f"({time.perf_counter() - t_start:.0f} s total)", file=sys.stderr, flush=True)

    run("c1", None, lambda: leg_c1(torch, fhd, x, cfg, args))
    if "roofline" in res:
        res["roofline"]["cache_read_gbs_measured"] = cache_read_rate(torch)
    run("quality", "quality", lambda: leg_quality(torch, fhd, oracle, np, x, f, cfg))
    run("c0", "c0", lambda: leg_c0(torch, fhd, oracle, np, synth))
    run("fwd_bwd", "fwd_bwd", lambda: leg_fwd_bwd(torch, fhd, np, x, f, cfg, args.steps))
    run("forms", "forms", lambda: leg_forms(torch, fhd, oracle, np, synth, not args.no_sweep))
    run("nlm", "nlm", lambda: leg_nlm(torch, fhd, oracle, np, synth, not args.no_sweep))
    run("batch", "batch", lambda: leg_batch(torch, np, fhd, oracle, synth))
    run("window", "window", lambda: leg_window(torch, fhd, x, cfg["sigma_r"], cfg["K"]))
    run("approx_error", "approx_error", lambda: leg_approx_error(torch, fhd, synth))
    run("exact_ls", "exact_ls", lambda: leg_exact_ls(torch, fhd, synth))
    run("volume", "volume", lambda: leg_volume(torch, fhd, synth))
    run("cpu", "cpu_baseline", lambda: leg_cpu(np, synth, f, cfg))
    print(json.dumps(res))


if __name__ == "__main__":
    main()
