"""Throughput of the fast high-dimensional filter on one MI355X.

One step = one whole call of Algorithm 1 on the 2048x2048 RGB bilateral
workload (sigma_s = 5, S = 15, sigma_r = 0.12, K = 32, guide = image):
bisecting K-means of the guide, the K x K solve, weights and coefficients, the
4K row-filtered planes and the column pass with the recombination.  Inputs
are resident in HBM before the timed region.

Prints one JSON line: the forward throughput (Mpix/s) as `value`; the
approximation quality (PSNR of eq. (21) against the GPU brute-force filter of
eqs. (1)-(2)) and the brute force's own throughput; forward + adjoint
throughput on the same workload; the FP32 and BF16 forms of the distance
contraction on the 512x512x32 hyperspectral workload (Mpix/s and PSNR each);
nonlocal means on the 1024x1024 workload (FP32 and FP16 forms); the ragged
batch of 16 images, forward and forward + adjoint, with its HBM fraction; the
roofline of the dominant kernel (algorithmic bytes and FLOPs per launch /
HIP-event duration on the library's stream); and the FP64 CPU oracle timed on
the same workload (whole image by default).

`--copy-calibration` instead runs a plain device copy of known size (the
reference for scaling rocprofv3's FETCH_SIZE / WRITE_SIZE counters).
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

# HBM bytes per launch of the two convolution passes at the 2048x2048 workload
# from rocprofv3 --pmc: FETCH_SIZE x 2.0 + WRITE_SIZE x 1.0 (KiB per dispatch,
# scaled by what the counters read for a 1 GiB device copy: 524,302 KiB
# fetched, 1,048,576 KiB written), for the kernels as they are in this tree;
# an entry is None when the counters have not been taken for that version.
MEASURED_TRAFFIC = {"row": 2250091136, "col": 2494573909}


def parse():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=20)
    ap.add_argument("--warmup", type=int, default=3)
    ap.add_argument("--no-cpu", action="store_true", help="skip the CPU oracle leg")
    ap.add_argument("--quick", action="store_true",
                    help="forward timing only (no quality, adjoint or precision legs)")
    ap.add_argument("--cpu-crop", type=int, default=2048,
                    help="side of the top-left crop the CPU oracle filters (2048 = whole image)")
    ap.add_argument("--copy-calibration", type=int, default=0, metavar="MIB",
                    help="run a device copy of MIB MiB three times and exit")
    return ap.parse_args()


def psnr(a, b):
    """Eq. (21): -10 log10 of the channel-summed squared error per pixel."""
    d = (a.double() - b.double())
    mse = float((d * d).sum()) / (a.shape[-1] * a.shape[-2])
    return float("inf") if mse == 0 else -10.0 * math.log10(mse)


def cpu_baseline(f, cfg, crop):
    """The FP64 oracle (Algorithm 1 end to end, separable convolutions) on a
    crop x crop top-left piece of the same input with the same parameters."""
    import oracle
    sub = f[:, :crop, :crop].copy()
    threads = int(os.environ.get("OMP_NUM_THREADS", os.cpu_count() or 1))
    t0 = time.perf_counter()
    oracle.fhd_filter(sub, sub, cfg["sigma_s"], cfg["sigma_r"], cfg["K"], S=cfg["S"],
                      conv_method="separable")
    dt = time.perf_counter() - t0
    h, w = sub.shape[1:]
    what = "the whole image" if (h, w) == f.shape[1:] else f"the {h}x{w} top-left crop"
    return {"value": round(h * w / dt / 1e6, 4), "unit": "Mpix/s", "cores": threads,
            "kind": "oracle",
            "sample": f"FP64 oracle, whole Algorithm 1 (bisecting K-means in NumPy, one thread; "
                      f"K x K solve; convolutions in C with OpenMP on {threads} threads) on {what} "
                      f"of the same input and parameters ({dt:.1f} s)"}


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


def copy_calibration(mib):
    import torch
    n = mib * (1 << 20) // 4
    src = torch.rand(n, device="cuda")
    dst = torch.empty_like(src)
    for _ in range(3):
        dst.copy_(src)
    torch.cuda.synchronize()
    print(json.dumps({"copy_bytes_read": n * 4, "copy_bytes_written": n * 4, "reps": 3}))


def row_col_models(n, rho, K, S):
    """Algorithmic bytes and FLOPs per output pixel of the two passes (FP32).
    FIR: a symmetric (2S+1)-tap filter costs S + 1 multiplies and 2S adds."""
    fir = K * (n + 1) * (3 * S + 1)
    weights = 2 * rho * K + K                   # distances and scaling (exp not counted)
    row_flops = weights + 2 * K * K + K * n + fir   # + c = A^+ b and c [f, 1]
    col_flops = weights + fir + 2 * K * (n + 1) + n  # + recombination and division
    row_bytes = 4 * (n + rho + K * (n + 1))
    col_bytes = 4 * (K * (n + 1) + rho + n)
    return {"row": (row_bytes, row_flops), "col": (col_bytes, col_flops)}


def error_stats(out, den, ref):
    """PSNR of eq. (21) against the reference, the median and maximum absolute
    error, and the normaliser statistics (the least-squares coefficients can
    drive r_hat to or through zero, where the unguarded ratio blows up)."""
    e = (out - ref).abs().amax(0)
    return {"psnr_vs_brute_db": round(psnr(out, ref), 2),
            "median_abs_err": float(e.median()), "max_abs_err": float(e.max()),
            "den_min": float(den.min()), "den_nonpos": int((den <= 0).sum()),
            "den_below_1e-2": int((den < 1e-2).sum())}


def nlm_leg(torch, fhd, synth):
    """Nonlocal means on the 1024x1024 workload: the patch-PCA guide, then the
    filter with FP32 and FP16 distance contractions; PSNR against the GPU
    brute force on the same guide and, for denoising, against the clean image."""
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
    leg = {"workload": "nlm_rgb_1024: 1024x1024 RGB, noise 0.1, 5x5x3 patches -> 16-d PCA guide, "
                       "box 21x21, sigma_r 0.1 sqrt(75), K 32",
           "guide_ms": round(ms_guide, 3), "brute_force_mpix_s": round(N / ms_b / 1e3, 1),
           "noisy_psnr_vs_clean_db": round(psnr(x, cl), 2)}
    for form, coef in (("fp32", "lsq"), ("fp16", "lsq"), ("fp32", "hard")):
        run = lambda: fhd.filter(x, g, K=c3["K"], contract=form, coef=coef, **kw)
        o, d = fhd.filter(x, g, K=c3["K"], contract=form, coef=coef, return_den=True, **kw)
        ms = timed(torch, run, 5)
        leg[form if coef == "lsq" else "hard_fp32"] = dict(
            error_stats(o, d, ref), mpix_s=round(N / ms / 1e3, 2),
            mpix_s_with_guide=round(N / (ms + ms_guide) / 1e3, 2),
            denoised_psnr_vs_clean_db=round(psnr(o, cl), 2))
    return leg


def window_leg(torch, fhd, x, sr, K):
    """The 2048x2048 RGB workload with the truncated-Gaussian FIR window and
    with the recursive Gaussian (the paper's O(1) convolution), at sigma_s 5
    and 20: Mpix/s and PSNR against the GPU brute force with the truncated
    window of radius 3 sigma_s.  The FIR's cost grows with the radius; the
    recursion's does not."""
    N = x.shape[1] * x.shape[2]
    leg = {"workload": "bf_rgb_2048, sigma_r 0.12, K 32: window forms at sigma_s 5 and 20"}
    for ss in (5.0, 20.0):
        S = int(round(3 * ss))
        brute = fhd.bruteforce(x, sigma_s=ss, sigma_r=sr, radius=S)
        ent = {}
        for name, kw in (("fir", dict(spatial="gaussian", radius=S)), ("recursive", dict(spatial="young"))):
            run = lambda: fhd.filter(x, sigma_s=ss, sigma_r=sr, K=K, **kw)
            o = run()
            ms = timed(torch, run, 5)
            ent[name] = {"mpix_s": round(N / ms / 1e3, 2), "ms": round(ms, 3),
                         "psnr_vs_brute_db": round(psnr(o, brute), 2)}
        leg[f"sigma_s_{int(ss)}_S{S}"] = ent
    return leg


def approx_error_leg(torch, fhd, synth):
    """E_ls (eq. (10) at c = A^+ b, averaged over the pixels: the least-squares
    error of Sec. II-A, not the clustering error E_K of eq. (20)) against K for a
    3-dimensional and a 32-dimensional guide, clusters from the library's own
    bisecting K-means: the fall of the approximation error with K (Sec. II-A)."""
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


def volume_leg(torch, fhd, synth):
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


def batch_leg(torch, np, fhd, synth):
    """The ragged batch of 16 RGB images (384x384 .. 768x1024): one batched
    forward call, then forward plus the batched adjoint (image, guide and
    sigma_r gradients).  HBM fraction from the algorithmic bytes per pixel of
    the two-pass design (forward 4 [2n + 2 rho + 2K(n+1)], adjoint
    4 [4K(n+1) + 2K + 7n + 5 rho + 2])."""
    c4 = synth.WORKLOADS["bf_rgb_batch16"]
    imgs = [torch.from_numpy(a).cuda() for a in synth.workload_input("bf_rgb_batch16")]
    flat, sizes = fhd.pack_batch(imgs)
    n, K, S = c4["n"], c4["K"], c4["S"]
    N = sum(h * w for h, w in sizes)
    kw = dict(sigma_s=c4["sigma_s"], sigma_r=c4["sigma_r"], radius=S)
    G = torch.from_numpy(np.random.default_rng(11).standard_normal(flat.numel()).astype(np.float32)).cuda()

    def fwd():
        return fhd.filter_batch(flat, sizes, n, K=K, return_den=True, **kw)

    def fb():
        out, den, cen, keff = fwd()
        fhd.filter_batch_backward(flat, sizes, n, cen, keff, out, den, G, **kw)

    fb()
    ms_f = timed(torch, fwd, 5)
    ms_fb = timed(torch, fb, 5)
    rho = n
    bf = 4 * (2 * n + 2 * rho + 2 * K * (n + 1))
    bb = 4 * (4 * K * (n + 1) + 2 * K + 7 * n + 5 * rho + 2)
    gbs = (bf + bb) * N / (ms_fb * 1e-3) / 1e9
    return {"workload": "bf_rgb_batch16: 16 RGB images 384x384 .. 768x1024, sigma_s 3 (S 9), "
                        "sigma_r 0.1, K 32",
            "pixels": N, "fwd_mpix_s": round(N / ms_f / 1e3, 2), "fwd_ms": round(ms_f, 3),
            "fwd_bwd_mpix_s": round(N / ms_fb / 1e3, 2), "fwd_bwd_ms": round(ms_fb, 3),
            "fwd_bwd_model_bytes_per_px": bf + bb, "fwd_bwd_hbm_gbs": round(gbs, 1),
            "fwd_bwd_hbm_frac": round(gbs / HBM_PEAK_GBS, 4)}


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

    cfg = synth.WORKLOADS["bf_rgb_2048"]
    H, W, n, K, S = cfg["H"], cfg["W"], cfg["n"], cfg["K"], cfg["S"]
    ss, sr = cfg["sigma_s"], cfg["sigma_r"]
    f = synth.workload_input("bf_rgb_2048")
    x = torch.from_numpy(f).cuda()
    torch.cuda.synchronize()

    def step():
        return fhd.filter(x, sigma_s=ss, sigma_r=sr, K=K, radius=S)

    for _ in range(args.warmup):
        step()
    torch.cuda.synchronize()
    fhd.timing_enable(0, True)
    fhd.timing_read(0)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for _ in range(args.steps):
        out = step()
    torch.cuda.synchronize()
    dt = time.perf_counter() - t0
    stages = fhd.timing_read(0)
    fhd.timing_enable(0, False)
    ms_step = dt * 1000.0 / args.steps
    N = H * W
    value = N * args.steps / dt / 1e6

    # dominant kernel: the longer of the two convolution passes
    avg = {s: (ms / cnt if cnt else 0.0) for s, (ms, cnt) in stages.items()}
    dom = "col" if avg["col"] >= avg["row"] else "row"
    models = row_col_models(n, n, K, S)
    bpx, fpx = models[dom]
    sec = avg[dom] * 1e-3
    gbs = bpx * N / sec / 1e9
    tfs = fpx * N / sec / 1e12
    # the row pass is VALU-bound (its counters show VALU busy, HBM at a fraction
    # of peak); the column pass is reported against HBM
    if dom == "row":
        roofline = {"bound": "alu", "achieved": round(tfs, 2), "peak": FP32_VECTOR_PEAK,
                    "unit": "TFLOP/s", "frac": round(tfs / FP32_VECTOR_PEAK, 4)}
    else:
        roofline = {"bound": "hbm", "achieved": round(gbs, 1), "peak": HBM_PEAK_GBS,
                    "unit": "GB/s", "frac": round(gbs / HBM_PEAK_GBS, 4)}
    roofline.update({"traffic": MEASURED_TRAFFIC.get(dom), "kernel": f"{dom} pass",
                     "flops_per_launch": fpx * N, "bytes_per_launch": bpx * N,
                     "hbm_gbs": round(gbs, 1), "hbm_frac": round(gbs / HBM_PEAK_GBS, 4),
                     "avg_ms": round(avg[dom], 4), "launches": stages[dom][1]})
    breakdown = {s: round(avg[s], 4) for s in avg if stages[s][1]}

    res = {
        "metric": METRIC,
        "value": round(value, 2),
        "unit": "Mpix/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": round(ms_step, 4),
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f32",
        "data": "synthetic",
        "config": {"workload": "bf_rgb_2048: 2048x2048 RGB bilateral, guide = image, "
                               "sigma_s 5 (S 15), sigma_r 0.12, K 32, forward, FP32 form",
                   "H": H, "W": W, "n": n, "rho": n, "K": K, "S": S,
                   "sigma_s": ss, "sigma_r": sr},
        "stage_ms": breakdown,
        "roofline": roofline,
    }

    if not args.quick:
        # quality: eq. (21) against the GPU brute force of eqs. (1)-(2)
        brute = fhd.bruteforce(x, sigma_s=ss, sigma_r=sr, radius=S)
        ms_brute = timed(torch, lambda: fhd.bruteforce(x, sigma_s=ss, sigma_r=sr, radius=S), 5)
        o, d = fhd.filter(x, sigma_s=ss, sigma_r=sr, K=K, radius=S, return_den=True)
        res["quality"] = dict(error_stats(o, d, brute),
                              brute_force_mpix_s=round(N / ms_brute / 1e3, 1),
                              brute_force_ms=round(ms_brute, 3))

        # forward + hand-written adjoint (image and guide gradients, sigma_r)
        G = torch.from_numpy(np.random.default_rng(7).standard_normal(f.shape).astype(np.float32)).cuda()

        def fb():
            o, d, c = fhd.filter(x, sigma_s=ss, sigma_r=sr, K=K, radius=S, return_den=True,
                                 return_centers=True)
            fhd.filter_backward(x, x, c, o, d, G, sigma_s=ss, sigma_r=sr, radius=S)

        fb()
        ms_fb = timed(torch, fb, max(3, args.steps // 4))
        res["fwd_bwd"] = {"mpix_s": round(N / ms_fb / 1e3, 2), "ms_per_step": round(ms_fb, 3),
                          "note": "one forward call plus one adjoint call (dL/df, dL/dguide, "
                                  "dL/dsigma_r), same workload"}

        # BF16 vs FP32 contraction on the 512x512x32 hyperspectral workload
        c2 = synth.WORKLOADS["bf_hyper_512x32"]
        h = torch.from_numpy(synth.workload_input("bf_hyper_512x32")).cuda()
        ref2 = fhd.bruteforce(h, sigma_s=c2["sigma_s"], sigma_r=c2["sigma_r"], radius=c2["S"])
        ms_b2 = timed(torch, lambda: fhd.bruteforce(h, sigma_s=c2["sigma_s"], sigma_r=c2["sigma_r"],
                                                    radius=c2["S"]), 3)
        N2 = c2["H"] * c2["W"]
        forms = {"workload": "hyper_512: 512x512x32 bands, guide = image, sigma_s 4 (S 12), "
                             "sigma_r 0.2, K 64",
                 "brute_force_mpix_s": round(N2 / ms_b2 / 1e3, 1)}
        outs = {}
        for form in ("fp32", "bf16"):
            run = lambda: fhd.filter(h, sigma_s=c2["sigma_s"], sigma_r=c2["sigma_r"], K=c2["K"],
                                     radius=c2["S"], contract=form)
            outs[form] = run()
            ms2 = timed(torch, run, 5)
            forms[form] = {"mpix_s": round(N2 / ms2 / 1e3, 2),
                           "psnr_vs_brute_db": round(psnr(outs[form], ref2), 2)}
        forms["bf16_vs_fp32_max_abs"] = float((outs["bf16"] - outs["fp32"]).abs().max())
        res["forms"] = forms
        res["nlm"] = nlm_leg(torch, fhd, synth)
        res["batch"] = batch_leg(torch, np, fhd, synth)
        res["window"] = window_leg(torch, fhd, x, sr, K)
        res["approx_error"] = approx_error_leg(torch, fhd, synth)
        res["volume"] = volume_leg(torch, fhd, synth)

    if not args.no_cpu and not args.quick:
        res["cpu_baseline"] = cpu_baseline(f, cfg, args.cpu_crop)
    print(json.dumps(res))


if __name__ == "__main__":
    main()
