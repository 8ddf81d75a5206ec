"""Benchmark: FFST forward + adjoint, 512 x 512 images, J = 3 (29 spectra), float32.

One step = forward transform and adjoint transform of one batch of B
synthetic cartoon images (default B = 16) in one call per direction (the
batched form). The plain form (one image per call) is timed on the same
images and reported alongside.

Prints ONE JSON line:
  value        Gcoef/s of the batched form = B * eta * M * N * steps / time
  roofline     the dominant kernel's algorithmic bytes per launch over its
               average duration (HIP events on the launch stream, timed
               region), against MI355X HBM peak 8 TB/s; `traffic` comes from
               the committed rocprofv3 counter summary when it was taken on
               the current kernel sources, else null
  path_roofline  the whole step's algorithmic bytes over the step time
  cpu_baseline the FP64 CPU oracle on a bounded sample (1 thread)
  cpu_library  context only: the same transform on the same sample with
               scipy.fft on every host core and the plan's spectra, in
               float64 and float32
  complex_shearlets  the same images with complex (one-sided) shearlets
  uneven_batch the 64-image uneven batch (256^2 .. 1024^2, seed 401) through
               one HIP graph launch per direction, with the built-in launch
               settings and after the autotuner
  large_image  one 2048 x 2048 image, J = 5 (125 spectra)
  smooth_shearlets  the headline images with smooth shearlets
  l1_denoise   one step of l1 denoising by gradient descent (forward
               transform, gradient through the adjoint kernels, update) on
               16 noisy 512 x 512 images
The batched and plain plans are autotuned (launch settings only) before any
timing unless --no-tune is given.

Usage: python bench.py [--gpus 1] [--steps K] [--warmup W] [--batch B]
"""

import argparse
import json
import os
import platform
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

from paper_1202_1773_amd.build import source_sha  # noqa: E402

HBM_PEAK_GBS = 8000.0
METRIC = "Gcoef/s fwd+adjoint @512² J=3 FP32 (%HBM roofline); batched vs plain"


def committed_traffic(kernel, M, N, J, B):
    """HBM bytes per launch of `kernel` from the profiles/traffic_*.md
    summaries, if one was measured on the current kernel sources and this
    workload."""
    import glob
    want = source_sha()
    for path in sorted(glob.glob(os.path.join(ROOT, "profiles", "traffic_*.md"))):
        for line in open(path):
            if line.startswith("TRAFFIC {"):
                try:
                    rec = json.loads(line[len("TRAFFIC "):])
                except ValueError:
                    continue
                if (rec.get("kernel") == kernel and rec.get("source_sha") == want
                        and rec.get("workload") == [M, N, J, B]):
                    return rec["bytes_per_launch"]
    return None


def cpu_model():
    try:
        for line in open("/proc/cpuinfo"):
            if line.startswith("model name"):
                return line.split(":", 1)[1].strip()
    except OSError:
        pass
    return platform.processor()


def cpu_baseline(M, N, J, images):
    """The FP64 oracle, as it stands, on a bounded sample: forward + adjoint
    of the given images on one thread."""
    import numpy as np
    from threadpoolctl import threadpool_limits
    from oracle import spectra as ospec
    from oracle import transform as otr

    with threadpool_limits(1):
        psi = ospec.spectra(M, N, J)          # plan creation, not timed (as on the GPU)
        t0 = time.perf_counter()
        for f in images:
            c = otr.forward(f.astype(np.float64), psi)
            otr.adjoint(c, psi)
        dt = time.perf_counter() - t0
    coef = len(images) * psi.shape[0] * M * N
    return {"value": coef / dt / 1e9, "unit": "Gcoef/s", "cores": 1, "kind": "oracle",
            "sample": f"{len(images)} image(s) of {M}x{N}, J={J}: forward+adjoint, FP64 NumPy, "
                      f"{dt:.1f} s on {cpu_model()} (os.cpu_count()={os.cpu_count()})"}


def library_transform(x, p, M, N, workers):
    """Forward coefficients and adjoint images of the images x [B][M][N] with
    scipy.fft and half-plane spectra p [eta][M][N/2+1]."""
    import scipy.fft as sf

    F = sf.rfft2(x, workers=workers)
    c = sf.irfft2(F[:, None] * p[None], s=(M, N), workers=workers)
    A = (sf.rfft2(c, workers=workers) * p[None]).sum(axis=1)
    return c, sf.irfft2(A, s=(M, N), workers=workers)


def cpu_library(psi, images, M, N, reps=3):
    """Context only: the same forward + adjoint with a library CPU FFT
    (scipy.fft rfft2 / irfft2 on every host core), given the half-plane
    spectra psi [eta][M][N/2+1], in float64 and in float32; best of `reps`.
    fft2 unnormalised and 1/(MN) in ifft2, as in the transform's definition."""
    import numpy as np

    workers = os.cpu_count() or 1
    eta = psi.shape[0]
    x64 = np.stack(images).astype(np.float64)
    out = {"unit": "Gcoef/s", "cores": workers, "kind": "library (scipy.fft, same spectra)"}
    for name, dt in (("f64", np.float64), ("f32", np.float32)):
        x = x64.astype(dt)
        p = psi.astype(dt)
        best = None
        for _ in range(reps):
            t0 = time.perf_counter()
            _, y = library_transform(x, p, M, N, workers)
            t = time.perf_counter() - t0
            best = t if best is None else min(best, t)
        out[name] = len(images) * eta * M * N / best / 1e9
        out[name + "_reconstruction_rel_l2"] = float(np.linalg.norm(y - x64) / np.linalg.norm(x64))
    out["sample"] = (f"{len(images)} image(s) of {M}x{N}, {eta} spectra: forward+adjoint, best of {reps}, "
                     f"{workers} threads on {cpu_model()}")
    return out


def nnz_half(plan):
    """Nonzero half-plane spectrum values of a plan (read once per direction)."""
    return int((plan.spectra(full_plane=False) != 0).sum().item())


def time_steps(step, steps, warmup):
    import torch
    for _ in range(warmup):
        step()
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for _ in range(steps):
        step()
    torch.cuda.synchronize()
    return (time.perf_counter() - t0) / steps


# Algorithmic bytes per step of the coefficient row passes: every
# coefficient of the step is read (adjoint) or written (forward) once.
COEF_PASSES = {"k_c2r_rows(planes)": 4, "k_r2c_rows(planes)": 4,
               "k_c2c_rows(planes, inverse)": 8, "k_c2c_rows(planes)": 8}


def leg_roofline(step, steps, coefs_per_step, workload=None):
    """The dominant kernel of a leg's step (found with HIP events, one kernel
    per short pass) and its average launch duration over `steps` steps with
    only that kernel bracketed. For a coefficient row pass, achieved =
    algorithmic bytes per launch (coefficients of the step x bytes each /
    launches per step) over that duration; for other kernels the duration
    only; `traffic` from a committed counter summary of this workload
    (M, N, J, B), if given and measured on the current kernel sources. Graph
    replays are not timed by the library, so legs that run as graphs do not
    use this."""
    import torch
    from paper_1202_1773_amd import _lib

    per_kernel = {}
    for k in range(_lib.ffst_num_kernels()):
        _lib.ffst_profile_reset()
        _lib.ffst_profile_enable(1 << k)
        for _ in range(3):
            step()
        torch.cuda.synchronize()
        ms, n = _lib.ffst_profile_read(k)
        if n:
            per_kernel[_lib.ffst_kernel_name(k)] = (ms / 3, n / 3, k)
    _lib.ffst_profile_enable(0)
    name, (_, per_step, kid) = max(per_kernel.items(), key=lambda kv: kv[1][0])
    _lib.ffst_profile_reset()
    _lib.ffst_profile_enable(1 << kid)
    for _ in range(steps):
        step()
    torch.cuda.synchronize()
    _lib.ffst_profile_enable(0)
    ms, n = _lib.ffst_profile_read(kid)
    avg = ms / max(n, 1)
    out = {"kernel": name, "avg_launch_ms": round(avg, 5), "launches_per_step": round(per_step, 2)}
    if name in COEF_PASSES:
        alg = COEF_PASSES[name] * coefs_per_step / per_step
        out.update({"bound": "hbm", "alg_bytes_per_launch": int(alg), "achieved": round(alg / avg / 1e6, 2),
                    "peak": HBM_PEAK_GBS, "unit": "GB/s", "frac": round(alg / avg / 1e6 / HBM_PEAK_GBS, 4),
                    "traffic": committed_traffic(name, *workload) if workload else None})
    return out


def bench_uneven(steps, warmup, tune):
    """The uneven batch: 64 images drawn from 256^2 .. 1024^2 (seed 401), one
    graph launch per direction; forward + adjoint per step."""
    import torch
    from paper_1202_1773_amd import BatchPlan, Plan
    from paper_1202_1773_amd.synthetic import uneven_images, uneven_sizes

    sizes, Js = uneven_sizes()
    imgs = uneven_images(sizes)
    bp = BatchPlan(sizes, Js)
    f = bp.pack([torch.from_numpy(i) for i in imgs])
    c = bp.empty_coefficients()
    y = bp.empty_images()

    def step():
        bp.forward(f, out=c)
        bp.adjoint(c, out=y)

    coef = sum(e * m * n for e, (m, n) in zip(bp.etas, sizes))
    pix = sum(m * n for m, n in sizes)
    nnz = 0
    for key in dict.fromkeys(zip(sizes, Js)):
        (m, n), j = key
        p = Plan(m, n, j)
        nnz += nnz_half(p)
        p.close()
    b_alg = 4 * (2 * coef + 2 * pix + 2 * nnz)
    t_default = time_steps(step, steps, warmup)
    rec = max(float(torch.linalg.norm(a - b) / torch.linalg.norm(b))
              for a, b in zip(bp.images(y), [torch.from_numpy(i).to(y.device) for i in imgs]))
    out = {"images": len(sizes), "classes": bp.classes, "coefficients": coef,
           "ms_per_step": round(t_default * 1e3, 4), "value": round(coef / t_default / 1e9, 3), "unit": "Gcoef/s",
           "alg_bytes_per_step": b_alg, "path_frac": round(b_alg / t_default / 1e9 / HBM_PEAK_GBS, 4),
           "reconstruction_rel_l2_max": rec}
    if tune:
        bp.tune(f)
        t_tuned = time_steps(step, steps, warmup)
        out["tuned"] = {"ms_per_step": round(t_tuned * 1e3, 4), "value": round(coef / t_tuned / 1e9, 3),
                        "path_frac": round(b_alg / t_tuned / 1e9 / HBM_PEAK_GBS, 4),
                        "class_tuning": bp.class_tuning()}
    bp.close()
    return out


def bench_complex(x, M, N, J, steps, warmup):
    """Complex shearlets on the headline images: forward + adjoint per step."""
    import torch
    from paper_1202_1773_amd import Plan

    plan = Plan(M, N, J, complex_shearlets=True)
    B = x.shape[0]
    c = torch.empty((B, plan.eta, M, N), dtype=torch.complex64, device=x.device)
    y = torch.empty_like(x)

    def step():
        plan.forward(x, out=c)
        plan.adjoint(c, out=y)

    t = time_steps(step, steps, warmup)
    coef = B * plan.eta * M * N
    # complex coefficients: 8 bytes each, written then read
    b_alg = 2 * 8 * coef + 2 * 4 * B * M * N + 2 * 4 * int((plan.spectra(full_plane=True) != 0).sum().item())
    rec = float(torch.linalg.norm(y - x) / torch.linalg.norm(x))
    roof = leg_roofline(step, steps, coef, (M, N, J, B))
    plan.close()
    return {"ms_per_step": round(t * 1e3, 4), "value": round(coef / t / 1e9, 3), "unit": "Gcoef/s",
            "alg_bytes_per_step": b_alg, "path_frac": round(b_alg / t / 1e9 / HBM_PEAK_GBS, 4),
            "reconstruction_rel_l2": rec, "roofline": roof}


def bench_smooth(x, M, N, J, steps, warmup):
    """Smooth shearlets (Sec. 3.4) on the headline images: forward + adjoint per
    step; the same kernels with other spectra."""
    import torch
    from paper_1202_1773_amd import Plan

    plan = Plan(M, N, J, shearlet="smooth")
    B = x.shape[0]
    c = torch.empty((B, plan.eta, M, N), dtype=torch.float32, device=x.device)
    y = torch.empty_like(x)

    def step():
        plan.forward(x, out=c)
        plan.adjoint(c, out=y)

    t = time_steps(step, steps, warmup)
    coef = B * plan.eta * M * N
    b_alg = 4 * (2 * coef + 2 * B * M * N + 2 * nnz_half(plan))
    rec = float(torch.linalg.norm(y - x) / torch.linalg.norm(x))
    # the headline's kernels with other spectra: the headline's traffic
    # summary does not apply, so none is looked up
    roof = leg_roofline(step, steps, coef)
    plan.close()
    return {"ms_per_step": round(t * 1e3, 4), "value": round(coef / t / 1e9, 3), "unit": "Gcoef/s",
            "alg_bytes_per_step": b_alg, "path_frac": round(b_alg / t / 1e9 / HBM_PEAK_GBS, 4),
            "reconstruction_rel_l2": rec, "roofline": roof}


def bench_denoise(steps, warmup):
    """l1 denoising by gradient descent through the differentiable transform:
    16 images 512 x 512, J = 3, y = cartoon + N(0, 0.1^2) (seeds 301..316),
    lambda = 0.05; one step = loss (forward transform) + gradient (adjoint
    kernels through autograd) + update."""
    import numpy as np
    import torch
    from paper_1202_1773_amd import Plan
    from paper_1202_1773_amd.autograd import l1_loss
    from paper_1202_1773_amd.synthetic import cartoon

    M = N = 512
    plan = Plan(M, N, 3)
    yimg = torch.from_numpy(np.stack([cartoon(M, N, 20, 10, 0.1, seed=301 + b) for b in range(16)])).to("cuda")
    x = yimg.clone().requires_grad_(True)
    losses = []

    def step():
        loss = l1_loss(x, yimg, plan, 0.05)
        (g,) = torch.autograd.grad(loss, x)
        with torch.no_grad():
            x.sub_(0.25 * g)
        losses.append(loss.detach())

    t = time_steps(step, steps, warmup)
    coef = 16 * plan.eta * M * N
    first, last = float(losses[0]), float(losses[-1])
    plan.close()
    return {"ms_per_step": round(t * 1e3, 4), "value": round(coef / t / 1e9, 3), "unit": "Gcoef/s",
            "lambda": 0.05, "loss_first": first, "loss_last": last}


def bench_large(steps, warmup, tune):
    """One 2048 x 2048 image, J = 5 (125 spectra), forward + adjoint per step."""
    import torch
    from paper_1202_1773_amd import Plan
    from paper_1202_1773_amd.synthetic import config5_image

    M = N = 2048
    plan = Plan(M, N, 5)
    x = torch.from_numpy(config5_image()).to("cuda")
    c = torch.empty((plan.eta, M, N), dtype=torch.float32, device=x.device)
    y = torch.empty_like(x)
    if tune:
        plan.tune(x)

    def step():
        plan.forward(x, out=c)
        plan.adjoint(c, out=y)

    t = time_steps(step, steps, warmup)
    coef = plan.eta * M * N
    b_alg = 4 * (2 * coef + 2 * M * N + 2 * nnz_half(plan))
    rec = float(torch.linalg.norm(y - x) / torch.linalg.norm(x))
    out = {"ms_per_step": round(t * 1e3, 4), "value": round(coef / t / 1e9, 3), "unit": "Gcoef/s",
           "alg_bytes_per_step": b_alg, "path_frac": round(b_alg / t / 1e9 / HBM_PEAK_GBS, 4),
           "reconstruction_rel_l2": rec, "launch_tuning": plan.tuning_ex(),
           "roofline": leg_roofline(step, steps, coef, (M, N, 5, 1))}
    plan.close()
    return out


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=100)
    ap.add_argument("--warmup", type=int, default=10)
    ap.add_argument("--batch", type=int, default=16)
    ap.add_argument("--size", type=int, default=512)
    ap.add_argument("--scales", type=int, default=3)
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--cpu-images", type=int, default=6)
    ap.add_argument("--no-extras", action="store_true",
                    help="skip the uneven-batch and complex-shearlet measurements")
    ap.add_argument("--no-tune", action="store_true", help="time the built-in launch settings only")
    ap.add_argument("--legs", default="complex_shearlets,uneven_batch,large_image,smooth_shearlets,l1_denoise",
                    help="comma-separated extra legs to run after the headline (e.g. for profiling one leg)")
    ap.add_argument("--tuning", default=None, metavar="NPARTS,BLOCKS_PER_CU,COL_VALUES,ROW_BLOCK[,FWD_NPARTS]",
                    help="use these launch settings for the batched and plain plans instead of autotuning "
                         "(ffst_tuning in include/ffst.h; for profiling runs that must not sweep)")
    ap.add_argument("--copy-calibration-mb", type=int, default=0,
                    help="after timing, run one device copy of this many MiB (for counter calibration)")
    args = ap.parse_args()

    if args.gpus != 1 or int(os.environ.get("WORLD_SIZE", "1")) != 1:
        print("bench.py: the benchmark runs on one GPU only; --gpus must be 1 "
              "(sharding over several GPUs is not implemented)", file=sys.stderr)
        sys.exit(2)

    import numpy as np
    import torch
    from paper_1202_1773_amd import Plan, _lib
    from paper_1202_1773_amd.synthetic import cartoon_batch, config2_batch

    M = N = args.size
    J = args.scales
    B = args.batch
    dev = torch.device("cuda", 0)
    torch.cuda.set_device(dev)

    plan = Plan(M, N, J)            # batched form: B images per call
    plan1 = Plan(M, N, J)           # plain form: one image per call
    eta = plan.eta
    imgs = config2_batch(B) if M == 512 else cartoon_batch(M, N, range(201, 201 + B))
    x = torch.from_numpy(imgs).to(dev)
    c = torch.empty((B, eta, M, N), dtype=torch.float32, device=dev)
    y = torch.empty((B, M, N), dtype=torch.float32, device=dev)
    c1 = torch.empty((eta, M, N), dtype=torch.float32, device=dev)
    y1 = torch.empty((M, N), dtype=torch.float32, device=dev)
    tuning = None
    if args.tuning:
        vals = [int(v) for v in args.tuning.split(",")]
        for p_ in (plan, plan1):
            p_.set_tuning(*vals)
        tuning = {"batched": plan.tuning_ex(), "plain": plan1.tuning_ex(), "given": True}
    elif not args.no_tune:
        # launch settings picked by the autotuner, per plan, before any timing
        plan.tune(x)
        plan1.tune(x[0])
        tuning = {"batched": plan.tuning_ex(), "plain": plan1.tuning_ex()}
    plan.workspace(B)
    plan1.workspace(1)

    def step_batched():
        plan.forward(x, out=c)
        plan.adjoint(c, out=y)

    def step_plain():
        for b in range(B):
            plan1.forward(x[b], out=c1)
            plan1.adjoint(c1, out=y1)

    # warm-up, then one short pass per kernel (only that kernel bracketed by
    # HIP events, so host-side work never lands inside a bracket) to find
    # the dominant kernel
    for _ in range(args.warmup):
        step_batched()
    torch.cuda.synchronize()
    nk = _lib.ffst_num_kernels()
    per_kernel = {}
    for k in range(nk):
        _lib.ffst_profile_reset()
        _lib.ffst_profile_enable(1 << k)
        for _ in range(3):
            step_batched()
        torch.cuda.synchronize()
        ms, n = _lib.ffst_profile_read(k)
        if n:
            per_kernel[_lib.ffst_kernel_name(k)] = (ms / 3, n // 3, k)   # per step
    _lib.ffst_profile_enable(0)
    dom_name, (dom_step_ms, _, dom_id) = max(per_kernel.items(), key=lambda kv: kv[1][0])
    for _ in range(max(1, args.warmup // 2)):
        step_plain()
    torch.cuda.synchronize()
    rec_err = float(torch.linalg.norm(y - x) / torch.linalg.norm(x))

    # timed region: batched form, dominant kernel bracketed by HIP events
    _lib.ffst_profile_reset()
    _lib.ffst_profile_enable(1 << dom_id)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for _ in range(args.steps):
        step_batched()
    torch.cuda.synchronize()
    t_batched = time.perf_counter() - t0
    _lib.ffst_profile_enable(0)
    dom_ms, dom_n = _lib.ffst_profile_read(dom_id)
    dom_avg_ms = dom_ms / max(dom_n, 1)

    # plain form on the same images
    plain_steps = max(1, args.steps // 2)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for _ in range(plain_steps):
        step_plain()
    torch.cuda.synchronize()
    t_plain = time.perf_counter() - t0

    coef_per_step = B * eta * M * N
    value = coef_per_step * args.steps / t_batched / 1e9
    value_plain = coef_per_step * plain_steps / t_plain / 1e9
    ms_step = t_batched / args.steps * 1e3

    # algorithmic bytes (per-unit figures are documented with the kernels)
    lo, hi = plan.windows()
    psi_half = plan.spectra(full_plane=False)
    nnz_half = int((psi_half != 0).sum().item())
    coef_bytes = 4 * coef_per_step
    img_bytes = 4 * B * M * N
    b_alg = 2 * coef_bytes + 2 * img_bytes + 2 * 4 * nnz_half
    b_dense = 2 * coef_bytes + 2 * img_bytes + 2 * 4 * eta * M * (N // 2 + 1)
    b_floor = 2 * coef_bytes + 2 * img_bytes
    kernel_alg = {
        "k_c2r_rows(planes)": coef_bytes,     # coefficients written
        "k_r2c_rows(planes)": coef_bytes,     # coefficients read
        "k_r2c_rows(image)": img_bytes,       # images read
        "k_c2r_rows(image)": img_bytes,       # images written
        "k_fwd_cols": 4 * nnz_half,           # nonzero spectrum values read
        "k_adj_cols": 4 * nnz_half,
    }
    alg = kernel_alg.get(dom_name)
    achieved = (alg / (dom_avg_ms * 1e-3) / 1e9) if alg else None
    traffic = committed_traffic(dom_name, M, N, J, B)

    out = {
        "metric": METRIC,
        "value": round(value, 3),
        "unit": "Gcoef/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": round(ms_step, 4),
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f32",
        "data": "synthetic",
        "config": {"workload": f"FFST forward+adjoint, {B} cartoon images {M}x{N} per call, J={J} "
                               f"({eta} spectra), batched form; plain form = 1 image per call",
                   "M": M, "N": N, "J": J, "eta": eta, "batch": B, "parallelism": "single GPU",
                   "launch_tuning": tuning},
        "plain": {"value": round(value_plain, 3), "unit": "Gcoef/s",
                  "ms_per_step": round(t_plain / plain_steps * 1e3, 4),
                  "batched_over_plain": round(value / value_plain, 3)},
        "roofline": {"bound": "hbm", "kernel": dom_name,
                     "achieved": round(achieved, 2) if achieved else None,
                     "peak": HBM_PEAK_GBS, "unit": "GB/s",
                     "frac": round(achieved / HBM_PEAK_GBS, 4) if achieved else None,
                     "traffic": traffic,
                     "alg_bytes_per_launch": alg, "avg_launch_ms": round(dom_avg_ms, 5),
                     "launches_timed": dom_n},
        "path_roofline": {"alg_bytes_per_step": b_alg,
                          "achieved": round(b_alg / (ms_step * 1e-3) / 1e9, 2),
                          "peak": HBM_PEAK_GBS, "unit": "GB/s",
                          "frac": round(b_alg / (ms_step * 1e-3) / 1e9 / HBM_PEAK_GBS, 4),
                          "nnz_half_spectra": nnz_half,
                          # the same with the spectra read densely (eta * M * (N/2+1)
                          # values per direction), and without them (the floor)
                          "dense_half_bytes_per_step": b_dense,
                          "dense_half_frac": round(b_dense / (ms_step * 1e-3) / 1e9 / HBM_PEAK_GBS, 4),
                          "floor_bytes_per_step": b_floor,
                          "floor_frac": round(b_floor / (ms_step * 1e-3) / 1e9 / HBM_PEAK_GBS, 4)},
        "kernels_ms_per_step": {k: round(v[0], 5) for k, v in per_kernel.items()},
        "check": {"reconstruction_rel_l2": rec_err},
        "source_sha": source_sha(),
    }

    if args.copy_calibration_mb:
        n = args.copy_calibration_mb * (1 << 20) // 4
        a = torch.empty(n, dtype=torch.float32, device=dev).fill_(1.0)
        bcopy = torch.empty_like(a)
        torch.cuda.synchronize()
        bcopy.copy_(a)
        torch.cuda.synchronize()
        out["copy_calibration_bytes"] = 4 * n

    if not args.no_extras:
        extra_steps = max(3, args.steps // 5)
        legs = {"complex_shearlets": lambda: bench_complex(x, M, N, J, extra_steps, 2),
                "uneven_batch": lambda: bench_uneven(extra_steps, 2, not args.no_tune),
                "large_image": lambda: bench_large(extra_steps, 2, not args.no_tune),
                "smooth_shearlets": lambda: bench_smooth(x, M, N, J, extra_steps, 2),
                "l1_denoise": lambda: bench_denoise(extra_steps, 2)}
        for name in [n for n in args.legs.split(",") if n]:
            if name not in legs:
                raise SystemExit(f"unknown leg {name!r} (known: {', '.join(legs)})")
            out[name] = legs[name]()

    psi_half = plan.spectra(full_plane=False).cpu().numpy() if not args.no_cpu_baseline else None
    plan.close()
    plan1.close()
    del c, y, x
    torch.cuda.empty_cache()

    if not args.no_cpu_baseline:
        sample = [imgs[i] for i in range(min(args.cpu_images, B))]
        out["cpu_baseline"] = cpu_baseline(M, N, J, sample)
        out["cpu_library"] = cpu_library(psi_half, sample, M, N)
    else:
        out["cpu_baseline"] = None
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
