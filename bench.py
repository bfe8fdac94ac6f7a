"""Benchmark of the even-odd Wilson Dslash and BiCGStab on one MI355X.

Workload (default): 32^3 x 64 lattice, Wilson operator, links
U = exp(0.3 i H) (H random traceless Hermitian), kappa = 0.1350, Gaussian
source, antiperiodic in time; even-odd preconditioned BiCGStab to a true FP64
residual of 1e-10.

One timed step = one whole solve through the hot path: source preparation,
FP32 inner BiCGStab (Dslash, fused BLAS-1 and reductions, device scalars,
hipGraph replay) inside the FP64 defect-correction loop, FP64 residuals,
reconstruction and the final FP64 true residual. Fields are resident on the
GPU before the timed region starts.

value = Dslash GFlop/s of the whole job: hopping-term flops executed in the
timed steps (1320 flop per output site per hop application) divided by the
timed wall clock. The JSON line also carries the Dslash kernel's roofline
(HIP events on the library's stream), the FP64-vs-mixed solve comparison and
the CPU oracle baseline.

Usage: python bench.py [--gpus 1] [--steps K] [--warmup W]
"""

from __future__ import annotations

import argparse
import concurrent.futures as cf
import json
import os
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

import fieldgen as fg  # noqa: E402

HBM_PEAK_GBS = 8000.0
DIMS = (32, 32, 32, 64)
KAPPA = 0.1350
EPS = 0.3
SEED = 1002
HOP_FLOPS = 1320
# algorithmic bytes per output site of one hop: 8 links x 12 reals + 24 in + 24 out
HOP_BYTES = {0: (8 * 12 + 48) * 8, 1: (8 * 12 + 48) * 4, 2: 8 * 12 * 2 + 48 * 2 + 2 * 4}


def log(msg):
    print(f"[bench] {msg}", file=sys.stderr, flush=True)


def _slice(args):
    kind, dims, seed, t = args
    if kind == "gauge":
        return fg.gauge_field(dims, seed, "smooth", EPS, t_slices=[t])
    return fg.gaussian_spinor(dims, seed, t_slices=[t])


def generate(dims, seed, workers=8):
    lt = dims[3]
    with cf.ProcessPoolExecutor(max_workers=workers) as ex:
        U = np.concatenate(list(ex.map(_slice, [("gauge", dims, seed, t) for t in range(lt)])))
        b = np.concatenate(list(ex.map(_slice, [("src", dims, seed, t) for t in range(lt)])))
    return U, b


def time_hop(torch, lat, prec, reps=40, nbuf=3):
    """Average duration (ms) of the Dslash kernel (HOP_EO) with HIP events on
    the library's stream; inputs and outputs rotate over nbuf pairs of fields so
    that successive launches do not hit in the 256 MB Infinity Cache."""
    nbytes = lat.field_bytes(prec)
    ins = [torch.empty(nbytes, dtype=torch.uint8, device="cuda") for _ in range(nbuf)]
    outs = [torch.empty(nbytes, dtype=torch.uint8, device="cuda") for _ in range(nbuf)]
    src = torch.from_numpy(fg.gaussian_spinor(lat.dims, 5)).cuda()
    for t in ins:
        lat.import_field(prec, 1, src, t)
    lat.apply_native_repeat("HOP_EO", prec, ins, outs, 3)
    torch.cuda.synchronize()
    e0 = torch.cuda.Event(enable_timing=True)
    e1 = torch.cuda.Event(enable_timing=True)
    e0.record(lat.stream)
    lat.apply_native_repeat("HOP_EO", prec, ins, outs, reps)
    e1.record(lat.stream)
    e1.synchronize()
    return e0.elapsed_time(e1) / reps


def copy_probe(torch, mib=1024):
    """A plain device copy of known size (calibrates the traffic counters)."""
    a = torch.empty(mib << 20, dtype=torch.uint8, device="cuda")
    b = torch.empty_like(a)
    b.copy_(a)
    torch.cuda.synchronize()
    e0 = torch.cuda.Event(enable_timing=True)
    e1 = torch.cuda.Event(enable_timing=True)
    e0.record()
    b.copy_(a)
    e1.record()
    e1.synchronize()
    ms = e0.elapsed_time(e1)
    return 2 * (mib << 20) / (ms * 1e-3) / 1e9


TRAFFIC_FILE = os.path.join(ROOT, "profiles", "hop_traffic_32x32x32x64.txt")


def kernel_sources_hash():
    import hashlib
    h = hashlib.sha256()
    for f in ("hop.hip", "fieldio.h"):
        with open(os.path.join(ROOT, "paper_2303_05883_amd", "csrc", f), "rb") as fh:
            h.update(fh.read())
    return h.hexdigest()[:16]


def measured_traffic(prec_name):
    """HBM bytes per launch of the Dslash kernel from the committed rocprofv3
    counter summary (2 x FETCH_SIZE + WRITE_SIZE, calibrated on a plain copy),
    or None when the kernel sources changed since the counters were taken."""
    try:
        lines = open(TRAFFIC_FILE).read().splitlines()
    except OSError:
        return None
    want = None
    for ln in lines:
        if ln.startswith("sources_sha256_16:"):
            want = ln.split(":", 1)[1].strip()
    if want != kernel_sources_hash():
        return None
    for ln in lines:
        if ln.startswith(prec_name + ":"):
            parts = ln.split()
            return int(parts[parts.index("traffic_bytes") + 1])
    return None


def hop_applications(st, inner_prec):
    """Hop launches of one solve: 4 per BiCGStab iteration (two Schur applies of
    two hops), 2 per FP64 residual (one per outer pass plus the initial one), 1
    for the source, 1 for the reconstruction and 2 for the final full-D residual."""
    return 4 * st.inner_iters + 2 * (st.outer_iters + 1) + 1 + 1 + 2


def cpu_baseline(U, b, budget_s=30.0):
    """The CPU oracle's hopping term on the same 32^3 x 64 field (one full-lattice
    application = 1320 flop x V), timed on the host."""
    from oracle import dirac
    os.environ.setdefault("OMP_NUM_THREADS", "1")
    reps = 2
    t0 = time.perf_counter()
    for _ in range(reps):
        dirac.hop(U, b, -1)
    dt = (time.perf_counter() - t0) / reps
    v = int(np.prod(DIMS))
    return {"value": round(HOP_FLOPS * v / dt / 1e9, 4), "unit": "GFlop/s", "cores": 1, "kind": "oracle",
            "sample": f"{reps} oracle hopping-term applications H psi on the full 32^3x64 lattice "
                      f"(1320 flop/site x {v} sites each, NumPy float64, one thread), {dt:.1f} s each"}


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=10)
    ap.add_argument("--warmup", type=int, default=2)
    ap.add_argument("--inner", choices=["f32", "f16"], default="f32")
    ap.add_argument("--no-cpu", action="store_true", help="skip the CPU oracle baseline")
    ap.add_argument("--no-compare", action="store_true", help="skip the FP64-vs-mixed solve comparison")
    ap.add_argument("--tune-cache", default=None,
                    help="JSON launch-shape cache: read if present (no tuning sweep), written after tuning otherwise")
    ap.add_argument("--kernels-only", action="store_true",
                    help="set-up, autotune, the Dslash kernel timings and a copy of known size; no solves "
                         "(the short program the hardware-counter profiles are taken on)")
    a = ap.parse_args()
    if a.gpus != 1 or int(os.environ.get("WORLD_SIZE", "1")) != 1:
        print("bench.py runs on one GPU only: the lattice is not sharded across GPUs in this build "
              "(see the sharding design); run with --gpus 1", file=sys.stderr)
        sys.exit(2)

    import torch
    from paper_2303_05883_amd import lqcd

    if not torch.cuda.is_available():
        print("bench.py needs a GPU", file=sys.stderr)
        sys.exit(1)
    t0 = time.perf_counter()
    U, b = generate(DIMS, SEED)
    log(f"fields generated in {time.perf_counter() - t0:.1f} s")
    vh = int(np.prod(DIMS)) // 2
    cached = bool(a.tune_cache) and os.path.exists(a.tune_cache)
    if a.tune_cache:
        os.environ["LQCD_TUNE_CACHE"] = os.path.abspath(a.tune_cache)
    lat = lqcd.Lattice(DIMS, -1)
    Ud = torch.from_numpy(U).cuda()
    bd = torch.from_numpy(b).cuda()
    lat.set_gauge(Ud)
    del Ud
    lat.set_clover(KAPPA, 0.0)
    if not cached:
        for p in (lqcd.F64, lqcd.F32, lqcd.F16):
            lat.autotune(p)
        log("autotuned" + (f" (cache {a.tune_cache})" if a.tune_cache else ""))
    else:
        log(f"launch shapes from {a.tune_cache}")
    inner = lqcd.F32 if a.inner == "f32" else lqcd.F16
    if a.kernels_only:
        for p, name in ((lqcd.F64, "f64"), (lqcd.F32, "f32"), (lqcd.F16, "f16")):
            ms = time_hop(torch, lat, p, reps=10)
            log(f"hop {name}: {1000 * ms:.2f} us, {HOP_BYTES[p] * vh / (ms * 1e-3) / 1e9:.1f} GB/s")
        log(f"copy probe: {copy_probe(torch, mib=512):.1f} GB/s (512 MiB read + 512 MiB written per launch)")
        return
    x = torch.zeros_like(bd)
    for _ in range(a.warmup):
        st = lat.solve(bd, x, inner_prec=inner)
    log(f"warmup solve: {st}")

    # ---- timed region: K whole solves
    torch.cuda.synchronize()
    t_start = time.perf_counter()
    stats = []
    for _ in range(a.steps):
        stats.append(lat.solve(bd, x, inner_prec=inner))
    torch.cuda.synchronize()
    elapsed = time.perf_counter() - t_start
    worst = max(s.true_rel_resid for s in stats)
    if not worst <= 1e-10:
        log(f"true residual {worst} above 1e-10")
        sys.exit(1)
    hops = sum(hop_applications(s, inner) for s in stats)
    value = HOP_FLOPS * vh * hops / elapsed / 1e9
    ms_step = 1000 * elapsed / a.steps
    log(f"timed {a.steps} solves: {ms_step:.1f} ms each, {stats[-1]}")

    # ---- roofline of the Dslash kernel, on the library's stream
    hop = {}
    for p, name in ((lqcd.F64, "f64"), (lqcd.F32, "f32"), (lqcd.F16, "f16")):
        ms = time_hop(torch, lat, p)
        gbs = HOP_BYTES[p] * vh / (ms * 1e-3) / 1e9
        hop[name] = {"us": round(1000 * ms, 2), "gflops": round(HOP_FLOPS * vh / (ms * 1e-3) / 1e9, 1),
                     "gbs": round(gbs, 1), "frac_hbm": round(gbs / HBM_PEAK_GBS, 4)}
    log(f"hop kernel: {hop}")
    dom = "f32" if inner == lqcd.F32 else "f16"
    copy_gbs = copy_probe(torch)
    roofline = {"bound": "hbm", "achieved": hop[dom]["gbs"], "peak": HBM_PEAK_GBS, "unit": "GB/s",
                "frac": hop[dom]["frac_hbm"], "traffic": measured_traffic(dom),
                "kernel": f"k_hop<{1 if dom == 'f32' else 2},EPI_SCALE> (Dslash, {dom} storage)",
                "bytes_per_launch": HOP_BYTES[1 if dom == "f32" else 2] * vh,
                "copy_gbs": round(copy_gbs, 1)}

    # ---- FP64 vs mixed time to solution
    compare = None
    if not a.no_compare:
        compare = {}
        for name, prec in (("f64", lqcd.F64), ("mixed_f32", lqcd.F32), ("mixed_f16", lqcd.F16)):
            xs = torch.zeros_like(bd)
            lat.solve(bd, xs, inner_prec=prec)
            torch.cuda.synchronize()
            t1 = time.perf_counter()
            s = lat.solve(bd, xs, inner_prec=prec)
            torch.cuda.synchronize()
            compare[name] = {"ms": round(1000 * (time.perf_counter() - t1), 2), "outer": s.outer_iters,
                             "inner": s.inner_iters, "true_rel_resid": s.true_rel_resid}
        for name in ("mixed_f32", "mixed_f16"):
            compare[name]["speedup_vs_f64"] = round(compare["f64"]["ms"] / compare[name]["ms"], 3)
        log(f"solve comparison: {compare}")

    cpu = None
    if not a.no_cpu:
        cpu = cpu_baseline(U, b)
        log(f"cpu baseline: {cpu}")

    out = {
        "metric": "Dslash GFlop/s & %HBM peak; mixed vs FP64 solve time to residual 1e-10",
        "value": round(value, 2),
        "unit": "GFlop/s",
        "n_gpus": 1,
        "steps": a.steps,
        "warmup": a.warmup,
        "ms_per_step": round(ms_step, 3),
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f32+f64" if inner == lqcd.F32 else "f16+f32+f64",
        "data": "synthetic (seeded SU(3) links exp(0.3 i H), Gaussian source)",
        "config": {"workload": "32^3x64 Wilson even-odd BiCGStab, kappa=0.1350, eps=0.3, antiperiodic t, "
                               f"{a.inner} inner / f64 outer to true residual 1e-10",
                   "lattice": list(DIMS), "kappa": KAPPA, "step": "one whole solve",
                   "inner_iters_per_solve": stats[-1].inner_iters, "outer_iters_per_solve": stats[-1].outer_iters,
                   "parallelism": "single GPU"},
        "roofline": roofline,
        "dslash_kernel": hop,
        "solve_compare": compare,
        "cpu_baseline": cpu,
    }
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
