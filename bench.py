"""Benchmark of the even-odd Wilson/clover Dslash and BiCGStab on one MI355X.

Default workload (the configuration the metric is quoted on): 32^3 x 64
lattice, Wilson operator, links U = exp(0.3 i H) (H random traceless
Hermitian), kappa = 0.1350, Gaussian source, antiperiodic in time, even-odd
preconditioned BiCGStab to a true FP64 residual of 1e-10.

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

Other workloads (not the headline line; same JSON shape):
  --workload clover  32^3x64 clover, c_SW = 1.0, kappa = 0.1370, eps = 0.3
  --workload batch   12 point sources on each of 32^3x64, 24^3x48, 16^3x32
                     clover lattices (own fields), one batched solve per step,
                     against 36 sequential single-RHS FP64 solves
  --workload large   64^3x128 clover, eps = 0.25, kappa = 0.1372
  --workload sap     the clover workload solved on the full lattice by FP64
                     flexible BiCGStab with the FP32 SAP preconditioner
  --workload staggered  32^3x64 staggered operator, mass 0.05, FP64 CG on the
                     even-odd normal system (timed steps), then the same with
                     FP32 inner CG under FP64 defect correction
  --workload mg      the clover workload with the two-level multigrid
                     preconditioner
  --workload dwf     64x32x16x8 x Ls 8 Moebius domain wall: FP64 CG on the
                     normal equations (timed steps), then the even-odd form
                     with FP64 CG and with FP32 inner CG under FP64 defect
                     correction

Usage: python bench.py [--gpus 1] [--steps K] [--warmup W] [--workload NAME]
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
HOP_FLOPS = 1320
# algorithmic bytes per output site of one hop: 8 links x 12 reals + 24 in + 24 out
HOP_BYTES = {0: (8 * 12 + 48) * 8, 1: (8 * 12 + 48) * 4, 2: 8 * 12 * 2 + 48 * 2 + 2 * 4}
DIMS = (32, 32, 32, 64)
KAPPA = 0.1350
SEED = 1002

WORKLOADS = {
    "wilson": dict(dims=(32, 32, 32, 64), eps=0.3, kappa=0.1350, csw=0.0, seed=1002,
                   text="32^3x64 Wilson even-odd BiCGStab, kappa=0.1350, eps=0.3, antiperiodic t"),
    "clover": dict(dims=(32, 32, 32, 64), eps=0.3, kappa=0.1370, csw=1.0, seed=1003,
                   text="32^3x64 clover (c_SW=1.0) even-odd BiCGStab, kappa=0.1370, eps=0.3, antiperiodic t"),
    # H scale sqrt(2): at scale 1 this kappa is past the critical one of the
    # eps = 0.25 ensemble on lattices from 16^4 up (BiCGStab stalls)
    "large": dict(dims=(64, 64, 64, 128), eps=0.25, kappa=0.1372, csw=1.0, seed=1005, scale=2 ** 0.5,
                  text="64^3x128 clover (c_SW=1.0) even-odd BiCGStab, kappa=0.1372, eps=0.25 with H scale sqrt(2), "
                       "antiperiodic t"),
}
BATCH = [((32, 32, 32, 64), 1004), ((24, 24, 24, 48), 1005), ((16, 16, 16, 32), 1006)]


def log(msg):
    print(f"[bench] {msg}", file=sys.stderr, flush=True)


def _slice(args):
    kind, dims, seed, eps, scale, t = args
    if kind == "gauge":
        return fg.gauge_field(dims, seed, "smooth", eps, scale, t_slices=[t])
    return fg.gaussian_spinor(dims, seed, t_slices=[t])


def generate(dims, seed, eps=0.3, workers=None, source=True, scale=1.0):
    lt = dims[3]
    if workers is None:
        workers = max(1, min(16, len(os.sched_getaffinity(0))))
    with cf.ProcessPoolExecutor(max_workers=workers) as ex:
        U = np.concatenate(list(ex.map(_slice, [("gauge", dims, seed, eps, scale, t) for t in range(lt)])))
        b = (np.concatenate(list(ex.map(_slice, [("src", dims, seed, eps, scale, t) for t in range(lt)])))
             if source else None)
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
    del src
    lat.apply_native_repeat("HOP_EO", prec, ins, outs, 3)
    torch.cuda.synchronize()
    e0 = torch.cuda.Event(enable_timing=True)
    e1 = torch.cuda.Event(enable_timing=True)
    e0.record(lat.stream)
    lat.apply_native_repeat("HOP_EO", prec, ins, outs, reps)
    e1.record(lat.stream)
    e1.synchronize()
    return e0.elapsed_time(e1) / reps


def time_hop_rotated(torch, lqcd, lat, U, kappa, csw, prec, reps=30, nctx=3):
    """Average Dslash duration (ms) with the links rotated as well as the
    spinors: nctx contexts holding copies of the same gauge field, in the tuned
    launch shape of lat, are launched in turn on one stream, each with its own
    input and output, so that neither the links nor the spinors of a launch
    were touched by the launch before it (the 256 MB Infinity Cache then
    cannot serve them)."""
    stream = torch.cuda.Stream()
    Ud = torch.from_numpy(U).cuda()
    lats = []
    try:
        for _ in range(nctx):
            c = lqcd.Lattice(lat.dims, -1, stream=stream)
            lats.append(c)
            c.set_gauge(Ud)
            c.set_clover(kappa, csw)
            c.set_hop_shape(prec, *lat.get_hop_shape(prec))
        del Ud
        nbytes = lat.field_bytes(prec)
        src = torch.from_numpy(fg.gaussian_spinor(lat.dims, 5)).cuda()
        ins = [torch.empty(nbytes, dtype=torch.uint8, device="cuda") for _ in range(nctx)]
        outs = [torch.empty(nbytes, dtype=torch.uint8, device="cuda") for _ in range(nctx)]
        for c, t in zip(lats, ins):
            c.import_field(prec, 1, src, t)
        del src
        for k in range(nctx):
            lats[k].apply_native("HOP_EO", prec, ins[k], outs[k])
        torch.cuda.synchronize()
        e0 = torch.cuda.Event(enable_timing=True)
        e1 = torch.cuda.Event(enable_timing=True)
        e0.record(stream)
        for r in range(reps):
            k = r % nctx
            lats[k].apply_native("HOP_EO", prec, ins[k], outs[k])
        e1.record(stream)
        e1.synchronize()
        return e0.elapsed_time(e1) / reps
    finally:
        for c in lats:
            c.close()


def copy_probe(torch, mib=1024, reps=5):
    """A plain device copy of known size, best of reps (the practical HBM
    ceiling on this machine; also calibrates the traffic counters)."""
    a = torch.empty(mib << 20, dtype=torch.uint8, device="cuda")
    b = torch.empty_like(a)
    b.copy_(a)
    torch.cuda.synchronize()
    best = float("inf")
    for _ in range(reps):
        e0 = torch.cuda.Event(enable_timing=True)
        e1 = torch.cuda.Event(enable_timing=True)
        e0.record()
        b.copy_(a)
        e1.record()
        e1.synchronize()
        best = min(best, e0.elapsed_time(e1))
    return 2 * (mib << 20) / (best * 1e-3) / 1e9


TRAFFIC_FILE = os.path.join(ROOT, "profiles", "hop_traffic_32x32x32x64.txt")
KERNEL_SOURCES = ("hop.hip", "hopcore.h", "fieldio.h")


def kernel_sources_hash(sources=KERNEL_SOURCES):
    import hashlib
    h = hashlib.sha256()
    for f in sources:
        with open(os.path.join(ROOT, "paper_2303_05883_amd", "csrc", f), "rb") as fh:
            h.update(fh.read())
    return h.hexdigest()[:16]


def measured_traffic(prec_name, path=TRAFFIC_FILE, sources=KERNEL_SOURCES, kernel=None):
    """HBM bytes per launch of a kernel from a committed rocprofv3 counter
    summary (2 x FETCH_SIZE + WRITE_SIZE, calibrated on a plain copy), or None
    when the kernel sources changed since the counters were taken or, with
    kernel given, when the summary's kernel is another form (the autotuner
    may pick a different one on another run)."""
    try:
        lines = open(path).read().splitlines()
    except OSError:
        return None
    want = None
    for ln in lines:
        if ln.startswith("sources_sha256_16:"):
            want = ln.split(":", 1)[1].strip()
    if want != kernel_sources_hash(sources):
        return None
    for ln in lines:
        if ln.startswith(prec_name + ":"):
            if kernel is not None and f"lq::{kernel}<" not in ln and f" {kernel}<" not in ln:
                return None
            parts = ln.split()
            return int(parts[parts.index("traffic_bytes") + 1])
    return None


DWF_TRAFFIC_FILE = os.path.join(ROOT, "profiles", "dwf_traffic_64x32x16x8_ls8.txt")
DWF_SOURCES = ("dwf.hip", "hopcore.h", "fieldio.h")


def dwf_traffic():
    """HBM bytes per launch of the FP64 D^dag domain-wall kernel from the
    committed counter summary, or None when its sources changed since."""
    return measured_traffic("f64_Ddag", DWF_TRAFFIC_FILE, DWF_SOURCES)


def hop_applications(st):
    """Hop launches of one solve: 4 per BiCGStab iteration (two Schur applies of
    two hops), 2 per FP64 residual (one per outer pass plus the initial one), 1
    for the source, 1 for the reconstruction and 2 for the final full-D residual."""
    return 4 * st.inner_iters + 2 * (st.outer_iters + 1) + 1 + 1 + 2


def host_info():
    model = None
    try:
        with open("/proc/cpuinfo") as fh:
            for ln in fh:
                if ln.startswith("model name"):
                    model = ln.split(":", 1)[1].strip()
                    break
    except OSError:
        pass
    return {"nproc": os.cpu_count(), "usable_cpus": len(os.sched_getaffinity(0)), "cpu_model": model}


_HOST_HOP = None  # (U, psi, sites) shared with forked workers


def _host_hop_chunk(span):
    from oracle import sampled
    U, psi, sites = _HOST_HOP
    out = sampled.hop_at(U, sampled.full_lookup(psi), -1, sites[span[0]:span[1]])
    return float(np.vdot(out, out).real)


def _host_ready(_):
    return os.getpid()


def cpu_all_cores(U, b, dims, workers):
    """The oracle's site-list hop (oracle.sampled, pinned to the whole-field
    hop) over every site of the lattice, the sites split evenly among worker
    processes: one full-lattice application on all usable host cores."""
    import multiprocessing as mp
    global _HOST_HOP
    lx, ly, lz, lt = dims
    t, z, y, x = np.meshgrid(np.arange(lt), np.arange(lz), np.arange(ly), np.arange(lx), indexing="ij")
    sites = np.stack([x.ravel(), y.ravel(), z.ravel(), t.ravel()], axis=1)
    _HOST_HOP = (U, b, sites)
    n = len(sites)
    pieces = 4 * workers
    spans = [(k * n // pieces, (k + 1) * n // pieces) for k in range(pieces)]
    with mp.get_context("fork").Pool(workers) as pool:
        pool.map(_host_ready, range(workers))
        t0 = time.perf_counter()
        pool.map(_host_hop_chunk, spans, chunksize=1)
        dt = time.perf_counter() - t0
    _HOST_HOP = None
    return dt


def cpu_baseline(U, b, dims, kappa=None, gpu_iters=None):
    """The CPU oracle timed on the host: its hopping term on the benchmark's
    own field (one full-lattice application = 1320 flop x V) on one thread and
    on all usable cores; one application of its even-odd Wilson operator
    S = 1 - kappa^2 H_eo H_oe on that field, two of which make a BiCGStab
    iteration, extrapolated to the GPU's FP64 iteration count; and the 8^4 Haar
    Wilson system (kappa 0.12) applied and solved by its unpreconditioned
    BiCGStab."""
    from oracle import dirac, solvers
    host = host_info()
    reps = 2
    t0 = time.perf_counter()
    for _ in range(reps):
        dirac.hop(U, b, -1)
    dt = (time.perf_counter() - t0) / reps
    v = int(np.prod(dims))
    workers = max(1, min(16, host["usable_cpus"]))
    dt_all = cpu_all_cores(U, b, dims, workers)
    c2 = None
    if kappa is not None:
        xe = dirac.mask(b, 0)
        t0 = time.perf_counter()
        dirac.mask(xe - kappa * kappa * dirac.hop(U, dirac.mask(dirac.hop(U, xe, -1), 1), -1), 0)
        dt_s = time.perf_counter() - t0
        c2 = {"schur_apply_s": round(dt_s, 2), "per_iteration_s": round(2 * dt_s, 2),
              "sample": "one oracle application of S = 1 - kappa^2 H_eo H_oe on the benchmark's field "
                        "(NumPy float64, one thread); a BiCGStab iteration applies S twice"}
        if gpu_iters:
            c2["iterations"] = gpu_iters
            c2["solve_s_extrapolated"] = round(2 * dt_s * gpu_iters, 1)
    c1_dims = (8, 8, 8, 8)
    U1 = fg.gauge_field(c1_dims, 1001, "haar")
    b1 = fg.gaussian_spinor(c1_dims, 1001)
    op = dirac.Operator(U1, 0.12, 0.0)
    t0 = time.perf_counter()
    op.D(b1)
    dt_apply = time.perf_counter() - t0
    t0 = time.perf_counter()
    x1, info = solvers.bicgstab(op.D, b1, tol=1e-10)
    dt_solve = time.perf_counter() - t0
    return {"value": round(HOP_FLOPS * v / dt / 1e9, 4), "unit": "GFlop/s", "cores": 1, "kind": "oracle",
            "sample": f"{reps} oracle hopping-term applications H psi on the full {dims[0]}^3x{dims[3]} lattice "
                      f"(1320 flop/site x {v} sites each, NumPy float64, one thread), {dt:.1f} s each",
            "host": host,
            "all_cores": {"value": round(HOP_FLOPS * v / dt_all / 1e9, 4), "unit": "GFlop/s", "cores": workers,
                          "sample": f"one application of the oracle's site-list hop over all {v} sites, "
                                    f"split among {workers} worker processes, {dt_all:.2f} s"},
            "c1_8x8x8x8": {"apply_ms": round(1000 * dt_apply, 2), "solve_s": round(dt_solve, 3),
                           "iterations": info.iterations, "rel_resid": info.residual,
                           "sample": "oracle D apply and unpreconditioned FP64 BiCGStab to 1e-10, Haar links, "
                                     "kappa 0.12, one thread"},
            "c2_even_odd_iteration": c2}


def make_lattice(torch, lqcd, dims, seed, eps, kappa, csw, stream=None, source=True, scale=1.0):
    t0 = time.perf_counter()
    U, b = generate(dims, seed, eps, source=source, scale=scale)
    log(f"{dims} fields generated in {time.perf_counter() - t0:.1f} s")
    lat = lqcd.Lattice(dims, -1, stream=stream)
    Ud = torch.from_numpy(U).cuda()
    lat.set_gauge(Ud)
    del Ud
    lat.set_clover(kappa, csw)
    return lat, U, b


def tune(lat, lqcd, cached, label):
    if cached:
        log(f"launch shapes of {label} from the tune cache")
        return
    for p in (lqcd.F64, lqcd.F32, lqcd.F16):
        lat.autotune(p)
    log(f"autotuned {label}")


def roofline_of(torch, lat, lqcd, dom, vh, U=None, kappa=None, csw=None):
    hop = {}
    for p, name in ((lqcd.F64, "f64"), (lqcd.F32, "f32"), (lqcd.F16, "f16")):
        ms = time_hop(torch, lat, p)
        gbs = HOP_BYTES[p] * vh / (ms * 1e-3) / 1e9
        hop[name] = {"us": round(1000 * ms, 2), "gflops": round(HOP_FLOPS * vh / (ms * 1e-3) / 1e9, 1),
                     "gbs": round(gbs, 1), "frac_hbm": round(gbs / HBM_PEAK_GBS, 4)}
    log(f"hop kernel: {hop}")
    pd = 1 if dom == "f32" else 2
    block, split, xmap, nt = lat.get_hop_shape(pd)
    kname = {1: "k_hop", 2: "k_hop2", 4: "k_hop4", 0: "k_hopz"}[split]
    shape = ({"lanes": block, "z_planes_per_block": xmap} if split == 0 else
             {"block": block, "lanes_per_site": split, "xcd_map": xmap})
    shape["nt_links"] = nt
    roof = {"bound": "hbm", "achieved": hop[dom]["gbs"], "peak": HBM_PEAK_GBS, "unit": "GB/s",
            "frac": hop[dom]["frac_hbm"],
            "traffic": measured_traffic(dom, kernel=kname) if tuple(lat.dims) == DIMS else None,
            "kernel": f"{kname}<{pd},EPI_SCALE> (Dslash, {dom} storage)", "launch_shape": shape,
            "bytes_per_launch": HOP_BYTES[pd] * vh}
    if U is not None and tuple(lat.dims) == DIMS:
        ms = time_hop_rotated(torch, lqcd, lat, U, kappa, csw, pd)
        gbs = HOP_BYTES[pd] * vh / (ms * 1e-3) / 1e9
        roof["links_rotated"] = {"us": round(1000 * ms, 2), "achieved": round(gbs, 1),
                                 "frac": round(gbs / HBM_PEAK_GBS, 4)}
        log(f"hop {dom} with links rotated over 3 contexts: {roof['links_rotated']}")
    return roof, hop


def compare_solves(torch, lat, lqcd, bd):
    out = {}
    for name, prec in (("f64", lqcd.F64), ("mixed_f32", lqcd.F32), ("mixed_f16", lqcd.F16)):
        xs = torch.zeros_like(bd)
        lat.solve(bd, xs, inner_prec=prec)
        torch.cuda.synchronize()
        t1 = time.perf_counter()
        s = lat.solve(bd, xs, inner_prec=prec)
        torch.cuda.synchronize()
        out[name] = {"ms": round(1000 * (time.perf_counter() - t1), 2), "outer": s.outer_iters,
                     "inner": s.inner_iters, "true_rel_resid": s.true_rel_resid}
    for name in ("mixed_f32", "mixed_f16"):
        out[name]["speedup_vs_f64"] = round(out["f64"]["ms"] / out[name]["ms"], 3)
    log(f"solve comparison: {out}")
    return out


def c1_gpu(torch, lqcd):
    """C1: the 8^4 Haar Wilson system (kappa 0.12) solved by BiCGStab on the
    full operator (no preconditioning) and by the even-odd FP64 solve."""
    dims = (8, 8, 8, 8)
    U = fg.gauge_field(dims, 1001, "haar")
    b = torch.from_numpy(fg.gaussian_spinor(dims, 1001)).cuda()
    lat = lqcd.Lattice(dims, -1)
    lat.set_gauge(torch.from_numpy(U).cuda())
    lat.set_clover(0.12, 0.0)
    out = {}
    for name, eo in (("unpreconditioned_f64", False), ("even_odd_f64", True)):
        x = torch.zeros_like(b)
        lat.solve(b, x, even_odd=eo)
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        st = lat.solve(b, x, even_odd=eo)
        torch.cuda.synchronize()
        out[name] = {"ms": round(1000 * (time.perf_counter() - t0), 3), "iterations": st.inner_iters,
                     "true_rel_resid": st.true_rel_resid}
    lat.close()
    log(f"C1 8^4 solves: {out}")
    return out


def clover_compare(a, torch, lqcd):
    """C3: the 32^3x64 clover system solved in FP64 and mixed FP32 / FP16."""
    w = WORKLOADS["clover"]
    lat, U, b = make_lattice(torch, lqcd, w["dims"], w["seed"], w["eps"], w["kappa"], w["csw"])
    del U
    tune(lat, lqcd, a.cached, "clover " + str(w["dims"]))
    bd = torch.from_numpy(b).cuda()
    out = compare_solves(torch, lat, lqcd, bd)
    lat.close()
    return out


def run_single(a, torch, lqcd):
    w = WORKLOADS[a.workload]
    dims = w["dims"]
    vh = int(np.prod(dims)) // 2
    lat, U, b = make_lattice(torch, lqcd, dims, w["seed"], w["eps"], w["kappa"], w["csw"], scale=w.get("scale", 1.0))
    bd = torch.from_numpy(b).cuda()
    tune(lat, lqcd, a.cached, str(dims))
    inner = lqcd.F32 if a.inner == "f32" else lqcd.F16
    if a.kernels_only:
        for p, name in ((lqcd.F64, "f64"), (lqcd.F32, "f32"), (lqcd.F16, "f16")):
            ms = time_hop(torch, lat, p, reps=10)
            log(f"hop {name}: {1000 * ms:.2f} us, {HOP_BYTES[p] * vh / (ms * 1e-3) / 1e9:.1f} GB/s")
        log(f"copy probe: {copy_probe(torch, mib=512):.1f} GB/s (512 MiB read + 512 MiB written per launch)")
        return None
    x = torch.zeros_like(bd)
    st = None
    for _ in range(a.warmup):
        st = lat.solve(bd, x, inner_prec=inner)
    log(f"warmup solve: {st}")

    # ---- timed region: K whole solves
    torch.cuda.synchronize()
    t_start = time.perf_counter()
    stats = [lat.solve(bd, x, inner_prec=inner) for _ in range(a.steps)]
    torch.cuda.synchronize()
    elapsed = time.perf_counter() - t_start
    worst = max(s.true_rel_resid for s in stats)
    if not worst <= 1e-10:
        log(f"true residual {worst} above 1e-10")
        sys.exit(1)
    value = HOP_FLOPS * vh * sum(hop_applications(s) for s in stats) / elapsed / 1e9
    ms_step = 1000 * elapsed / a.steps
    log(f"timed {a.steps} solves: {ms_step:.1f} ms each, {stats[-1]}")

    dom = "f32" if inner == lqcd.F32 else "f16"
    roof, hop = roofline_of(torch, lat, lqcd, dom, vh, U, w["kappa"], w["csw"])
    roof["copy_gbs"] = round(copy_probe(torch), 1)
    roof["read_gbs"] = round(lat.bandwidth_probe(0), 1)
    compare = None if a.no_compare else compare_solves(torch, lat, lqcd, bd)
    cpu = None if (a.no_cpu or a.workload != "wilson") else cpu_baseline(
        U, b, dims, w["kappa"], compare["f64"]["inner"] if compare else None)
    if cpu:
        log(f"cpu baseline: {cpu}")
    if a.workload == "wilson" and not a.no_compare and not a.no_extra:
        # the other two targets of the metric, timed in the same run: C3 clover
        # mixed vs FP64, C4 batched vs sequential FP64, and C1
        del U, b, bd, x
        lat.close()
        compare = {"wilson": compare, "clover": clover_compare(a, torch, lqcd),
                   "batch": batch_compare(a, torch, lqcd), "c1": c1_gpu(torch, lqcd)}
    config = {"workload": w["text"] + f", {a.inner} inner / f64 outer to true residual 1e-10",
              "lattice": list(dims), "kappa": w["kappa"], "csw": w["csw"], "step": "one whole solve",
              "inner_iters_per_solve": stats[-1].inner_iters, "outer_iters_per_solve": stats[-1].outer_iters,
              "parallelism": "single GPU"}
    return value, ms_step, config, roof, hop, compare, cpu, inner


BHOP_TRAFFIC_FILE = os.path.join(ROOT, "profiles", "batch_hop_traffic_36rhs.txt")
BHOP_SOURCES = ("bhop.h", "bhop_f32.hip", "bhop_f16.hip", "hopcore.h", "fieldio.h")

# algorithmic bytes per site of the batched A_oo^-1 H_oe hop: links (8 x 12
# reals) and the clover block (72 reals) once per site, the input and output
# spinor once per site and right-hand side (FP16: 24 codes + the FP32 scale)
BHOP_SITE = {0: (8 * 96, 576, 192), 1: (8 * 48, 288, 96), 2: (8 * 24, 144, 52)}
BHOP_FLOPS = HOP_FLOPS + 504  # per site and right-hand side: hop + clover term


def batched_hop_roofline(lqcd, lats, nrhs, vhs, prec):
    """The batched hop's launch shape (autotuned or from the cache) and its
    roofline: algorithmic bytes per launch over the average launch time, HIP
    events on the batch's stream (inside the library, 20 launches)."""
    shape, us = lqcd.batch_autotune(lats, nrhs, prec)
    links, clov, spin = BHOP_SITE[prec]
    nbytes = sum(vh * (links + clov + n * 2 * spin) for vh, n in zip(vhs, nrhs))
    site_rhs = sum(vh * n for vh, n in zip(vhs, nrhs))
    gbs = nbytes / (us * 1e-6) / 1e9
    name = {0: "f64", 1: "f32", 2: "f16"}[prec]
    # the committed counters hold for the kernel instantiation and launch shape they were taken on
    tmpl = f"k_bhop<{prec}, 1, true, 0, {'true' if shape[4] else 'false'}, {shape[0]}>"
    shp = "shape " + ",".join(str(v) for v in shape)
    traffic = None
    if len(vhs) == 3 and measured_traffic(name, BHOP_TRAFFIC_FILE, BHOP_SOURCES) is not None:
        for ln in open(BHOP_TRAFFIC_FILE).read().splitlines():
            if ln.startswith(name + ":") and tmpl in ln and shp + " " in ln:
                traffic = measured_traffic(name, BHOP_TRAFFIC_FILE, BHOP_SOURCES)
    out = {"bound": "hbm", "achieved": round(gbs, 1), "peak": HBM_PEAK_GBS, "unit": "GB/s",
           "frac": round(gbs / HBM_PEAK_GBS, 4), "traffic": traffic,
           "kernel": f"k_bhop<{prec},EPI_SCALE_CLOV> (batched A_oo^-1 H_oe hop, {name} storage, all right-hand "
                     "sides of all lattices in one launch)",
           "launch_shape": {"rhs_per_lane": shape[0], "waves_per_workgroup": shape[1], "workgroups_per_xcd": shape[2],
                            "walk": ["linear", "slab", "slab/2", "slab/4"][shape[3]], "nt_links_clover": shape[4]},
           "us": round(us, 2), "bytes_per_launch": nbytes,
           "gflops": round(BHOP_FLOPS * site_rhs / (us * 1e-6) / 1e9, 1)}
    log(f"batched hop ({name}): {out}")
    return out


def batch_setup(a, torch, lqcd):
    """The three clover lattices of the batched workload with 12 point sources each."""
    stream = torch.cuda.Stream()
    lats, bs, xs, vhs = [], [], [], []
    for dims, seed in BATCH:
        lat, U, _ = make_lattice(torch, lqcd, dims, seed, 0.3, 0.1370, 1.0, stream=stream, source=False)
        del U
        tune(lat, lqcd, a.cached, str(dims))
        src = np.stack([fg.point_source(dims, k // 3, k % 3) for k in range(12)])
        lats.append(lat)
        bs.append(torch.from_numpy(src).cuda())
        xs.append(torch.zeros_like(bs[-1]))
        vhs.append(int(np.prod(dims)) // 2)
    return lats, bs, xs, vhs


def time_batched(torch, lqcd, lats, bs, xs, inner, steps, warmup):
    for _ in range(warmup):
        lqcd.solve_batch(lats, bs, xs, inner_prec=inner)
    torch.cuda.synchronize()
    t_start = time.perf_counter()
    stats = None
    for _ in range(steps):
        stats = lqcd.solve_batch(lats, bs, xs, inner_prec=inner)
    torch.cuda.synchronize()
    elapsed = time.perf_counter() - t_start
    worst = max(s.true_rel_resid for s in stats)
    if not worst <= 1e-10:
        log(f"true residual {worst} above 1e-10")
        sys.exit(1)
    return elapsed, stats


def time_sequential_f64(torch, lqcd, lats, bs, xs):
    """The same 36 right-hand sides one after another, plain FP64 BiCGStab
    (one warm-up solve per lattice first)."""
    for lat, b, x in zip(lats, bs, xs):
        lat.solve(b[0], x[0], inner_prec=lqcd.F64)
    torch.cuda.synchronize()
    t1 = time.perf_counter()
    worst = 0.0
    for lat, b, x in zip(lats, bs, xs):
        for r in range(12):
            worst = max(worst, lat.solve(b[r], x[r], inner_prec=lqcd.F64).true_rel_resid)
    torch.cuda.synchronize()
    if not worst <= 1e-10:
        log(f"true residual {worst} above 1e-10")
        sys.exit(1)
    return time.perf_counter() - t1


def batch_compare(a, torch, lqcd):
    """C4: one batched solve of the 36 right-hand sides with FP32 and with FP16
    inner iterations against 36 sequential FP64 solves."""
    lats, bs, xs, vhs = batch_setup(a, torch, lqcd)
    out = {}
    for name, inner in (("batched_f32", lqcd.F32), ("batched_f16", lqcd.F16)):
        roof = batched_hop_roofline(lqcd, lats, [12] * len(lats), vhs, inner)
        el, stats = time_batched(torch, lqcd, lats, bs, xs, inner, 1, 1)
        out[name] = {"ms": round(1000 * el, 1), "propagators_per_s": round(3 / el, 3),
                     "inner_iters_max": max(s.inner_iters for s in stats),
                     "true_rel_resid_max": max(s.true_rel_resid for s in stats), "batched_hop": roof}
    seq = time_sequential_f64(torch, lqcd, lats, bs, xs)
    out["sequential_f64"] = {"ms": round(1000 * seq, 1), "propagators_per_s": round(3 / seq, 3)}
    for name in ("batched_f32", "batched_f16"):
        out[name]["speedup_vs_sequential_f64"] = round(seq * 1000 / out[name]["ms"], 3)
    for lat in lats:
        lat.close()
    log(f"batch vs sequential FP64: {out}")
    return out


def run_batch(a, torch, lqcd):
    lats, bs, xs, vhs = batch_setup(a, torch, lqcd)
    inner = lqcd.F32 if a.inner == "f32" else lqcd.F16
    broof = batched_hop_roofline(lqcd, lats, [12] * len(lats), vhs, inner)
    elapsed, stats = time_batched(torch, lqcd, lats, bs, xs, inner, a.steps, a.warmup)
    seg_vh = [vh for vh in vhs for _ in range(12)]
    flops = sum(HOP_FLOPS * vh * hop_applications(s) for vh, s in zip(seg_vh, stats)) * a.steps
    value = flops / elapsed / 1e9
    ms_step = 1000 * elapsed / a.steps
    props = 3 * a.steps / elapsed
    log(f"timed {a.steps} batched solves of 36 RHS: {ms_step:.1f} ms each, {props:.2f} propagators/s")
    compare = None
    if not a.no_compare:
        seq = time_sequential_f64(torch, lqcd, lats, bs, xs)
        compare = {"batched_ms": round(ms_step, 2), "sequential_f64_ms": round(1000 * seq, 2),
                   "propagators_per_s_batched": round(props, 3),
                   "propagators_per_s_sequential_f64": round(3 / seq, 3),
                   "speedup": round(seq / (ms_step / 1000), 3)}
        log(f"batch vs sequential FP64: {compare}")
    _, hop = roofline_of(torch, lats[0], lqcd, "f32" if inner == lqcd.F32 else "f16", vhs[0])
    roof = broof
    config = {"workload": "12 point sources on each of 32^3x64, 24^3x48, 16^3x32 clover lattices (c_SW=1.0, "
                          f"kappa=0.1370, eps=0.3), one batched solve of 36 RHS, {a.inner} inner / f64 outer to 1e-10",
              "step": "one batched solve", "propagators_per_s": round(props, 3), "parallelism": "single GPU"}
    return value, ms_step, config, roof, hop, compare, None, inner


SAP_BLOCK, SAP_NCY, SAP_NMR = (16, 4, 2, 2), 6, 6


def sap_face_flops(block):
    """Flops per site of a SAP block launch's right-hand side update: the hops
    that cross the block faces (on average sum_mu 2 / b_mu of the 8 hops, 165
    flop each) and the addition to the stored residual (24 flop)."""
    return (HOP_FLOPS / 8) * sum(2.0 / b for b in block) + 24


def sap_application_flops(vh, ncy, nmr, block):
    """One SAP preconditioner application: 2 ncy block launches, each over
    half of the 2 vh sites, with nmr block operators (1320 + 504 flop) and MR
    updates (96 flop) per site; every launch but the first also updates its
    right-hand side (sap_face_flops)."""
    return vh * ((2 * ncy - 1) * sap_face_flops(block) + 2 * ncy * nmr * (1320 + 504 + 96))


def sap_flops(vh, st, ncy, nmr, block):
    """Flops of one SAP-preconditioned solve: the FP64 full operator (two hops
    and two clover terms per application: 2 per flexible BiCGStab iteration
    and 1 per restart check) and the preconditioner applications."""
    full = 2 * (1320 + 504) * vh
    return full * (2 * st.outer_iters + st.restarts + 1) + st.inner_iters * sap_application_flops(vh, ncy, nmr, block)


def sap_kernel_roofline(torch, lat, vh):
    """Average duration of the SAP block kernel, from HIP events on the library's
    stream: preconditioner applications with ncy cycles minus those with one
    cycle (the import/export around them cancels), per block-kernel launch.
    Work per launch (half the lattice's sites): the right-hand side update
    (sap_face_flops) and nmr block-operator + MR steps (1320 + 504 + 96 flop)
    per site."""
    b = torch.from_numpy(fg.gaussian_spinor(lat.dims, 5)).cuda()
    out = torch.zeros_like(b)

    def run(ncy, reps=4):
        lat.apply_sap(b, out, SAP_BLOCK, ncy, SAP_NMR)
        e0 = torch.cuda.Event(enable_timing=True)
        e1 = torch.cuda.Event(enable_timing=True)
        torch.cuda.synchronize()
        e0.record(lat.stream)
        for _ in range(reps):
            lat.apply_sap(b, out, SAP_BLOCK, ncy, SAP_NMR)
        e1.record(lat.stream)
        e1.synchronize()
        return e0.elapsed_time(e1) / reps

    ms = (run(SAP_NCY) - run(1)) / (2 * (SAP_NCY - 1))
    flops = vh * (sap_face_flops(SAP_BLOCK) + SAP_NMR * (1320 + 504 + 96))
    tf = flops / (ms * 1e-3) / 1e12
    return {"bound": "alu", "achieved": round(tf, 3), "peak": 157.3, "unit": "TFLOP/s", "frac": round(tf / 157.3, 4),
            "traffic": None, "kernel": "k_sap_block (FP32, one workgroup per block)", "us_per_launch": round(1000 * ms, 1),
            "flops_per_launch": flops}


def run_sap(a, torch, lqcd):
    w = WORKLOADS["clover"]
    dims = w["dims"]
    vh = int(np.prod(dims)) // 2
    lat, U, b = make_lattice(torch, lqcd, dims, w["seed"], w["eps"], w["kappa"], w["csw"])
    bd = torch.from_numpy(b).cuda()
    tune(lat, lqcd, a.cached, str(dims))
    x = torch.zeros_like(bd)
    for _ in range(a.warmup):
        lat.solve_sap(bd, x, SAP_BLOCK, SAP_NCY, SAP_NMR)
    torch.cuda.synchronize()
    t_start = time.perf_counter()
    stats = [lat.solve_sap(bd, x, SAP_BLOCK, SAP_NCY, SAP_NMR) for _ in range(a.steps)]
    torch.cuda.synchronize()
    elapsed = time.perf_counter() - t_start
    worst = max(s.true_rel_resid for s in stats)
    if not worst <= 1e-10:
        log(f"true residual {worst} above 1e-10")
        sys.exit(1)
    value = sum(sap_flops(vh, s, SAP_NCY, SAP_NMR, SAP_BLOCK) for s in stats) / elapsed / 1e9
    ms_step = 1000 * elapsed / a.steps
    log(f"timed {a.steps} SAP solves: {ms_step:.1f} ms each, {stats[-1]}")
    roof = sap_kernel_roofline(torch, lat, vh)
    log(f"SAP kernel: {roof}")
    compare = None
    if not a.no_compare:
        compare = compare_solves(torch, lat, lqcd, bd)
        compare["sap_fbicgstab"] = {"ms": round(ms_step, 2), "outer": stats[-1].outer_iters,
                                    "preconditioner_applications": stats[-1].inner_iters,
                                    "true_rel_resid": stats[-1].true_rel_resid,
                                    "speedup_vs_f64": round(compare["f64"]["ms"] / ms_step, 3)}
    config = {"workload": w["text"].replace("even-odd BiCGStab", "full-lattice flexible BiCGStab (FP64)") +
              f", SAP preconditioner (FP32) blocks {'x'.join(map(str, SAP_BLOCK))}, {SAP_NCY} cycles, "
              f"{SAP_NMR} MR steps, to true residual 1e-10",
              "lattice": list(dims), "kappa": w["kappa"], "csw": w["csw"], "step": "one whole solve",
              "outer_iters_per_solve": stats[-1].outer_iters, "parallelism": "single GPU"}
    return value, ms_step, config, roof, None, compare, None, lqcd.F32


# two-level multigrid on the clover workload; the smoother uses the SAP
# workload's block shape and MR steps (the same kernel, whose roofline is
# reported)
MG = dict(agg=(4, 4, 4, 4), nvec=8, setup_iters=6, sap_block=SAP_BLOCK, ncycles=4, nmr=SAP_NMR, coarse_tol=0.05,
          coarse_max_iter=200)


def mg_fine_flops(vh, st, ncy, nmr):
    """Fine-lattice flops of one multigrid solve: the FP64 full operator (two
    hops and two clover terms per application: 2 per flexible BiCGStab
    iteration and one per restart check), and per preconditioner application
    one FP32 full operator and 2 ncy SAP block launches over half the sites.
    The coarse grid, restriction and prolongation are not counted."""
    full = 2 * (1320 + 504) * vh
    return full * (2 * st.outer_iters + st.restarts + 2) + st.inner_iters * (
        full + sap_application_flops(vh, ncy, nmr, MG["sap_block"]))


def run_mg(a, torch, lqcd):
    w = WORKLOADS["clover"]
    dims = w["dims"]
    vh = int(np.prod(dims)) // 2
    lat, U, b = make_lattice(torch, lqcd, dims, w["seed"], w["eps"], w["kappa"], w["csw"])
    bd = torch.from_numpy(b).cuda()
    tune(lat, lqcd, a.cached, str(dims))
    lx, ly, lz, lt = dims
    gen = torch.Generator(device="cuda")
    gen.manual_seed(w["seed"] + 17)
    shape = (MG["nvec"], lt, lz, ly, lx, 4, 3)
    start = torch.complex(torch.randn(shape, generator=gen, device="cuda", dtype=torch.float64),
                          torch.randn(shape, generator=gen, device="cuda", dtype=torch.float64)) / np.sqrt(2)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    lat.mg_setup(start, **MG)
    torch.cuda.synchronize()
    setup_s = time.perf_counter() - t0
    del start
    torch.cuda.empty_cache()
    log(f"multigrid setup: {setup_s:.3f} s, coarse vectors of {lat.mg_coarse_size()} entries")
    x = torch.zeros_like(bd)
    for _ in range(a.warmup):
        lat.solve_mg(bd, x)
    torch.cuda.synchronize()
    t_start = time.perf_counter()
    stats = [lat.solve_mg(bd, x) for _ in range(a.steps)]
    torch.cuda.synchronize()
    elapsed = time.perf_counter() - t_start
    worst = max(s.true_rel_resid for s in stats)
    if not worst <= 1e-10:
        log(f"true residual {worst} above 1e-10")
        sys.exit(1)
    value = sum(mg_fine_flops(vh, s, MG["ncycles"], MG["nmr"]) for s in stats) / elapsed / 1e9
    ms_step = 1000 * elapsed / a.steps
    log(f"timed {a.steps} multigrid solves: {ms_step:.1f} ms each, {stats[-1]}")
    roof = sap_kernel_roofline(torch, lat, vh)
    log(f"SAP kernel: {roof}")
    compare = None
    if not a.no_compare:
        compare = compare_solves(torch, lat, lqcd, bd)
        compare["mg_fbicgstab"] = {"ms": round(ms_step, 2), "outer": stats[-1].outer_iters,
                                   "preconditioner_applications": stats[-1].inner_iters,
                                   "setup_s": round(setup_s, 3), "true_rel_resid": stats[-1].true_rel_resid,
                                   "speedup_vs_f64": round(compare["f64"]["ms"] / ms_step, 3)}
    config = {"workload": w["text"].replace("even-odd BiCGStab", "full-lattice flexible BiCGStab (FP64)") +
              f", two-level multigrid preconditioner (FP32): aggregates {'x'.join(map(str, MG['agg']))}, "
              f"{MG['nvec']} test vectors, {MG['setup_iters']} setup rounds, SAP smoother blocks "
              f"{'x'.join(map(str, MG['sap_block']))} ({MG['ncycles']} cycles, {MG['nmr']} MR steps), coarse "
              f"BiCGStab to {MG['coarse_tol']}, to true residual 1e-10; setup timed apart",
              "lattice": list(dims), "kappa": w["kappa"], "csw": w["csw"], "step": "one whole solve (setup excluded)",
              "setup_s": round(setup_s, 3), "outer_iters_per_solve": stats[-1].outer_iters,
              "value_counts": "fine-lattice operator and SAP flops only", "parallelism": "single GPU"}
    return value, ms_step, config, roof, None, compare, None, lqcd.F32


STAG_MASS = 0.05
STAG_FLOPS = 570            # per output site per staggered hop
STAG_BYTES = {0: 8 * 96 + 48 + 48, 1: 8 * 48 + 24 + 24}  # 8 links x 12 reals, vector in, vector out


def stag_hops(st):
    """Staggered hops of one solve: 2 per CG iteration, 1 for the source, and
    per pass 2 (normal-operator residual) + 3 (reconstruction, true residual)."""
    return 2 * st.inner_iters + 1 + 5 * (st.outer_iters + 1)


def time_stag_hop(torch, lat, prec, reps=40, nbuf=3):
    nbytes = lat.stag_field_bytes(prec)
    ins = [torch.empty(nbytes, dtype=torch.uint8, device="cuda") for _ in range(nbuf)]
    outs = [torch.empty(nbytes, dtype=torch.uint8, device="cuda") for _ in range(nbuf)]
    lx, ly, lz, lt = lat.dims
    rng = np.random.default_rng(5)
    src = torch.from_numpy(rng.normal(size=(lt, lz, ly, lx, 3)) + 1j * rng.normal(size=(lt, lz, ly, lx, 3))).cuda()
    for t in ins:
        lat.stag_import(prec, 1, src, t)
    del src
    lat.stag_hop_native_repeat(prec, 0, ins, outs, 3)
    torch.cuda.synchronize()
    e0 = torch.cuda.Event(enable_timing=True)
    e1 = torch.cuda.Event(enable_timing=True)
    e0.record(lat.stream)
    lat.stag_hop_native_repeat(prec, 0, ins, outs, reps)
    e1.record(lat.stream)
    e1.synchronize()
    return e0.elapsed_time(e1) / reps


def run_staggered(a, torch, lqcd):
    w = WORKLOADS["wilson"]
    dims = w["dims"]
    vh = int(np.prod(dims)) // 2
    U, _ = generate(dims, w["seed"], w["eps"], source=False)
    lat = lqcd.Lattice(dims, -1)
    lat.set_gauge(torch.from_numpy(U).cuda())
    del U
    lat.set_clover(w["kappa"], 0.0)
    lx, ly, lz, lt = dims
    rng = np.random.default_rng(w["seed"])
    b = torch.from_numpy((rng.normal(size=(lt, lz, ly, lx, 3)) + 1j * rng.normal(size=(lt, lz, ly, lx, 3))) /
                         np.sqrt(2)).cuda()
    x = torch.zeros_like(b)
    for _ in range(a.warmup):
        lat.stag_solve(STAG_MASS, b, x)
    torch.cuda.synchronize()
    t_start = time.perf_counter()
    stats = [lat.stag_solve(STAG_MASS, b, x) for _ in range(a.steps)]
    torch.cuda.synchronize()
    elapsed = time.perf_counter() - t_start
    worst = max(s.true_rel_resid for s in stats)
    if not worst <= 1e-10:
        log(f"true residual {worst} above 1e-10")
        sys.exit(1)
    value = STAG_FLOPS * vh * sum(stag_hops(s) for s in stats) / elapsed / 1e9
    ms_step = 1000 * elapsed / a.steps
    log(f"timed {a.steps} staggered CG solves: {ms_step:.1f} ms each, {stats[-1]}")
    # the same with FP32 inner CG under FP64 defect correction (inner tolerance 1e-6)
    xm = torch.zeros_like(b)
    lat.stag_solve(STAG_MASS, b, xm, inner_prec=lqcd.F32)
    torch.cuda.synchronize()
    t1 = time.perf_counter()
    st_mx = lat.stag_solve(STAG_MASS, b, xm, inner_prec=lqcd.F32)
    torch.cuda.synchronize()
    ms_mx = 1000 * (time.perf_counter() - t1)
    if not st_mx.true_rel_resid <= 1e-10:
        log(f"mixed true residual {st_mx.true_rel_resid} above 1e-10")
        sys.exit(1)
    compare = {"f64_cg": {"ms": round(ms_step, 2), "cg_iters": stats[-1].inner_iters,
                          "true_rel_resid": stats[-1].true_rel_resid},
               "mixed_f32_cg": {"ms": round(ms_mx, 2), "cg_iters": st_mx.inner_iters, "passes": st_mx.outer_iters,
                                "true_rel_resid": st_mx.true_rel_resid,
                                "speedup_vs_f64": round(ms_step / ms_mx, 3)}}
    log(f"staggered solves: {compare}")
    del xm
    hop = {}
    for p, name in ((lqcd.F64, "f64"), (lqcd.F32, "f32")):
        ms = time_stag_hop(torch, lat, p)
        gbs = STAG_BYTES[p] * vh / (ms * 1e-3) / 1e9
        hop[name] = {"us": round(1000 * ms, 2), "gflops": round(STAG_FLOPS * vh / (ms * 1e-3) / 1e9, 1),
                     "gbs": round(gbs, 1), "frac_hbm": round(gbs / HBM_PEAK_GBS, 4)}
    log(f"staggered hop kernel: {hop}")
    roof = {"bound": "hbm", "achieved": hop["f64"]["gbs"], "peak": HBM_PEAK_GBS, "unit": "GB/s",
            "frac": hop["f64"]["frac_hbm"], "traffic": None,
            "kernel": "k_stag_hop<0> (staggered hop, f64 storage)", "bytes_per_launch": STAG_BYTES[0] * vh}
    config = {"workload": f"32^3x64 staggered, mass {STAG_MASS}, links of the Wilson workload (eps 0.3), "
                          "antiperiodic t, FP64 CG on the even-odd normal system to true residual 1e-10",
              "lattice": list(dims), "mass": STAG_MASS, "step": "one whole solve",
              "cg_iters_per_solve": stats[-1].inner_iters, "parallelism": "single GPU"}
    return value, ms_step, config, roof, hop, compare, None, lqcd.F64


DWF = dict(dims=(64, 32, 16, 8), Ls=8, M5=1.8, mf=0.05, b5=1.5, c5=0.5, eps=0.3, seed=1007)
DWF_KERNEL = "k_dwf<0,true,false> (fused Moebius domain-wall D^dag, one launch per application, f64 storage)"
# per 5-d site per D or D^dag application: the 4-d hop (1320) and the
# diagonal, s-hop and Moebius combination terms (192)
DWF_FLOPS = 1320 + 192
# algorithmic bytes per 5-d output site of the D^dag kernel: the hop input,
# the own spinor, the output, and the 8 links shared by the Ls slices
DWF_BYTES = {0: lambda ls: 3 * 192 + 8 * 96 / ls, 1: lambda ls: 3 * 96 + 8 * 48 / ls}


def dwf_applications(st):
    """D and D^dag applications of one domain-wall CG solve: D^dag b, then per
    pass the true residual D x (one more at the end) and D^dag of it, and two
    per CG iteration."""
    return 2 + 2 * st.outer_iters + 2 * st.inner_iters


def time_dwf_apply(torch, lat, d, prec, dag, reps=20, nbuf=2):
    """Average duration (ms) of one D (or D^dag) application on native 5-d
    fields, with HIP events on the library's stream."""
    Ls = d["Ls"]
    nbytes = lat.dwf_field_bytes(prec, Ls)
    ins = [torch.empty(nbytes, dtype=torch.uint8, device="cuda") for _ in range(nbuf)]
    outs = [torch.empty(nbytes, dtype=torch.uint8, device="cuda") for _ in range(nbuf)]
    tmp = torch.empty(nbytes, dtype=torch.uint8, device="cuda")
    lx, ly, lz, lt = lat.dims
    shape = (Ls, lt, lz, ly, lx, 4, 3)
    rng = np.random.default_rng(6)
    src = torch.from_numpy(rng.normal(size=shape) + 1j * rng.normal(size=shape)).cuda()
    for t in ins:
        lat.dwf_import(prec, Ls, src, t)
    del src
    args = (Ls, d["M5"], d["mf"], prec, ins, outs)
    kw = dict(dag=dag, b5=d["b5"], c5=d["c5"], tmp=tmp)
    lat.dwf_apply_native_repeat(*args, 2, **kw)
    torch.cuda.synchronize()
    e0 = torch.cuda.Event(enable_timing=True)
    e1 = torch.cuda.Event(enable_timing=True)
    e0.record(lat.stream)
    lat.dwf_apply_native_repeat(*args, reps, **kw)
    e1.record(lat.stream)
    e1.synchronize()
    return e0.elapsed_time(e1) / reps


def run_dwf(a, torch, lqcd):
    d = DWF
    dims, Ls = d["dims"], d["Ls"]
    vol5 = int(np.prod(dims)) * Ls
    U, _ = generate(dims, d["seed"], d["eps"], source=False)
    lat = lqcd.Lattice(dims, -1)
    lat.set_gauge(torch.from_numpy(U).cuda())
    del U
    lat.set_clover(0.12, 0.0)
    if a.kernels_only:
        for p, name in ((lqcd.F64, "f64"), (lqcd.F32, "f32")):
            for dag in (False, True):
                ms = time_dwf_apply(torch, lat, d, p, dag, reps=10)
                bw = f", {DWF_BYTES[p](Ls) * vol5 / (ms * 1e-3) / 1e9:.1f} GB/s" if dag else ""
                log(f"dwf {name} {'D^dag' if dag else 'D'}: {1000 * ms:.2f} us{bw}")
        log(f"copy probe: {copy_probe(torch, mib=512):.1f} GB/s (512 MiB read + 512 MiB written per launch)")
        return None
    lx, ly, lz, lt = dims
    shape = (Ls, lt, lz, ly, lx, 4, 3)
    rng = np.random.default_rng(d["seed"])
    b = torch.from_numpy((rng.normal(size=shape) + 1j * rng.normal(size=shape)) / np.sqrt(2)).cuda()
    x = torch.zeros_like(b)
    mob = dict(b5=d["b5"], c5=d["c5"])
    for _ in range(a.warmup):
        lat.dwf_solve(Ls, d["M5"], d["mf"], b, x, **mob)
    torch.cuda.synchronize()
    t_start = time.perf_counter()
    stats = [lat.dwf_solve(Ls, d["M5"], d["mf"], b, x, **mob) for _ in range(a.steps)]
    torch.cuda.synchronize()
    elapsed = time.perf_counter() - t_start
    worst = max(s.true_rel_resid for s in stats)
    if not worst <= 1e-10:
        log(f"true residual {worst} above 1e-10")
        sys.exit(1)
    value = DWF_FLOPS * vol5 * sum(dwf_applications(s) for s in stats) / elapsed / 1e9
    ms_step = 1000 * elapsed / a.steps
    log(f"timed {a.steps} domain-wall CG solves: {ms_step:.1f} ms each, {stats[-1]}")
    # the even-odd Schur complement and CG on its normal equations, same system
    xe = torch.zeros_like(b)
    lat.dwf_solve_eo(Ls, d["M5"], d["mf"], b, xe, **mob)
    torch.cuda.synchronize()
    t1 = time.perf_counter()
    st_eo = lat.dwf_solve_eo(Ls, d["M5"], d["mf"], b, xe, **mob)
    torch.cuda.synchronize()
    ms_eo = 1000 * (time.perf_counter() - t1)
    # the same with FP32 inner CG under FP64 defect correction (inner tolerance 1e-6)
    xe.zero_()
    lat.dwf_solve_eo(Ls, d["M5"], d["mf"], b, xe, inner_prec=lqcd.F32, **mob)
    torch.cuda.synchronize()
    t1 = time.perf_counter()
    st_mx = lat.dwf_solve_eo(Ls, d["M5"], d["mf"], b, xe, inner_prec=lqcd.F32, **mob)
    torch.cuda.synchronize()
    ms_mx = 1000 * (time.perf_counter() - t1)
    if not max(st_eo.true_rel_resid, st_mx.true_rel_resid) <= 1e-10:
        log(f"even-odd true residuals {st_eo.true_rel_resid}, {st_mx.true_rel_resid} above 1e-10")
        sys.exit(1)
    compare = {"full_cg": {"ms": round(ms_step, 2), "cg_iters": stats[-1].inner_iters,
                           "true_rel_resid": stats[-1].true_rel_resid},
               "even_odd_cg": {"ms": round(ms_eo, 2), "cg_iters": st_eo.inner_iters,
                               "true_rel_resid": st_eo.true_rel_resid,
                               "speedup_vs_full": round(ms_step / ms_eo, 3)},
               "even_odd_cg_mixed_f32": {"ms": round(ms_mx, 2), "cg_iters": st_mx.inner_iters,
                                         "passes": st_mx.outer_iters, "true_rel_resid": st_mx.true_rel_resid,
                                         "speedup_vs_full": round(ms_step / ms_mx, 3),
                                         "speedup_vs_even_odd_f64": round(ms_eo / ms_mx, 3)}}
    log(f"domain-wall solves: {compare}")
    del b, x, xe
    torch.cuda.empty_cache()
    ops = {}
    for p, name in ((lqcd.F64, "f64"), (lqcd.F32, "f32")):
        for dag in (False, True):
            ms = time_dwf_apply(torch, lat, d, p, dag)
            e = {"us": round(1000 * ms, 2), "gflops": round(DWF_FLOPS * vol5 / (ms * 1e-3) / 1e9, 1)}
            if dag:  # one kernel per application: its HBM roofline
                gbs = DWF_BYTES[p](Ls) * vol5 / (ms * 1e-3) / 1e9
                e.update(gbs=round(gbs, 1), frac_hbm=round(gbs / HBM_PEAK_GBS, 4))
            ops[name + ("_Ddag" if dag else "_D")] = e
    log(f"domain-wall operator: {ops}")
    roof = {"bound": "hbm", "achieved": ops["f64_Ddag"]["gbs"], "peak": HBM_PEAK_GBS, "unit": "GB/s",
            "frac": ops["f64_Ddag"]["frac_hbm"], "traffic": dwf_traffic(), "kernel": DWF_KERNEL,
            "bytes_per_launch": DWF_BYTES[0](Ls) * vol5}
    config = {"workload": f"64x32x16x8 x Ls {Ls} Moebius domain-wall, b5 {d['b5']}, c5 {d['c5']}, M5 {d['M5']}, "
                          f"m_f {d['mf']}, links exp(i eps H) with eps {d['eps']}, antiperiodic t, FP64 CG on the "
                          "normal equations to true residual 1e-10",
              "lattice": list(dims), "Ls": Ls, "M5": d["M5"], "mf": d["mf"], "b5": d["b5"], "c5": d["c5"],
              "step": "one whole solve",
              "cg_iters_per_solve": stats[-1].inner_iters, "parallelism": "single GPU"}
    return value, ms_step, config, roof, ops, compare, None, lqcd.F64


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=10)
    ap.add_argument("--warmup", type=int, default=2)
    ap.add_argument("--workload", choices=["wilson", "clover", "batch", "large", "sap", "mg", "staggered", "dwf"], default="wilson")
    ap.add_argument("--inner", choices=["f32", "f16"], default="f32")
    ap.add_argument("--no-cpu", action="store_true", help="skip the CPU oracle baseline")
    ap.add_argument("--no-compare", action="store_true", help="skip the FP64-vs-mixed solve comparison")
    ap.add_argument("--no-extra", action="store_true",
                    help="wilson workload: skip the clover (C3), batched (C4) and 8^4 (C1) comparisons")
    ap.add_argument("--tune-cache", default=None,
                    help="JSON launch-shape cache: read if present (no tuning sweep), written after tuning otherwise")
    ap.add_argument("--kernels-only", action="store_true",
                    help="set-up, autotune, the Dslash kernel timings and a copy of known size; no solves "
                         "(the short program the hardware-counter profiles are taken on)")
    a = ap.parse_args()
    if a.gpus != 1 or int(os.environ.get("WORLD_SIZE", "1")) != 1:
        print("bench.py runs on one GPU only: the library does not shard the lattice across GPUs "
              "(the halo-exchange design is described but not implemented); run with --gpus 1", file=sys.stderr)
        sys.exit(2)

    import torch
    from paper_2303_05883_amd import lqcd

    if not torch.cuda.is_available():
        print("bench.py needs a GPU", file=sys.stderr)
        sys.exit(1)
    a.cached = bool(a.tune_cache) and os.path.exists(a.tune_cache)
    if a.tune_cache:
        os.environ["LQCD_TUNE_CACHE"] = os.path.abspath(a.tune_cache)
    runner = {"batch": run_batch, "sap": run_sap, "mg": run_mg, "staggered": run_staggered, "dwf": run_dwf}.get(a.workload, run_single)
    res = runner(a, torch, lqcd)
    if res is None:
        return
    value, ms_step, config, roof, hop, compare, cpu, inner = res
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
        "dtype": {lqcd.F64: "f64", lqcd.F32: "f32+f64"}.get(inner, "f16+f32+f64"),
        "data": "synthetic (seeded SU(3) links exp(i eps H), Gaussian or point sources)",
        "config": config,
        "roofline": roof,
        "dslash_kernel": hop,
        "solve_compare": compare,
        "cpu_baseline": cpu,
    }
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
