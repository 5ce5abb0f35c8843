"""Benchmark of the Wilson-Dirac inverter hot path on one MI355X.

Headline workload (the largest single-GPU configuration): 32^3 x 64 lattice,
smooth random links U = exp(i 0.3 H) (plaquette ~0.61, seed 1003), kappa =
0.1248, one Gaussian source (seed 2003), true residual 1e-10.  A step is one
complete solve of D psi = eta by mixed-precision even-odd CGNR: FP16 storage
of links (12-real compression) and spinors (per-site FP32 norm), FP32
arithmetic, FP64 reliable updates, reductions and true residual.  Every
kernel of the solve is inside the step: source packing, each D-slash and
BLAS kernel of the iteration, the FP64 residual recomputations, the odd-site
reconstruction and the FP64 true residual.  Inputs are resident in HBM before
the timed region.

value  = algorithmic HBM bytes of every kernel of the solve / solve time (GB/s)
roofline = the dominant kernel (the FP16 single-parity hop): algorithmic bytes
           per launch / mean launch duration (HIP events recorded by each hop's
           dispatch on the solver's stream; the device steady-clock span of
           the same launches reported beside it), against the 8 TB/s HBM peak;
           traffic = the committed rocprofv3 counter reading per launch while
           the hop's sources are unchanged
cpu_baseline = the FP64 CPU oracle on a bounded sample of the same workload:
           CGNR iterations of the same 32^3 x 64 system with every host
           thread, in the same byte model; single-parity hops with every
           thread and with one thread beside it.

Usage: python bench.py [--gpus 1] [--steps K] [--warmup W] [--sloppy f16]
"""
import argparse
import hashlib
import json
import os
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

METRIC = "Dslash GB/s & % HBM peak; CG time to 1e-10 resid, mixed/batched vs FP64"
HBM_PEAK_GBS = 8000.0


PROFILE = os.path.join(ROOT, "profiles", "k_hop_cg_f16_32c64.md")
HOP_SOURCES = ("paper_2001_05706_amd/csrc/wl_core.h", "paper_2001_05706_amd/csrc/hop.hip")


def measured_traffic(sloppy, recon, L):
    """HBM bytes per launch of the FP16 recon-12 hop of the 32^3 x 64 solve from
    the committed rocprofv3 counter summary (scaled FETCH_SIZE + WRITE_SIZE), or
    None when the hop's sources have changed since the counters were taken or
    another kernel or lattice is timed."""
    if (sloppy, recon, tuple(L)) != ("f16", 12, (32, 32, 32, 64)) or not os.path.exists(PROFILE):
        return None
    rec = None
    for line in open(PROFILE):
        if line.startswith("traffic_record: "):
            rec = json.loads(line[len("traffic_record: "):])
    if rec is None:
        return None
    h = hashlib.sha256()
    for f in HOP_SOURCES:
        h.update(open(os.path.join(ROOT, f), "rb").read())
    if h.hexdigest() != rec["sources_sha256"]:
        return None
    return rec["traffic_bytes"]


def log(msg):
    print("[bench] " + msg, file=sys.stderr, flush=True)


def cg_iteration_bytes(w, prec, recon, vh):
    """Algorithmic bytes of one CGNR iteration per the library's byte model:
    4 hops (+2 epilogue reads), r update (3 passes), x += alpha p with
    p = s + beta p (5)."""
    site = {"f64": 192, "f32": 96, "f16": 52, "bf16": 52}[prec]
    return vh * (4 * w.wl_hop_bytes_per_site(prec, recon, 1) + 2 * site + 3 * site + 5 * site)


def _guard(fn):
    try:
        return fn()
    except Exception as e:  # a failed side measurement is reported, not fatal
        log("side measurement failed: %r" % (e,))
        return {"error": repr(e)}


def _timed(torch, fn, reps=3):
    fn()
    torch.cuda.synchronize()
    best, res = 1e30, None
    for _ in range(reps):
        t = time.perf_counter()
        res = fn()
        torch.cuda.synchronize()
        best = min(best, time.perf_counter() - t)
    return best, res


def _dev(torch, a, dev):
    return torch.from_numpy(np.ascontiguousarray(a).view(np.float64)).to(dev)


def bench_batch12(w, torch, li, dev, a):
    """12 spin-colour point sources on 24^3 x 48: one batched solve vs 12 single solves."""
    L = (24, 24, 24, 48)
    U = li.near_identity_links(L, 0.3, 1004)
    eta = li.point_sources(L)
    g = w.Gauge(L, _dev(torch, U, dev))
    e = _dev(torch, eta, dev).reshape(-1)
    x = torch.zeros_like(e)
    per = e.numel() // 12

    def batched():
        x.zero_()
        return w.wilson_cg(g, e, x, 12, 0.1245, 1e-10, 5000, "f32", 12, a.delta)[1]

    def single():
        infos = []
        for r in range(12):
            xr = x[r * per:(r + 1) * per]
            xr.zero_()
            infos += w.wilson_cg(g, e[r * per:(r + 1) * per], xr, 1, 0.1245, 1e-10, 5000, "f32", 12, a.delta)[1]
        return infos

    tb, ib = _timed(torch, batched)
    ts, is_ = _timed(torch, single, reps=1)
    g.close()
    r = {"batched_ms": round(tb * 1e3, 2), "sequential_ms": round(ts * 1e3, 2),
         "speedup": round(ts / tb, 3), "ms_per_rhs": round(tb * 1e3 / 12, 3),
         "max_iters": max(i["iters"] for i in ib), "worst_true_resid": max(i["true_resid"] for i in ib),
         "batched_GBs": round(ib[0]["gbytes"] / tb, 1)}
    log("batched 12 rhs: %s" % r)
    return r


def bench_uneven(w, torch, li, dev, a):
    """4 x {8^4, 12^4, 16^3x32, 24^3x48}, Gaussian sources: one batched solve vs 16 solves."""
    sizes = [(8, 8, 8, 8), (12, 12, 12, 12), (16, 16, 16, 32), (24, 24, 24, 48)]
    specs = [L for L in sizes for _ in range(4)]
    gs, es, xs = [], [], []
    for n, L in enumerate(specs):
        gs.append(w.Gauge(L, _dev(torch, li.near_identity_links(L, 0.3, 3000 + n), dev)))
        es.append(_dev(torch, li.gaussian_spinor(L, 4000 + n), dev))
        xs.append(torch.zeros_like(es[-1]))

    def batched():
        for x in xs:
            x.zero_()
        return w.wilson_cg_multi(gs, es, xs, [1] * 16, [0.1245] * 16, 1e-10, 5000, "f32", 12, a.delta)[1]

    def single():
        out = []
        for gg, e, x in zip(gs, es, xs):
            x.zero_()
            out += w.wilson_cg(gg, e, x, 1, 0.1245, 1e-10, 5000, "f32", 12, a.delta)[1]
        return out

    tb, ib = _timed(torch, batched)
    ts, is_ = _timed(torch, single, reps=1)
    for gg in gs:
        gg.close()
    r = {"batched_ms": round(tb * 1e3, 2), "sequential_ms": round(ts * 1e3, 2), "speedup": round(ts / tb, 3),
         "sites": int(sum(np.prod(L) for L in specs)), "worst_true_resid": max(i["true_resid"] for i in ib),
         "batched_GBs": round(ib[0]["gbytes"] / tb, 1)}
    log("uneven batch: %s" % r)
    return r


def bench_c2(w, torch, li, dev, a, U, eta):
    """The 24^3 x 48 workload (kappa 0.1245, seeds 1002/2002): plain FP64 and
    FP32 solves, and the mixed FP16 solve beside them, CGNR and BiCGStab."""
    L = (24, 24, 24, 48)
    g = w.Gauge(L, _dev(torch, U, dev))
    e = _dev(torch, eta, dev)
    x = torch.zeros_like(e)
    r = {}
    for meth, fn in (("cgnr", w.wilson_cg), ("bicgstab", w.wilson_bicgstab)):
        for sl, rc in [("f64", 18), ("f32", 12), ("f16", 12)]:
            def run():
                x.zero_()
                return fn(g, e, x, 1, 0.1245, 1e-10, 5000, sl, rc, a.delta)[1][0]
            try:
                t, inf = _timed(torch, run, reps=3)
                r["%s_%s" % (meth, sl)] = {"ms": round(t * 1e3, 3), "iters": inf["iters"],
                                           "updates": inf["reliable_updates"], "true_resid": inf["true_resid"],
                                           "GBs": round(inf["gbytes"] / t, 1)}
            except w.WilsonError as ex:
                r["%s_%s" % (meth, sl)] = {"error": str(ex)}
            log("24^3x48 %s %s: %s" % (meth, sl, r["%s_%s" % (meth, sl)]))
    g.close()
    return r


def bench_sign(w, torch, li, dev, a):
    """Degree-200 Chebyshev sign function of H_W (rho 1.5) on 12 RHS, 16^3 x 32, FP32."""
    L = (16, 16, 16, 32)
    vh = int(np.prod(L)) // 2
    g = w.Gauge(L, _dev(torch, li.near_identity_links(L, 0.2, 1005), dev))
    v = _dev(torch, li.gaussian_spinor(L, 2005, nrhs=12), dev)
    out = torch.zeros_like(v)
    back = torch.zeros_like(v)
    t, _ = _timed(torch, lambda: w.overlap_sign_cheb(g, v, out, 12, 1.5, 200, 0.003, 1.0, 42.25, "f32", 12), reps=2)
    w.overlap_sign_cheb(g, out, back, 12, 1.5, 200, 0.003, 1.0, 42.25, "f32", 12)
    torch.cuda.synchronize()
    res = float(torch.linalg.norm(back - v) / torch.linalg.norm(v))
    g.close()
    # per Clenshaw step and RHS: two whole-lattice H_W (4 hops) with 1 + 4 epilogue
    # reads; links shared by the 12 RHS
    site, link = 96, 48
    step = 2 * (2 * vh) * (8 * link / 12.0 + 2 * site) + 2 * vh * (1 + 4) * site
    gb = 12 * 202 * step / 1e9
    r = {"ms": round(t * 1e3, 2), "ms_per_rhs": round(t * 1e3 / 12, 3), "eps2_resid_f32": res,
         "GBs": round(gb / t, 1), "hw_applications_per_rhs": 2 * 201 + 1}
    log("sign function: %s" % r)
    return r


def bench_clover(w, torch, li, dev, a, U, eta):
    """Wilson-clover e/o CGNR (c_sw 1.0, kappa 0.12) on the 24^3 x 48 workload's
    links and source: FP64 against the mixed FP16 solve, to 1e-10."""
    L = (24, 24, 24, 48)
    g = w.Gauge(L, _dev(torch, U, dev))
    eta = _dev(torch, eta, dev)
    x = torch.zeros_like(eta)
    r = {}
    for sloppy, recon in (("f64", 18), ("f32", 12), ("f16", 12)):
        def run():
            x.zero_()
            return w.wilson_clover_cg(g, eta, x, 1, 0.12, 1.0, 1e-10, 5000, sloppy, recon, a.delta)

        t, (st, info) = _timed(torch, run, reps=2)
        i = info[0]
        r[sloppy] = {"ms": round(t * 1e3, 2), "iters": i["iters"], "true_resid": i["true_resid"],
                     "GBs": round(i["gbytes"] / t, 1)}
    r["speedup_f16_vs_f64"] = round(r["f64"]["ms"] / r["f16"]["ms"], 3)
    g.close()
    log("clover cg: %s" % r)
    return r


def bench_overlap(w, torch, li, dev, a):
    """Overlap solve D_ov(m) x = eta (rho 1.5, m 0.2, degree-200 sign, window
    [0.003, 1] x 42.25) on 16^3 x 32, one Gaussian RHS, FP32 inner solves with
    FP64 defect correction to 1e-10."""
    L = (16, 16, 16, 32)
    g = w.Gauge(L, _dev(torch, li.near_identity_links(L, 0.2, 1005), dev))
    eta = _dev(torch, li.gaussian_spinor(L, 2005), dev)
    x = torch.zeros_like(eta)

    def run():
        x.zero_()
        return w.overlap_cg(g, eta, x, 1, 1.5, 0.2, 200, 0.003, 1.0, 42.25, 1e-10, 5000, "f32", 12, 1e-3)

    t, (st, info) = _timed(torch, run, reps=1)
    g.close()
    i = info[0]
    r = {"ms": round(t * 1e3, 1), "iters": i["iters"], "defect_corrections": i["reliable_updates"] + 1,
         "true_resid": i["true_resid"], "GBs": round(i["gbytes"] / t, 1),
         # 2 operator applications per inner iteration, 1 D^dagger per cycle, cycles + 1 FP64 residuals
         "hw_applications": (2 * i["iters"] + 2 * i["reliable_updates"] + 3) * (2 * 201 + 1)}
    log("overlap solve: %s" % r)
    return r


def dslash_sets(w, prec, recon, nrhs, vh):
    """Operand sets rotated by the cold protocol: at least 3, and together more
    than twice the 256 MB last-level cache, so no launch finds its operands
    left in a cache by the previous ones (the library allows at most 16)."""
    link = {"f64": 8, "f32": 4, "f16": 2, "bf16": 2}[prec] * recon * 8 * vh   # both parities, 4 directions
    site = {"f64": 192, "f32": 96, "f16": 52, "bf16": 52}[prec]
    per_set = link + 2 * nrhs * site * vh                                      # links, in, out
    n = max(3, -(-(2 * 256 * 2 ** 20 + 1) // per_set))
    return min(n, 16), per_set


# bytes per output site of a hop that reads every neighbour spinor from memory
NAIVE_BYTES = {("f64", 18): 2880, ("f64", 12): 2496, ("f32", 18): 1440, ("f32", 12): 1248, ("f16", 12): 660,
               ("bf16", 12): 660}

DSLASH_CASES = [("32", "f16", 12, 1), ("32", "f32", 12, 1), ("32", "bf16", 12, 1), ("32", "f64", 18, 1),
                ("24", "f64", 18, 1), ("24", "f64", 12, 1), ("24", "f32", 18, 1), ("24", "f32", 12, 1),
                ("24", "f16", 12, 1), ("24b", "f32", 12, 12), ("24b", "f16", 12, 12)]
DSLASH_LATTICE = {"32": (32, 32, 32, 64), "24": (24, 24, 24, 48), "24b": (24, 24, 24, 48)}


def dslash_tag(lat, prec, rc, nrhs):
    L = DSLASH_LATTICE[lat]
    return "%dc%d_%s_r%d%s" % (L[0], L[3], prec, rc, "" if nrhs == 1 else "_%drhs" % nrhs)


def bench_dslash(w, torch, li, dev, a, gauges, only=None, protocols=("warm", "cold")):
    """Stand-alone single-parity hops (D-slash) in the warm (operands reused,
    as inside a solver) and cold (rotated operand sets) protocols.  gauges maps
    "32", "24" and "24b" (a second 24^3x48 handle for the multi-RHS cases) to
    gauge handles; `only`, if given, is the set of case tags to run."""
    ds = {}
    stream = torch.cuda.current_stream()
    for lat, prec, rc, nrhs in DSLASH_CASES:
        tag = dslash_tag(lat, prec, rc, nrhs)
        if only is not None and tag not in only:
            continue
        g, L = gauges[lat], DSLASH_LATTICE[lat]
        vh = int(np.prod(L)) // 2
        bps = nrhs * w.wl_hop_bytes_per_site(prec, rc, nrhs)
        nsets, per_set = dslash_sets(w, prec, rc, nrhs, vh)
        for ns, name in [(1, "warm"), (nsets, "cold")]:
            if name not in protocols:
                continue
            # one untimed trial (tuning, packing, warm-up launches), then the
            # median of 5 timed trials of back-to-back launches
            reps = 100 if nrhs == 1 else 20
            try:
                w.wl_bench_dslash(g, prec, rc, nrhs, 0, ns, 10, stream)
                trials = sorted(w.wl_bench_dslash(g, prec, rc, nrhs, 0, ns, reps, stream) for _ in range(5))
            except w.WilsonError as e:
                ds["%s_%s" % (tag, name)] = {"error": str(e)}
                continue
            sec = trials[2]
            gbs = bps * vh / sec / 1e9
            rec = {"us": round(sec * 1e6, 2), "us_min_max": [round(trials[0] * 1e6, 2), round(trials[-1] * 1e6, 2)],
                   "GBs": round(gbs, 1), "frac": round(gbs / HBM_PEAK_GBS, 4),
                   "TFLOPs": round(nrhs * 1320 * vh / sec / 1e12, 3),
                   "sets": ns, "rotated_MB": round(ns * per_set / 1e6, 1)}
            if nrhs == 1:
                # the byte count of a hop that reads all 8 neighbours' full
                # spinors and 18-real links (QUDA's naive model)
                rec["naive_GBs"] = round(NAIVE_BYTES[(prec, rc)] * vh / sec / 1e9, 1)
            ds["%s_%s" % (tag, name)] = rec
            log("dslash %s %s: %s" % (tag, name, rec))
    return ds


def copy_reference(w, stream, ds):
    """Bandwidth reference: a plain non-temporal copy of a known size (read +
    write); its rocprofv3 FETCH_SIZE / WRITE_SIZE readings calibrate the
    traffic counters.  Beside it, what ordinary (cached) accesses reach when
    the operands fit the 256 MB last-level cache (a 64 MiB copy, a 128 MiB
    read) and when they do not (a 1 GiB read).  Adds each D-slash record's
    fraction of the copy rate."""
    copy_bytes = 256 << 20
    sec = w.wl_bench_copy(copy_bytes, 4, stream)
    ref = {"bytes_each_way": copy_bytes, "GBs": round(2 * copy_bytes / sec / 1e9, 1)}
    for key, nbytes, mode, moved in (("cached_copy_64MiB_GBs", 64 << 20, 1, 2), ("cached_read_128MiB_GBs", 128 << 20, 2, 1),
                                     ("read_1GiB_GBs", 1 << 30, 2, 1)):
        ref[key] = round(moved * nbytes / w.wl_bench_copy(nbytes, 50 if nbytes < (1 << 30) else 10, stream, mode) / 1e9, 1)
    for rec in (ds or {}).values():
        if isinstance(rec, dict) and "GBs" in rec:
            rec["frac_of_copy"] = round(rec["GBs"] / ref["GBs"], 4)
    log("copy %d MiB: %.1f GB/s (read + write)" % (copy_bytes >> 20, ref["GBs"]))
    return ref


def cpu_model():
    try:
        for line in open("/proc/cpuinfo"):
            if line.startswith("model name"):
                return line.split(":", 1)[1].strip()
    except OSError:
        pass
    return "unknown"


def cpu_baseline(w, L, U, eta, kappa, tol, a):
    """The FP64 oracle on a bounded sample of the headline workload: a capped
    number of CGNR iterations with every host thread (setup and true residual
    included), and single-parity hops with every thread and with one; and a
    sample of the sign-function workload."""
    import lattice_inputs as li
    import oracle

    vh = int(np.prod(L)) // 2
    nthreads = oracle.num_threads()
    t0 = time.perf_counter()
    _, _, it, _ = oracle.cg_eo(L, U, eta, kappa, tol, maxiter=a.cpu_iters)
    dt = time.perf_counter() - t0
    n_it = int(it[0])
    cg_bytes = n_it * cg_iteration_bytes(w, "f64", 18, vh)
    hop_b = w.wl_hop_bytes_per_site("f64", 18, 1) * vh
    t0 = time.perf_counter()
    for _ in range(2):
        oracle.hop(L, U, eta, out_parity=0)
    hop_all = (time.perf_counter() - t0) / 2
    oracle.set_num_threads(1)
    try:
        t0 = time.perf_counter()
        oracle.hop(L, U, eta, out_parity=0)
        hop_one = time.perf_counter() - t0
    finally:
        oracle.set_num_threads(nthreads)
    r = {
        "value": round(cg_bytes / dt / 1e9, 3),
        "unit": "GB/s",
        "cores": nthreads,
        "kind": "oracle",
        "sample": "FP64 oracle e/o CGNR on the same %dx%dx%dx%d system (kappa %g), capped at %d iterations "
                  "(%.1f s incl. setup; FP64 recon-18 byte model of the iterations only), %d threads"
                  % (L + (kappa, n_it, dt, nthreads)),
        "cpu_model": cpu_model(),
        "ms_per_cg_iteration": round(dt * 1e3 / max(n_it, 1), 1),
        "dslash_all_threads": {"ms": round(hop_all * 1e3, 1), "GBs": round(hop_b / hop_all / 1e9, 3),
                               "GFLOPs": round(1320 * vh / hop_all / 1e9, 2), "threads": nthreads},
        "dslash_one_thread": {"ms": round(hop_one * 1e3, 1), "GBs": round(hop_b / hop_one / 1e9, 3),
                              "GFLOPs": round(1320 * vh / hop_one / 1e9, 2), "threads": 1},
    }
    # the sign-function workload (16^3 x 32, rho 1.5), sampled: one right-hand
    # side at degree 10 (21 H_W applications) instead of 12 at degree 200
    # (403 each); per H_W application, and the time the full workload would take
    Ls = (16, 16, 16, 32)
    Us = li.near_identity_links(Ls, 0.2, 1005)
    vs = li.gaussian_spinor(Ls, 2005)
    t0 = time.perf_counter()
    oracle.sign_cheb(Ls, Us, vs, 1.5, 10, 0.003, 1.0, 42.25)
    ts = time.perf_counter() - t0
    # the small exact case (4^4 Haar links, kappa 0.12, tol 1e-12), whole solve
    L1 = (4, 4, 4, 4)
    U1 = li.haar_links(L1, 1001)
    e1 = li.gaussian_spinor(L1, 2001)
    t0 = time.perf_counter()
    _, _, it1, _ = oracle.cg_eo(L1, U1, e1, 0.12, 1e-12)
    r["cg_4c4_exact_case"] = {"ms": round((time.perf_counter() - t0) * 1e3, 2), "iters": int(it1[0])}
    r["sign_function_16c32_sample"] = {
        "sample": "1 rhs, degree 10 (21 H_W applications), %d threads" % nthreads,
        "ms": round(ts * 1e3, 1), "ms_per_hw_application": round(ts * 1e3 / 21, 2),
        "full_workload_estimate_s": round(ts / 21 * 403 * 12, 1)}
    log("cpu oracle: %s" % r)
    return r


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=10)
    ap.add_argument("--warmup", type=int, default=2)
    ap.add_argument("--sloppy", default="f16", choices=["f64", "f32", "f16", "bf16"])
    ap.add_argument("--recon", type=int, default=12)
    ap.add_argument("--delta", type=float, default=0.1)
    ap.add_argument("--cpu-iters", type=int, default=20,
                    help="cap on the oracle CG iterations timed for the CPU baseline (a bounded sample)")
    ap.add_argument("--no-cpu", action="store_true")
    ap.add_argument("--no-extra", action="store_true", help="skip every side measurement")
    ap.add_argument("--extras", default="cg,c2,dslash,batch,uneven,sign,overlap,clover",
                    help="side measurements outside the timed region (comma list)")
    ap.add_argument("--dslash-only", default=None,
                    help="run only these D-slash cases (comma list of tags such as 24c48_f32_r12_12rhs) and print "
                         "their results: for counter profiles of one kernel")
    ap.add_argument("--dslash-protocols", default="warm", help="with --dslash-only: warm, cold or warm,cold")
    a = ap.parse_args()
    if a.gpus != 1:
        print("bench.py measures one GPU only: this build has no multi-GPU path (run with --gpus 1)", file=sys.stderr)
        return 2

    import torch

    import lattice_inputs as li
    from paper_2001_05706_amd import wilson as w

    w.lib()
    dev = torch.device("cuda:0")
    if a.dslash_only:
        only = set(a.dslash_only.split(","))
        known = {dslash_tag(*c) for c in DSLASH_CASES}
        if not only <= known:
            print("unknown D-slash case(s) %s; known: %s" % (sorted(only - known), sorted(known)), file=sys.stderr)
            return 2
        gauges = {}
        for lat, seed in (("32", 1003), ("24", 1002), ("24b", 1002)):
            if any(dslash_tag(*c) in only for c in DSLASH_CASES if c[0] == lat):
                gauges[lat] = w.Gauge(DSLASH_LATTICE[lat], _dev(torch, li.near_identity_links(
                    DSLASH_LATTICE[lat], 0.3, seed), dev))
        try:
            ds = bench_dslash(w, torch, li, dev, a, gauges, only, tuple(a.dslash_protocols.split(",")))
        finally:
            for g in gauges.values():
                g.close()
        out = {"dslash": ds, "copy_reference": copy_reference(w, torch.cuda.current_stream(), ds)}
        print(json.dumps(out), flush=True)
        return 0
    L = (32, 32, 32, 64)
    vh = int(np.prod(L)) // 2
    kappa, tol, maxiter = 0.1248, 1e-10, 5000

    t0 = time.time()
    U = li.near_identity_links(L, 0.3, 1003)
    eta = li.gaussian_spinor(L, 2003)
    log("inputs generated in %.1f s" % (time.time() - t0))
    Ud = torch.from_numpy(U.view(np.float64)).to(dev)
    etad = torch.from_numpy(eta.view(np.float64)).to(dev)
    x = torch.zeros_like(etad)
    g = w.Gauge(L, Ud)
    stream = torch.cuda.current_stream()

    def solve(sloppy, recon):
        x.zero_()
        st, info = w.wilson_cg(g, etad, x, 1, kappa, tol, maxiter, sloppy, recon, a.delta, stream=stream)
        return info[0]

    for i in range(a.warmup):
        info = solve(a.sloppy, a.recon)
        log("warmup %d: %d iters, %d updates, true resid %.2e, %.2f ms" %
            (i, info["iters"], info["reliable_updates"], info["true_resid"], info["seconds"] * 1e3))

    # ---- timed region: K complete solves, graphs on, nothing else on the stream
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    infos = [solve(a.sloppy, a.recon) for _ in range(a.steps)]
    torch.cuda.synchronize()
    t1 = time.perf_counter()
    ms_per_step = (t1 - t0) * 1e3 / a.steps
    gbytes = sum(i["gbytes"] for i in infos)
    value = gbytes / (t1 - t0)
    worst = max(i["true_resid"] for i in infos)
    log("timed: %d solves, %.3f ms/solve, %.1f GB/s algorithmic, worst true resid %.2e" %
        (a.steps, ms_per_step, value, worst))
    assert all(i["converged"] for i in infos) and worst <= tol

    # ---- per-kernel timing of the dominant kernel over the same K solves (the
    # solver runs without graphs while timing is on): HIP events recorded by
    # each hop's dispatch on the solver's stream give its launch duration (the
    # roofline's), and the blocks' device steady-clock stamps (first block
    # start to last block end) its own span beside it
    w.wl_prof_enable(True)
    w.wl_prof_select(a.sloppy)  # the dominant kernel: the sloppy-precision hop
    w.wl_prof_read()
    for _ in range(a.steps):
        solve(a.sloppy, a.recon)
    torch.cuda.synchronize()
    n_hop, hop_ms, hop_gb, hop_kms = w.wl_prof_read()
    w.wl_prof_enable(False)
    w.wl_prof_select(-1)
    hop_event_us = hop_ms * 1e3 / max(n_hop, 1)        # launch duration, HIP events
    hop_span_us = hop_kms * 1e3 / max(n_hop, 1)        # kernel span, device steady clock
    achieved = hop_gb / (hop_ms * 1e-3) if hop_ms > 0 else 0.0
    log("hop launches %d, mean launch %.2f us (HIP events; span %.2f us on the steady clock), %.1f GB/s" %
        (n_hop, hop_event_us, hop_span_us, achieved))

    storage = {"f64": "f64 links (recon-%d) and spinors", "f32": "f32 links (recon-%d) and spinors",
               "f16": "f16 links (recon-%d), f16 spinors with a per-site f32 norm",
               "bf16": "bf16 links (recon-%d), bf16 spinors with a per-site f32 norm"}[a.sloppy] % a.recon
    out = {
        "metric": METRIC,
        "value": round(value, 2),
        "unit": "GB/s",
        "n_gpus": 1,
        "steps": a.steps,
        "warmup": a.warmup,
        "ms_per_step": round(ms_per_step, 4),
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f64" if a.sloppy == "f64" else "f32",
        "data": "synthetic",
        "config": {
            "workload": "mixed-precision e/o CGNR solve to a 1e-10 true residual, %dx%dx%dx%d, eps=0.3 links "
                        "(seed 1003), kappa=%g, 1 Gaussian rhs (seed 2003)" % (L + (kappa,)),
            "lattice": list(L),
            "storage": storage,
            "arithmetic": "f32 iterations; f64 reliable updates, reductions and true residual"
                          if a.sloppy != "f64" else "f64",
            "sloppy_storage": a.sloppy,
            "recon": a.recon,
            "delta": a.delta,
            "iters": infos[0]["iters"],
            "reliable_updates": infos[0]["reliable_updates"],
            "true_resid": worst,
        },
        "roofline": {
            "kernel": "k_hop (single-parity Wilson hop, %s recon-%d, fused epilogue)" % (a.sloppy, a.recon),
            "bound": "hbm",
            "achieved": round(achieved, 1),
            "peak": HBM_PEAK_GBS,
            "unit": "GB/s",
            "frac": round(achieved / HBM_PEAK_GBS, 4),
            "traffic": measured_traffic(a.sloppy, a.recon, L),
            "mean_launch_us": round(hop_event_us, 3),
            "mean_span_us_clock": round(hop_span_us, 3),
            "launches": n_hop,
            "bytes_per_launch": round(hop_gb * 1e9 / max(n_hop, 1)),
        },
    }

    extras = set() if a.no_extra else set(a.extras.split(","))
    if "cg" in extras:
        # the plain FP64 GPU solver (recon 18) and the other storage formats on the
        # same workload, CGNR and BiCGStab
        cmp = {}
        for meth, fn in (("cgnr", w.wilson_cg), ("bicgstab", w.wilson_bicgstab)):
            for sl, rc in [("f64", 18), ("f32", 12), ("f16", 12), ("bf16", 12)]:
                def run():
                    x.zero_()
                    return fn(g, etad, x, 1, kappa, tol, maxiter, sl, rc, a.delta, stream=stream)[1][0]
                try:
                    t, inf = _timed(torch, run, reps=3)
                except w.WilsonError as e:
                    cmp["%s_%s" % (meth, sl)] = {"error": str(e)}
                    log("%s %s failed: %s" % (meth, sl, e))
                    continue
                cmp["%s_%s" % (meth, sl)] = {"ms": round(t * 1e3, 3), "iters": inf["iters"],
                                             "updates": inf["reliable_updates"],
                                             "escalations": inf["precision_escalations"],
                                             "true_resid": inf["true_resid"], "GBs": round(inf["gbytes"] / t, 1)}
                log("%s %s: %s" % (meth, sl, cmp["%s_%s" % (meth, sl)]))
        out["cg_time_to_1e-10_ms"] = cmp
        if "ms" in cmp.get("cgnr_f64", {}) and "ms" in cmp.get("cgnr_" + a.sloppy, {}):
            out["cg_speedup_vs_fp64"] = round(cmp["cgnr_f64"]["ms"] / cmp["cgnr_" + a.sloppy]["ms"], 3)
    side = {}
    U24 = eta24 = None
    if extras & {"c2", "clover", "dslash"}:
        L24 = (24, 24, 24, 48)
        U24 = li.near_identity_links(L24, 0.3, 1002)
        eta24 = li.gaussian_spinor(L24, 2002)
    if "dslash" in extras:
        def run_ds():
            g24 = w.Gauge((24, 24, 24, 48), _dev(torch, U24, dev))
            g24b = w.Gauge((24, 24, 24, 48), _dev(torch, U24, dev))
            try:
                return bench_dslash(w, torch, li, dev, a, {"32": g, "24": g24, "24b": g24b})
            finally:
                g24.close()
                g24b.close()
        out["dslash"] = _guard(run_ds)
    if "c2" in extras:
        side["solves_24c48"] = _guard(lambda: bench_c2(w, torch, li, dev, a, U24, eta24))
    if "batch" in extras:
        side["batched_12_point_sources"] = _guard(lambda: bench_batch12(w, torch, li, dev, a))
    if "uneven" in extras:
        side["uneven_batch_16_lattices"] = _guard(lambda: bench_uneven(w, torch, li, dev, a))
    if "sign" in extras:
        side["sign_function_16c32"] = _guard(lambda: bench_sign(w, torch, li, dev, a))
    if "overlap" in extras:
        side["overlap_solve_16c32"] = _guard(lambda: bench_overlap(w, torch, li, dev, a))
    if "clover" in extras:
        side["clover_cg_24c48"] = _guard(lambda: bench_clover(w, torch, li, dev, a, U24, eta24))
    if side:
        out["configs"] = side

    out["copy_reference"] = copy_reference(w, stream, out.get("dslash"))

    g.close()
    if not a.no_cpu:
        out["cpu_baseline"] = cpu_baseline(w, L, U, eta, kappa, tol, a)

    print(json.dumps(out), flush=True)
    return 0


if __name__ == "__main__":
    sys.exit(main())
