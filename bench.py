#!/usr/bin/env python3
"""Benchmark: multi-shift CG time-to-solution at 1e-10 relative residual
on the 32^4 lattice (smoothed links, m = 0.01, 16 shifts in [1e-6, 4]),
plus the HBM roofline of the dominant kernel and the FP64 CPU oracle timed
on the host beside it.

    python bench.py [--gpus 1] [--steps K] [--warmup W] [--prec mixed|f64|f32]

One step = one full multi-shift solve (all shifts to FP64 true relative
residual <= 1e-10, including the final true-residual check), with the gauge
field and the source already resident in HBM.  Prints one JSON line.
"""
from __future__ import annotations

import argparse
import json
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

HBM_PEAK_GBS = 8000.0  # MI355X published HBM3E bandwidth
PROFILES = os.path.join(ROOT, "profiles")
# instruction hashes of the kernels of this build, written by the build
KERNEL_HASHES = os.path.join(ROOT, "paper_1010_5433_amd", "libstag.kernels.json")
# byte counters are committed per kernel together with the hash of its
# instructions: they are reported only while the built kernel is that one
KERNEL_SYMBOL = {
    "k_dslash<double,1,PLAIN>": "void stag::k_dslash<double, 1, 0>(stag::DslashArgs)",
    "k_dslash<double,2,PLAIN>": "void stag::k_dslash<double, 2, 0>(stag::DslashArgs)",
    "k_dslash<double,3,PLAIN>": "void stag::k_dslash<double, 3, 0>(stag::DslashArgs)",
    "k_dslash<float,1,PLAIN>": "void stag::k_dslash<float, 1, 0>(stag::DslashArgs)",
    "k_dslash<float,2,PLAIN>": "void stag::k_dslash<float, 2, 0>(stag::DslashArgs)",
    "k_dslash<float,3,PLAIN>": "void stag::k_dslash<float, 3, 0>(stag::DslashArgs)",
    "k_force<1>": "void stag::k_force<1>(stag::ForceArgs)",
}


def log(msg):
    print(f"[bench] {msg}", file=sys.stderr, flush=True)


FMT_NROW = {"18": 3, "12": 2, "8": 1, "18p": 13, "12p": 12}   # "p": one field of float pairs


MALL_MB = 256.0   # Infinity Cache


def link_field_bytes(dbl: bool, nrow: int, vh: int) -> int:
    """Bytes of the packed link field the half-Dslash of this precision
    reads (8 links per even site pair: 4 V links); a float-pair field is read
    whole in double precision and its single precision half otherwise."""
    rows = nrow - 10 if nrow > 10 else nrow
    per_link = (16 if dbl else 8) * (4 if rows == 1 else 3 * rows)
    return 8 * vh * per_link


def dslash_bytes_per_site(dbl: bool, nrow: int, mode: str = "plain") -> int:
    """Minimum unique HBM traffic of one half-Dslash per output site: all 8
    links once, the input vector once (neighbours re-read from cache), the
    output once; the normal-operator epilogue also reads p.  Links take
    9, 6 or 4 complex words (18-, 12- or 8-real storage); a float-pair
    field moves the same bytes as the double field in double precision and
    its single precision half in single precision."""
    rows = nrow - 10 if nrow > 10 else nrow
    bl = (16 if dbl else 8) * (4 if rows == 1 else 3 * rows)
    bv = 48 if dbl else 24
    return 8 * bl + (3 if mode == "epilogue" else 2) * bv


def built_kernel_hash(kernel: str):
    try:
        with open(KERNEL_HASHES) as fh:
            return json.load(fh).get(KERNEL_SYMBOL.get(kernel, kernel))
    except (OSError, ValueError):
        return None


def read_traffic(kernel: str, summary: str = "dslash_traffic_32x32x32x32.txt"):
    """HBM bytes per launch from a committed rocprofv3 counter summary, or
    None when the built kernel's instructions differ from the ones the
    counters were taken on (or no counters exist for it)."""
    path = os.path.join(PROFILES, summary)
    if not os.path.exists(path):
        return None
    vals = {}
    for line in open(path):
        if ":" in line and not line.startswith("#"):
            k, v = line.split(":", 1)
            vals[k.strip()] = v.strip()
    h = built_kernel_hash(kernel)
    if h is None or vals.get(f"kernel_isa_hash[{kernel}]") != h:
        return None
    key = f"traffic_bytes_per_launch[{kernel}]"
    return float(vals[key]) if key in vals else None


def time_dslash(lat, prec, n_warm=5, n_time=100, n_rep=3):
    """Average duration of one half-Dslash launch: HIP events on the stream
    the library launches on (torch's current stream) around n_time
    back-to-back launches, the median over n_rep such loops.  A rocprofv3
    kernel trace of such loops shows the launches back to back (under 0.1 us
    between one kernel's end and the next one's start on average), so the
    figure is the kernel's own duration.  Events around single launches
    were measured to add several microseconds each, inside the solver as
    well as here, so the bench does not time launches one by one."""
    import torch
    vh = lat.Vh
    dt = torch.float64 if prec == "f64" else torch.float32
    x = torch.randn((3, vh, 2), dtype=dt, device="cuda")
    y = torch.empty_like(x)
    for _ in range(n_warm):
        lat.dslash_eo(0, x, y)
        lat.dslash_eo(1, y, x)
    s = torch.cuda.current_stream()
    loops = []
    for _ in range(n_rep):
        e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        e0.record(s)
        for k in range(n_time):
            if k & 1:
                lat.dslash_eo(1, y, x)
            else:
                lat.dslash_eo(0, x, y)
        e1.record(s)
        e1.synchronize()
        loops.append(e0.elapsed_time(e1) / n_time * 1e-3)
    return sorted(loops)[len(loops) // 2]


def time_dslash_burst(lat, prec, n_burst=20, n_warm=4, n_rep=5, idle_s=0.05):
    """Average duration of one half-Dslash launch at the operating point of
    the solve: HIP events on the launch stream around a burst of n_burst
    back-to-back launches (after n_warm untimed ones and an idle pause of
    idle_s), the median over n_rep bursts.  Kernel traces show the launches
    of a sustained back-to-back loop starting at the duration the kernel has
    inside the solve (where it alternates with the lighter vector kernels)
    and slowing by 10-30 % within about fifty launches; a short burst stays
    at the first figure, which is what the timed solve sees."""
    import torch
    vh = lat.Vh
    dt = torch.float64 if prec == "f64" else torch.float32
    x = torch.randn((3, vh, 2), dtype=dt, device="cuda")
    y = torch.empty_like(x)
    s = torch.cuda.current_stream()
    bursts = []
    for _ in range(n_rep):
        torch.cuda.synchronize()
        time.sleep(idle_s)
        for k in range(n_warm):
            if k & 1:
                lat.dslash_eo(1, y, x)
            else:
                lat.dslash_eo(0, x, y)
        e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        e0.record(s)
        for k in range(n_burst):
            if k & 1:
                lat.dslash_eo(1, y, x)
            else:
                lat.dslash_eo(0, x, y)
        e1.record(s)
        e1.synchronize()
        bursts.append(e0.elapsed_time(e1) / n_burst * 1e-3)
    return sorted(bursts)[len(bursts) // 2]


def _omp_set_threads(n: int):
    """Thread count of the oracle's OpenMP loops from now on (the loops run
    on the calling thread's team)."""
    import ctypes
    ctypes.CDLL("libgomp.so.1").omp_set_num_threads(int(n))


def cpu_baseline(dims, U, b, mass, shifts, tol, one_core_iters=5):
    """The FP64 oracle as it stands, on the host cores: the whole multi-shift
    solve of the same workload (every shift to 1e-10, the 16 final true
    residuals included), then the time of one iteration on one core (the
    first `one_core_iters` iterations of the same solve on one thread)."""
    import oracle
    cores = len(os.sched_getaffinity(0))
    oracle.default()
    _omp_set_threads(cores)
    t0 = time.perf_counter()
    _, rc, info = oracle.multishift_cg(dims, U, mass, shifts, b, tol=tol)
    dt = time.perf_counter() - t0
    if rc != 0:
        raise RuntimeError(f"oracle solve failed ({rc})")
    _omp_set_threads(1)
    t0 = time.perf_counter()
    oracle.multishift_cg(dims, U, mass, shifts, b, tol=tol, max_iter=one_core_iters)
    dt1 = (time.perf_counter() - t0) / one_core_iters
    _omp_set_threads(cores)
    return dict(value=round(dt, 3), unit="s", cores=cores, kind="oracle",
                sample=f"the whole solve on {cores} threads ({info['iters']} iterations, 16 final true "
                       f"residuals); one core: {dt1 * 1e3:.0f} ms per iteration (first {one_core_iters} "
                       f"iterations, their true residuals included)",
                iters=info["iters"], one_core_s_per_iter=round(dt1, 4))


# The paper's Table 2: its single precision Dirac kernel on a Tesla C1060
# (102 GB/s), 12-real links, on three lattices (N_t x N_s^3).
PAPER_TAB2 = {(16, 16, 16, 4): 56.84, (32, 32, 32, 32): 64.091, (48, 48, 48, 4): 69.94}
C1060_GBS = 102.0


def tab2_experiment():
    """The half-Dslash on the paper's three Table 2 lattices (4 x 16^3,
    32 x 32^3, 4 x 48^3): single precision with 12-real links, the paper's
    setting, and double precision with 8-real links, the solver's.  Bytes
    are the algorithmic ones (all links once, the input and output vectors
    once); the paper's GB/s and fraction of its GPU's peak stand beside,
    as context."""
    import torch

    import paper_1010_5433_amd as stag
    import stag_synth as syn

    out = {}
    for dims, paper_gbs in PAPER_TAB2.items():
        U = torch.from_numpy(syn.smooth_links(dims, 0.5, 11)).cuda()
        lat = stag.Lattice(dims)
        row = {}
        for fmt, prec in (("12", "f32"), ("8", "f64")):
            lat.set_links(U, fmt)
            s = time_dslash(lat, prec)
            dbl = prec == "f64"
            gbs = dslash_bytes_per_site(dbl, FMT_NROW[fmt]) * lat.Vh / s / 1e9
            link_mb = link_field_bytes(dbl, FMT_NROW[fmt], lat.Vh) / 1e6
            row[f"{prec}_{fmt}"] = dict(us=round(s * 1e6, 2), GBs=round(gbs, 1), frac=round(gbs / HBM_PEAK_GBS, 4),
                                        link_field_MB=round(link_mb, 1),
                                        label=("effective (MALL-resident)" if link_mb < MALL_MB else "HBM"))
        row["paper_f32_12"] = dict(GBs=paper_gbs, frac=round(paper_gbs / C1060_GBS, 4), gpu="Tesla C1060")
        out["x".join(str(d) for d in dims)] = row
        del lat, U
    log(f"paper Table 2 lattices: {out}")
    return out


def config2_experiment(fmt):
    """Time to solution of the 32^3x8 workload (m = 0.02, 12 shifts in
    [1e-5, 2], FP64) on the GPU and with the FP64 oracle on the host cores,
    with the largest true residual of each computed by the oracle's operator."""
    import numpy as np
    import torch

    import oracle
    import paper_1010_5433_amd as stag
    import stag_synth as syn

    c = syn.config("c2_32x32x32x8_smooth")
    dims, mass, tol = c["dims"], c["mass"], c["tol"]
    shifts = syn.logspace_shifts(*c["shifts"])
    U = syn.make_links(c["links"], dims)
    b = syn.gaussian_source(dims, c["source_seed"])
    lat = stag.Lattice(dims)
    lat.set_links(torch.from_numpy(U).cuda(), fmt)
    src = lat.pack(torch.from_numpy(b).cuda())
    sols = [torch.empty_like(src) for _ in shifts]
    lat.multishift_cg(mass, shifts, src, sols=sols, tol=tol)   # warm-up
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    _, rc, st = lat.multishift_cg(mass, shifts, src, sols=sols, tol=tol)
    torch.cuda.synchronize()
    t_gpu = time.perf_counter() - t0
    if rc != 0:
        raise RuntimeError(f"config-2 solve failed ({rc})")
    xs = [lat.unpack(x).cpu().numpy() for x in sols]
    cores = len(os.sched_getaffinity(0))
    _omp_set_threads(cores)
    t0 = time.perf_counter()
    xo, rco, info = oracle.multishift_cg(dims, U, mass, shifts, b, tol=tol)
    t_cpu = time.perf_counter() - t0
    r_gpu = max(oracle.true_residual(dims, U, mass, s, b, x) for s, x in zip(shifts, xs))
    diff = max(float(np.linalg.norm(x - y) / np.linalg.norm(y)) for x, y in zip(xs, xo))
    log(f"config 2: GPU {t_gpu:.4f} s ({st['iters']} iterations), oracle {t_cpu:.2f} s on {cores} threads "
        f"({info['iters']} iterations); GPU true residual by the oracle's operator {r_gpu:.2e}; "
        f"largest solution difference {diff:.2e}")
    lat.close()
    return dict(lattice=list(dims), mass=mass, n_shifts=len(shifts), links=f"{fmt}-real", gpu_s=round(t_gpu, 4),
                gpu_iters=st["iters"], oracle_s=round(t_cpu, 3), oracle_iters=info["iters"], oracle_cores=cores,
                gpu_max_true_resid_by_oracle=r_gpu, max_rel_solution_diff=diff)


def batched_experiment(args):
    """The batched workload (8 pseudo-fermions x 16 shifts on 24^3x6 plus
    single sources on 8^4, 12^4 and 16^3x8) in one batched call against the
    same systems solved one after another, in double and in mixed precision."""
    import torch

    import paper_1010_5433_amd as stag
    import stag_synth as syn

    c = syn.config("c4_batched")
    tol = c["tol"]
    systems = []
    for y in c["systems"]:
        U = syn.smooth_links(y["dims"], 0.5, y["links"][2])
        lat = stag.Lattice(y["dims"])
        lat.set_links(torch.from_numpy(U).cuda(), args.fmt)
        shifts = [float(v) for v in syn.logspace_shifts(*y["shifts"])]
        for ss in y["source_seeds"]:
            b = syn.gaussian_source(y["dims"], ss)
            systems.append(dict(lat=lat, mass=y["mass"], shifts=shifts, src=lat.pack(torch.from_numpy(b).cuda())))
    out = dict(systems=len(systems), shifts=sum(len(s["shifts"]) for s in systems),
               lattices=[list(y["dims"]) for y in c["systems"]])
    for prec in ("f64", "mixed"):
        stag.multishift_cg_batched(systems, tol=tol, prec=prec)      # warm-up: launch-shape timing
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        sols, rc, st = stag.multishift_cg_batched(systems, tol=tol, prec=prec)
        torch.cuda.synchronize()
        t_b = time.perf_counter() - t0
        if rc != 0 or max(max(s["resid_true"]) for s in st) > tol:
            raise RuntimeError(f"batched solve failed: rc={rc}")
        block, rpt = stag.batch_last_config()
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        for y in systems:
            _, rc1, st1 = y["lat"].multishift_cg(y["mass"], y["shifts"], y["src"], tol=tol, prec=prec)
            if rc1 != 0 or max(st1["resid_true"]) > tol:
                raise RuntimeError(f"unbatched solve failed: rc={rc1}")
        torch.cuda.synchronize()
        t_u = time.perf_counter() - t0
        # the same batch without graph replays, and with one Dslash launch per lattice
        variants = {}
        for name, kw in (("no_graph", dict(no_graph=True)), ("per_lattice", dict(per_lattice=True)),
                         ("no_graph_per_lattice", dict(no_graph=True, per_lattice=True))):
            stag.multishift_cg_batched(systems, tol=tol, prec=prec, **kw)   # warm-up (launch shape)
            torch.cuda.synchronize()
            t0 = time.perf_counter()
            _, rcv, stv = stag.multishift_cg_batched(systems, tol=tol, prec=prec, **kw)
            torch.cuda.synchronize()
            variants[name] = round(time.perf_counter() - t0, 4)
            if rcv != 0 or max(max(s["resid_true"]) for s in stv) > tol:
                raise RuntimeError(f"batched solve ({name}) failed: rc={rcv}")
        log(f"batched {prec}: {t_b:.4f} s in one call vs {t_u:.4f} s one system after another "
            f"(first lattice's launch shape: block {block}, {rpt} right-hand sides per launch); "
            f"without graphs {variants['no_graph']:.4f} s, one launch per lattice {variants['per_lattice']:.4f} s, "
            f"neither {variants['no_graph_per_lattice']:.4f} s")
        out[prec] = dict(batched_s=round(t_b, 4), sequential_s=round(t_u, 4), speedup=round(t_u / t_b, 3),
                         variants_s=variants,
                         iters=[s["iters"] for s in st], refine_iters=[s["refine_iters"] for s in st],
                         max_resid_true=max(max(s["resid_true"]) for s in st),
                         launch_shape_first_lattice=dict(block=block, rhs_per_launch=rpt))
    return out


def force_bytes_per_site(nrow: int, n: int) -> int:
    """Minimum HBM traffic of the two force launches per lattice site: the
    4 links of the site once, the 4 force matrices written once (144 B
    each), and per shift the two vectors of each parity (X_i on even sites,
    D_oe X_i on odd sites, 48 B per site each) read once per launch."""
    rows = nrow - 10 if nrow > 10 else nrow
    bl = 16 * (4 if rows == 1 else 3 * rows)
    return 4 * bl + 4 * 144 + 96 * n


def force_experiment(lat, sols, nrow, reps=5):
    """Pseudo-fermion force from the headline solve's solutions (all shifts,
    unit weights): the whole call (Z_i = D_oe X_i, eight vectors per
    multi-right-hand-side launch, then the force launch) timed with events
    on the launch stream."""
    import torch

    n = len(sols)
    alphas = [1.0 / n] * n
    out = torch.empty((4, lat.V, 3, 3), dtype=torch.complex128, device="cuda")
    lat.fermion_force(alphas, sols, out=out)   # warm-up
    torch.cuda.synchronize()
    e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    e0.record()
    for _ in range(reps):
        lat.fermion_force(alphas, sols, out=out)
    e1.record()
    torch.cuda.synchronize()
    t = e0.elapsed_time(e1) / 1e3 / reps
    b_force = force_bytes_per_site(nrow, n) * lat.V
    # Z: the links once per launch of up to 8 vectors, each vector in and out once
    z_launches = (n + 7) // 8
    bl = dslash_bytes_per_site(True, nrow) - 2 * 48   # the 8 links of a site
    b_z = (z_launches * bl + n * 2 * 48) * lat.Vh
    traffic = read_traffic("k_force<1>", "fermion_force_32x32x32x32.md") if nrow == 1 else None
    return dict(shifts=n, call_ms=round(t * 1e3, 3), call_GBs=round((b_force + b_z) / t / 1e9, 1),
                force_traffic=traffic, z_launches=z_launches, force_algorithmic_bytes=b_force,
                z_algorithmic_bytes=b_z, call_algorithmic_bytes=b_force + b_z,
                finite=bool(torch.isfinite(torch.view_as_real(out)).all()))


def rational_experiment(lat, mass, src, tol, n_poles):
    """The RHMC's rational functions on the headline lattice: Zolotarev's
    M^(1/2) (heatbath of two flavours) and M^(-1/2) (their Metropolis
    action) on [m^2, m^2 + 16], applied with the weighted solutions summed
    on the fly, against the multi-shift solve of the same poles followed by
    the weighted sum."""
    import torch

    import paper_1010_5433_amd as stag

    lo, hi = mass * mass, mass * mass + 16.0
    out = {"poles": n_poles, "range": [lo, hi]}
    for name, power in (("heatbath_sqrt", 1), ("action_inv_sqrt", -1)):
        a0, al, sh, err = stag.zolotarev(power, lo, hi, n_poles)
        out.setdefault("coefficients", {})[name] = "Zolotarev"
        res = torch.empty_like(src)
        lat.rational_apply(mass, a0, al, sh, src, out=res, tol=tol)   # warm-up
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        _, rc, st, dot = lat.rational_apply(mass, a0, al, sh, src, out=res, tol=tol)
        t_rat = time.perf_counter() - t0
        if rc != 0:
            raise RuntimeError(f"rational application failed: {rc}")
        sols = [torch.empty_like(src) for _ in sh]
        lat.multishift_cg(mass, sh, src, sols=sols, tol=tol)   # warm-up, with the sum below
        comb = a0 * src
        for a, x in zip(al, sols):
            comb.add_(x, alpha=a)
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        _, rc2, st2 = lat.multishift_cg(mass, sh, src, sols=sols, tol=tol)
        comb = a0 * src
        for a, x in zip(al, sols):
            comb.add_(x, alpha=a)
        torch.cuda.synchronize()
        t_ms = time.perf_counter() - t0
        diff = float(torch.linalg.vector_norm(comb - res) / torch.linalg.vector_norm(comb))
        log(f"rational {name}: {t_rat:.4f} s ({st['iters']} iterations) vs multi-shift + sum {t_ms:.4f} s; "
            f"max rel. approximation error {err:.1e}; results differ by {diff:.1e}")
        out[name] = dict(seconds=round(t_rat, 4), iters=st["iters"], multishift_then_sum_s=round(t_ms, 4),
                         max_rel_err=err, rel_diff_vs_multishift=diff, re_src_dot_out=dot)
    # two flavours: heatbath phi = M^(1/4) xi (Remez, 20 poles), then the
    # action <phi, M^(-1/2) phi>, which must equal <xi, xi>
    h0, hl, hs, herr = stag.rational_power(0.25, lo, hi, 20)
    s0, sl, ss, serr = stag.zolotarev(-1, lo, hi, n_poles)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    phi, rc1, st1, _ = lat.rational_apply(mass, h0, hl, hs, src, tol=tol)
    t_h = time.perf_counter() - t0
    t0 = time.perf_counter()
    _, rc2, st2, action = lat.rational_apply(mass, s0, sl, ss, phi, tol=tol)
    t_a = time.perf_counter() - t0
    xx = float((src.double() * src.double()).sum())
    log(f"two-flavour heatbath M^(1/4) {t_h:.4f} s, action {t_a:.4f} s; S / <xi,xi> - 1 = {action / xx - 1:.2e} "
        f"(approximation errors {herr:.1e}, {serr:.1e})")
    out["two_flavour"] = dict(heatbath_quarter_s=round(t_h, 4), heatbath_poles=20, heatbath_max_rel_err=herr,
                              action_s=round(t_a, 4), action_over_xi2_minus_1=action / xx - 1,
                              iters=[st1["iters"], st2["iters"]])
    # several pseudo-fermions: the heatbath of 4 fields in one batched call
    # against 4 single calls
    nf = 4
    gen = torch.Generator(device="cuda")
    gen.manual_seed(1234)
    xis = [torch.randn(src.shape, generator=gen, dtype=torch.float64, device="cuda") * (0.5 ** 0.5) for _ in range(nf)]
    lat.rational_apply_multi(mass, h0, hl, hs, xis, tol=tol)   # warm-up (launch shape)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    _, rcm, stm, _ = lat.rational_apply_multi(mass, h0, hl, hs, xis, tol=tol)
    torch.cuda.synchronize()
    t_multi = time.perf_counter() - t0
    t0 = time.perf_counter()
    for xk in xis:
        lat.rational_apply(mass, h0, hl, hs, xk, tol=tol)
    torch.cuda.synchronize()
    t_single = time.perf_counter() - t0
    if rcm != 0:
        raise RuntimeError(f"batched rational application failed: {rcm}")
    log(f"heatbath of {nf} pseudo-fermions: {t_multi:.4f} s in one call vs {t_single:.4f} s one after another")
    out["pseudo_fermions"] = dict(fields=nf, batched_s=round(t_multi, 4), one_by_one_s=round(t_single, 4),
                                  speedup=round(t_single / t_multi, 3))
    return out


def rhmc_experiment(dims=(16, 16, 16, 16), n_md=16, n_g=4, n_forced=8, n_metro=4, n_meas=3):
    """RHMC trajectories of two staggered flavours on the GPU (the paper's
    setting: single precision gauge update and force inversions, double
    precision heatbath and Metropolis action): phi = M^(1/4) xi (Remez),
    the action with M^(-1/2) (Zolotarev), the molecular dynamics force with
    a coarser M^(-1/2).  After the thermalisation below, n_meas
    trajectories are timed in each precision from the same field, and the
    reversibility of the molecular dynamics is measured there: forward,
    momenta flipped, forward again.  Then n_meas trajectories in each
    precision with two pseudo-fermion fields (the paper's multiple
    pseudo-fermions), each with half the flavours' determinant.

    The synthetic start field is far from equilibrium at this coupling:
    n_forced trajectories with half the outer steps are accepted regardless
    (the field relaxes; dH falls from about 30 to 1), then n_metro
    trajectories with the Metropolis step."""
    import numpy as np
    import torch

    import paper_1010_5433_amd as stag
    import stag_synth as syn

    beta, mass, tau = 5.6, 0.05, 1.0
    lo, hi = mass * mass, mass * mass + 16.0
    rat_act = stag.zolotarev(-1, lo, hi, 16)[:3]
    rat_md = stag.zolotarev(-1, lo, hi, 8)[:3]
    rat_hb = stag.rational_power(0.25, lo, hi, 16)[:3]
    V = int(np.prod(dims))
    rng = np.random.default_rng(700)

    def params(prec, steps=n_md):
        return stag.rhmc_params(beta, mass, tau, steps, n_g, prec=prec, tol_md=1e-6 if prec == "f32" else 1e-10,
                                tol_act=1e-10, rat_md=rat_md, rat_act=rat_act, rat_hb=rat_hb)

    def draws():
        p = torch.from_numpy(rng.standard_normal((4, V, 8))).cuda()
        xi = torch.from_numpy((rng.standard_normal((V // 2, 3)) + 1j * rng.standard_normal((V // 2, 3)))
                              * np.sqrt(0.5)).cuda()
        return p, xi

    out = dict(lattice=list(dims), beta=beta, mass=mass, tau=tau, n_md=n_md, n_g=n_g, pseudo_fermions=1,
               rational=dict(heatbath="Remez M^(1/4), 16 poles", action="Zolotarev M^(-1/2), 16 poles",
                             md="Zolotarev M^(-1/2), 8 poles"))
    lat = stag.Lattice(dims)
    lat.set_links(torch.from_numpy(syn.smooth_links(dims, 0.5, 700)).cuda(), "18p")
    t0 = time.perf_counter()
    forced = []
    for _ in range(n_forced):
        p, xi = draws()
        forced.append(lat.rhmc_trajectory(params("f32", n_md // 2), p, [lat.pack(xi)], u=-1.0)["dH"])
    acc, dhs = 0, []
    for _ in range(n_metro):
        p, xi = draws()
        info = lat.rhmc_trajectory(params("f32"), p, [lat.pack(xi)], u=float(rng.uniform()))
        acc += info["accepted"]
        dhs.append(info["dH"])
    out["thermalisation"] = dict(seconds=round(time.perf_counter() - t0, 3), forced_trajectories=n_forced,
                                 forced_dH=[float(f"{v:.3g}") for v in forced], metropolis_trajectories=n_metro,
                                 accepted=acc, dH=[float(f"{v:.3g}") for v in dhs])
    log(f"rhmc: thermalisation {out['thermalisation']}")
    U_eq = lat.links_get()
    for prec in ("f32", "f64"):
        lat.set_links(U_eq, "18p")
        res = []
        for _ in range(n_meas):
            p, xi = draws()
            torch.cuda.synchronize()
            t0 = time.perf_counter()
            info = lat.rhmc_trajectory(params(prec), p, [lat.pack(xi)], u=-1.0)
            res.append((time.perf_counter() - t0, info))
        t = [r[0] for r in res]
        info = res[-1][1]
        log(f"rhmc {prec}: trajectories {min(t):.3f}-{max(t):.3f} s, dH {[round(r[1]['dH'], 4) for r in res]}, "
            f"{info['fermion_forces']} fermion forces, {info['md_iters']} MD iterations, "
            f"{info['action_iters']} heatbath/action iterations")
        r = dict(trajectory_s=[round(v, 4) for v in t], dH=[r[1]["dH"] for r in res],
                 fermion_forces=info["fermion_forces"], gauge_forces=info["gauge_forces"],
                 md_iters=info["md_iters"], action_iters=info["action_iters"])
        # reversibility of the molecular dynamics from the thermalised field
        lat.set_links(U_eq, "18p")
        U0 = lat.links_get()
        p0, xi = draws()
        phi = lat.rational_apply(mass, rat_hb[0], rat_hb[1], rat_hb[2], lat.pack(xi), tol=1e-10)[0]
        mom = p0.clone()
        lat.md_integrate(params(prec), mom, [phi])
        mom.neg_()
        lat.md_integrate(params(prec), mom, [phi])
        mom.neg_()
        dU = lat.links_get() - U0
        n_dof = 2 * U0.numel() + p0.numel()
        viol = float(torch.sqrt((torch.sum(torch.abs(dU) ** 2) + torch.sum((mom - p0) ** 2)) / n_dof))
        r["reversibility_per_dof"] = viol
        log(f"rhmc {prec}: reversibility {viol:.2e} per degree of freedom (paper, single precision update: ~5e-6)")
        out[prec] = r
    # the paper's multiple pseudo-fermions: two fields, each carrying half of
    # the two flavours' determinant (action M^(-1/4), heatbath M^(1/8)); their
    # solves, forces and rational functions are batched over the fields
    rat2 = dict(act=stag.rational_power(-0.25, lo, hi, 16), md=stag.rational_power(-0.25, lo, hi, 8),
                hb=stag.rational_power(0.125, lo, hi, 16))
    two = dict(pseudo_fermions=2, rational=dict(heatbath="M^(1/8), 16 poles", action="M^(-1/4), 16 poles",
                                                md="M^(-1/4), 8 poles"),
               rational_max_rel_err={k: float(f"{v[3]:.3g}") for k, v in rat2.items()})
    for prec in ("f32", "f64"):
        prm2 = stag.rhmc_params(beta, mass, tau, n_md, n_g, prec=prec, tol_md=1e-6 if prec == "f32" else 1e-10,
                                tol_act=1e-10, rat_md=rat2["md"][:3], rat_act=rat2["act"][:3], rat_hb=rat2["hb"][:3])
        lat.set_links(U_eq, "18p")
        res = []
        for _ in range(n_meas):
            p, xi = draws()
            _, xi2 = draws()
            torch.cuda.synchronize()
            t0 = time.perf_counter()
            info = lat.rhmc_trajectory(prm2, p, [lat.pack(xi), lat.pack(xi2)], u=-1.0)
            res.append((time.perf_counter() - t0, info))
        t = [r[0] for r in res]
        info = res[-1][1]
        log(f"rhmc {prec}, two pseudo-fermions: trajectories {min(t):.3f}-{max(t):.3f} s, "
            f"dH {[round(r[1]['dH'], 4) for r in res]}, {info['md_iters']} MD iterations")
        two[prec] = dict(trajectory_s=[round(v, 4) for v in t], dH=[r[1]["dH"] for r in res],
                         fermion_forces=info["fermion_forces"], md_iters=info["md_iters"],
                         action_iters=info["action_iters"])
    out["two_pseudo_fermions"] = two
    lat.close()
    return out


def learned_experiment(args, n_test_fields):
    """Train the gauge-equivariant preconditioner on 16^4 fields and test it
    in flexible CG on held-out 32^4 fields against plain FP64 CG."""
    fmt = args.learned_fmt or args.fmt
    import numpy as np
    import torch

    import paper_1010_5433_amd as stag
    import stag_synth as syn
    from paper_1010_5433_amd import learn

    c = syn.config("c5_learned")
    mass, tol = c["mass"], c["tol"]
    nf = args.train_fields or len(c["train_link_seeds"])
    npairs = args.train_pairs or c["sources_per_field"]
    t0 = time.perf_counter()
    data = []
    for k, seed in enumerate(c["train_link_seeds"][:nf]):
        U = syn.smooth_links(c["train_dims"], c["eps"], seed)
        lat = stag.Lattice(c["train_dims"])
        lat.set_links(torch.from_numpy(U).cuda(), "12")
        maker = learn.solve_pairs if args.pairs == "solve" else learn.make_pairs
        B, X = maker(lat, mass, npairs, seed=c["train_source_seed"] + k)
        data.append((lat, B, X))
    torch.cuda.synchronize()
    t_data = time.perf_counter() - t0
    log(f"learned: {nf} fields x {npairs} pairs ({args.pairs}) in {t_data:.1f} s")
    net = stag.Net(learn.init_theta(0, args.init_scale))
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    losses = []
    lr = args.lr
    plateau = (args.plateau_window, args.plateau_rtol) if args.plateau_window > 0 else None
    for phase in range(3):   # step size lr, lr/3, lr/10; each phase ends early at a plateau
        n = args.train_steps // 3 if phase < 2 else args.train_steps - 2 * (args.train_steps // 3)
        losses += learn.train(net, data, n, args.batch, lr, seed=phase, log=log, plateau=plateau)
        lr = args.lr / (3.0 if phase == 0 else 10.0)
    torch.cuda.synchronize()
    t_train = time.perf_counter() - t0
    log(f"learned: {len(losses)} Adam steps (at most {args.train_steps}) of {args.batch} pairs in {t_train:.1f} s, "
        f"loss {losses[0]:.4f} -> {np.mean(losses[-20:]):.4f}")
    del data
    evals = []
    for k, seed in enumerate(c["test_link_seeds"][:n_test_fields]):
        U = syn.smooth_links(c["test_dims"], c["eps"], seed)
        lat = stag.Lattice(c["test_dims"])
        lat.set_links(torch.from_numpy(U).cuda(), fmt)
        b = syn.gaussian_source(c["test_dims"], c["test_source_seed"] + k)
        src = lat.pack(torch.from_numpy(b).cuda())
        learn.compare(lat, net, mass, src, tol=tol)          # warm-up
        res = learn.compare(lat, net, mass, src, tol=tol)
        # the fixed two-hop polynomial P = (a + b) - M, a = m^2, b = 1.1 lambda_max,
        # in the same folded bfloat16 kernels: the network's closed-form competitor
        lmax = 1.1 * learn.lambda_max(lat, mass)
        poly = stag.Net(learn.polynomial_theta(lmax, 1.0, scale=1.0 / lmax))
        learn.compare(lat, poly, mass, src, tol=tol, modes=("folded_bf16",))
        pres = learn.compare(lat, poly, mass, src, tol=tol, modes=("folded_bf16",))
        res["polynomial_folded_bf16"] = pres["folded_bf16"]
        for name in res:
            if res[name]["status"] != 0 or res[name]["resid_true"] > tol:
                raise RuntimeError(f"learned evaluation failed: {name} {res[name]}")
        log(f"held-out field {seed}: " + ", ".join(
            f"{n} {res[n]['iters']} it {res[n]['seconds']:.4f} s" for n in res))
        evals.append(dict(field_seed=seed, **{f"{n}_{k2}": v for n in res
                                               for k2, v in res[n].items() if k2 != "status"}))
        del lat
    gains = {}
    for mode in ("bf16", "folded", "folded_bf16", "polynomial_folded_bf16"):
        gains[mode] = dict(
            iteration_gain=round(float(np.mean([e["plain_iters"] / e[f"{mode}_iters"] for e in evals])), 3),
            tts_gain=round(float(np.mean([e["plain_seconds"] / e[f"{mode}_seconds"] for e in evals])), 3))
    return dict(train=dict(dims=list(c["train_dims"]), fields=nf, pairs_per_field=npairs, pairs=args.pairs,
                           steps=len(losses), max_steps=args.train_steps,
                           plateau=list(plateau) if plateau else None, batch=args.batch, lr=args.lr, mode="bf16",
                           seconds=round(t_train, 2), data_seconds=round(t_data, 2),
                           loss_first=round(losses[0], 5), loss_last=round(float(np.mean(losses[-20:])), 5)),
                test=dict(dims=list(c["test_dims"]), mass=mass, shift=0.0, tol=tol, links=f"{fmt}-real",
                          fields=evals),
                gains=gains)


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=3)
    ap.add_argument("--warmup", type=int, default=1)
    ap.add_argument("--prec", default="f64", choices=["mixed", "f64", "f32"])
    ap.add_argument("--fmt", default="8", choices=["18", "12", "8", "18p", "12p"])
    ap.add_argument("--cpu-one-core-iters", type=int, default=5)
    ap.add_argument("--no-config2", action="store_true", help="skip the 32^3x8 GPU/oracle comparison")
    ap.add_argument("--no-tab2", action="store_true", help="skip the half-Dslash on the paper's Table 2 lattices")
    ap.add_argument("--tab2-only", action="store_true", help="run only the paper's Table 2 lattices")
    ap.add_argument("--no-rhmc", action="store_true", help="skip the 16^4 RHMC trajectory")
    ap.add_argument("--rhmc-only", action="store_true", help="run only the RHMC trajectory experiment")
    ap.add_argument("--learned-test-fields", type=int, default=4,
                    help="held-out 32^4 fields evaluated in the default run")
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--no-f64-reference", action="store_true")
    ap.add_argument("--no-mixed", action="store_true")
    ap.add_argument("--only-dslash", type=int, default=0,
                    help="profiling aid: run N half-Dslash launches of the bench's precision and exit")
    ap.add_argument("--only-force", type=int, default=0,
                    help="profiling aid: run N fermion-force calls (16 shifts) and exit")
    ap.add_argument("--no-learned", action="store_true", help="skip the learned-preconditioner experiment")
    ap.add_argument("--no-batched", action="store_true", help="skip the batched-solver experiment")
    ap.add_argument("--batched-only", action="store_true", help="run only the batched-solver experiment")
    ap.add_argument("--learned-only", action="store_true",
                    help="run only the learned-preconditioner experiment (all held-out fields)")
    ap.add_argument("--train-steps", type=int, default=1500)
    ap.add_argument("--plateau-window", type=int, default=50,
                    help="end a training phase once the mean loss of this many steps stops falling (0: never)")
    ap.add_argument("--plateau-rtol", type=float, default=0.005,
                    help="relative fall of the window mean below which a phase ends")
    ap.add_argument("--batch", type=int, default=32)
    ap.add_argument("--lr", type=float, default=1e-2)
    ap.add_argument("--init-scale", type=float, default=0.1)
    ap.add_argument("--train-fields", type=int, default=0)
    ap.add_argument("--train-pairs", type=int, default=0)
    ap.add_argument("--pairs", default="mx", choices=["mx", "solve"])
    ap.add_argument("--test-fields", type=int, default=4, help="held-out fields of --learned-only")
    ap.add_argument("--no-rational", action="store_true")
    ap.add_argument("--no-force", action="store_true", help="skip the fermion-force measurement")
    ap.add_argument("--rational-poles", type=int, default=24)
    ap.add_argument("--learned-fmt", default=None, choices=["18", "12", "8"],
                    help="link storage of the held-out fields of the learned experiment (default: --fmt)")
    args = ap.parse_args()

    if args.gpus != 1:
        print(f"bench.py runs on one GPU only (asked for --gpus {args.gpus}): the library drives a single "
              "GPU, with no collectives between GPUs", file=sys.stderr)
        sys.exit(2)

    import numpy as np
    import torch

    import paper_1010_5433_amd as stag
    import stag_synth as syn

    if args.batched_only:
        torch.cuda.set_device(0)
        print(json.dumps({"batched": batched_experiment(args)}), flush=True)
        return
    if args.rhmc_only:
        torch.cuda.set_device(0)
        print(json.dumps({"rhmc": rhmc_experiment()}), flush=True)
        return
    if args.tab2_only:
        torch.cuda.set_device(0)
        print(json.dumps({"tab2": tab2_experiment()}), flush=True)
        return
    if args.learned_only:
        torch.cuda.set_device(0)
        print(json.dumps({"learned": learned_experiment(args, args.test_fields)}), flush=True)
        return

    c = syn.config("c3_32x32x32x32_smooth")
    dims, mass, tol = c["dims"], c["mass"], c["tol"]
    shifts = syn.logspace_shifts(*c["shifts"])
    log(f"generating 32^4 smoothed links (seed {c['links'][2]})")
    U = syn.make_links(c["links"], dims)
    b = syn.gaussian_source(dims, c["source_seed"])
    torch.cuda.set_device(0)
    lat = stag.Lattice(dims)
    lat.set_links(torch.from_numpy(U).cuda(), args.fmt)
    src = lat.pack(torch.from_numpy(b).cuda())
    sols = [torch.empty_like(src) for _ in shifts]
    torch.cuda.synchronize()

    it_prec = "f64" if args.prec == "f64" else "f32"
    if args.only_dslash or args.only_force:
        if args.only_dslash:
            log(f"profiling aid: {args.only_dslash} half-Dslash launches ({it_prec}, {args.fmt}-real)")
            sec = time_dslash(lat, it_prec, n_warm=2, n_time=args.only_dslash, n_rep=1)
            log(f"half-Dslash by HIP events: {sec * 1e6:.2f} us per launch over {args.only_dslash} launches")
        if args.only_force:
            log(f"profiling aid: {args.only_force} fermion-force calls, 16 random solutions ({args.fmt}-real)")
            xs = [torch.randn(3, lat.Vh, 2, dtype=torch.float64, device="cuda") for _ in range(16)]
            out = torch.empty((4, lat.V, 3, 3), dtype=torch.complex128, device="cuda")
            for _ in range(args.only_force):
                lat.fermion_force([1.0 / 16] * 16, xs, out=out)
        # calibration of the byte counters: the probe copy reads and writes
        # exactly 2 GiB per launch
        x = torch.zeros(256 << 20, dtype=torch.float64, device="cuda")
        y = torch.empty_like(x)
        for _ in range(5):
            stag._L.stag_hbm_probe(x.data_ptr(), y.data_ptr(), 2 << 30, 1,
                                   torch.cuda.current_stream().cuda_stream)
        torch.cuda.synchronize()
        log("done")
        return

    def solve(prec):
        out, rc, st = lat.multishift_cg(mass, shifts, src, sols=sols, tol=tol, prec=prec)
        if rc != 0 or max(st["resid_true"]) > tol:
            raise RuntimeError(f"solve failed: rc={rc} resid={max(st['resid_true']):.3e}")
        return st

    for w in range(args.warmup):
        st = solve(args.prec)
        log(f"warmup {w}: {st['iters']} iters + {st['refine_iters']} refine, {st['seconds']:.3f} s")
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    stats = []
    for k in range(args.steps):
        stats.append(solve(args.prec))
        log(f"step {k}: {stats[-1]['iters']} iters + {stats[-1]['refine_iters']} refine, "
            f"{stats[-1]['seconds']:.3f} s")
    torch.cuda.synchronize()
    elapsed = time.perf_counter() - t0
    tts = elapsed / args.steps
    st = stats[-1]

    # ---- roofline of the dominant kernel: the half-Dslash in the step's precision,
    # timed in short bursts right after the timed solves (the solve's operating
    # point); a sustained loop of 300 launches is recorded beside it
    dbl = it_prec == "f64"
    nrow = FMT_NROW[args.fmt]
    sec = time_dslash_burst(lat, it_prec)
    sec_loop = time_dslash(lat, it_prec)
    algo = dslash_bytes_per_site(dbl, nrow) * lat.Vh
    achieved = algo / sec / 1e9
    kname = f"k_dslash<{'double' if dbl else 'float'},{nrow},PLAIN>"
    traffic = read_traffic(kname)
    roof = dict(bound="hbm", achieved=round(achieved, 1), peak=HBM_PEAK_GBS, unit="GB/s",
                frac=round(achieved / HBM_PEAK_GBS, 4), traffic=traffic,
                kernel=kname, bytes_per_launch=algo, avg_launch_us=round(sec * 1e6, 2),
                timing="HIP events around bursts of 20 back-to-back launches, median of 5",
                sustained_loop_us=round(sec_loop * 1e6, 2),
                sustained_loop_frac=round(algo / sec_loop / 1e9 / HBM_PEAK_GBS, 4))
    log(f"roofline: {roof}")

    extra = {}
    if args.prec != "f64" and not args.no_f64_reference:
        st64 = solve("f64")
        log(f"f64 reference: {st64['iters']} iters, {st64['seconds']:.3f} s")
        extra["f64_tts_s"] = round(st64["seconds"], 4)
        extra["f64_iters"] = st64["iters"]
    if args.prec == "f64" and not args.no_mixed:
        stm = solve("mixed")
        stm = solve("mixed")
        log(f"mixed: {stm['iters']} iters + {stm['refine_iters']} refine, {stm['seconds']:.3f} s")
        extra["mixed"] = dict(tts_s=round(stm["seconds"], 4), iters=stm["iters"],
                              refine_iters=stm["refine_iters"], n_reliable=stm["n_reliable"],
                              max_resid_true=max(stm["resid_true"]),
                              resid_unrefined=[float(f"{v:.3g}") for v in stm["resid_unrefined"]],
                              refine_iters_shift=stm["refine_iters_shift"])

    # ---- achievable HBM bandwidth in this run (4 GiB read-only and copy sweeps)
    probe = {}
    nbytes = 4 << 30
    a = torch.empty(nbytes // 4, dtype=torch.float32, device="cuda").uniform_(0.0, 1.0)
    bbuf = torch.empty_like(a)
    for kind, name, mult in ((0, "read", 1), (1, "copy", 2)):
        for _ in range(2):
            stag._L.stag_hbm_probe(a.data_ptr(), bbuf.data_ptr(), nbytes, kind,
                                   torch.cuda.current_stream().cuda_stream)
        e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        e0.record()
        for _ in range(5):
            stag._L.stag_hbm_probe(a.data_ptr(), bbuf.data_ptr(), nbytes, kind,
                                   torch.cuda.current_stream().cuda_stream)
        e1.record()
        e1.synchronize()
        probe[f"{name}_GBs"] = round(mult * nbytes * 5 / (e0.elapsed_time(e1) * 1e-3) / 1e9, 1)
    del a, bbuf
    log(f"hbm probe: {probe}")
    extra["hbm_probe"] = probe

    # every precision and link format, for the record (same field, repacked)
    dsl = {}
    loaded = args.fmt
    for fmt in ("8", "12", "18", "12p", "18p"):
        if fmt != loaded:
            lat.set_links(torch.from_numpy(U).cuda(), fmt)
            loaded = fmt
        for p in ("f64", "f32"):
            d = p == "f64"
            s = time_dslash(lat, p)
            gbs = dslash_bytes_per_site(d, FMT_NROW[fmt]) * lat.Vh / s / 1e9
            link_mb = link_field_bytes(d, FMT_NROW[fmt], lat.Vh) / 1e6
            dsl[f"{p}_{fmt}"] = dict(us=round(s * 1e6, 2), GBs=round(gbs, 1), frac=round(gbs / HBM_PEAK_GBS, 4),
                                     link_field_MB=round(link_mb, 1),
                                     label=("effective (MALL-resident)" if link_mb < MALL_MB else "HBM"),
                                     traffic=read_traffic(f"k_dslash<{'double' if d else 'float'},{FMT_NROW[fmt]},PLAIN>"))
    if loaded != args.fmt:
        lat.set_links(torch.from_numpy(U).cuda(), args.fmt)
    log(f"dslash: {dsl}")

    if args.prec == "f64" and not args.no_force:
        extra["force"] = force_experiment(lat, sols, nrow)
        log(f"force: {extra['force']}")
    if not args.no_rational:
        extra["rational"] = rational_experiment(lat, mass, src, tol, args.rational_poles)
    if not args.no_batched:
        extra["batched"] = batched_experiment(args)
    if not args.no_learned:
        extra["learned"] = learned_experiment(args, args.learned_test_fields)
    if not args.no_config2:
        extra["config2"] = config2_experiment(args.fmt)
    if not args.no_tab2:
        extra["tab2"] = tab2_experiment()
    if not args.no_rhmc:
        extra["rhmc"] = rhmc_experiment()

    cpu = None
    if not args.no_cpu_baseline:
        log("cpu baseline: the oracle's whole solve of the same workload, then one core")
        cpu = cpu_baseline(dims, U, b, mass, shifts, tol, args.cpu_one_core_iters)
        log(f"cpu baseline: {cpu}")

    out = {
        "metric": "multi-shift CG time-to-solution @1e-10 rel resid; Dslash HBM GB/s (% of peak)",
        "value": round(tts, 4),
        "unit": "s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": round(tts * 1e3, 2),
        "higher_is_better": False,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": {"mixed": "f32+f64", "f64": "f64", "f32": "f32"}[args.prec],
        "data": "synthetic",
        "config": {"workload": "32^4 smoothed SU(3) links (eps 0.5, seed 301), m=0.01, "
                               "16 shifts logspace[1e-6,4], 1 Gaussian source (seed 302), tol 1e-10",
                   "lattice": list(dims), "mass": mass, "n_shifts": len(shifts), "tol": tol,
                   "precision": args.prec, "links": f"{args.fmt}-real", "parallelism": "single GPU"},
        "iters": st["iters"],
        "refine_iters": st["refine_iters"],
        "n_reliable": st["n_reliable"],
        "max_resid_true": max(st["resid_true"]),
        "max_resid_unrefined": max(st["resid_unrefined"]),
        "resid_unrefined": [float(f"{v:.3g}") for v in st["resid_unrefined"]],
        "refine_iters_shift": st["refine_iters_shift"],
        "iters_shift": st["iters_shift"],
        "roofline": roof,
        "dslash": dsl,
        "cpu_baseline": cpu,
    }
    out.update(extra)
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
