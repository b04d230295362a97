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
import hashlib
import json
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

HBM_PEAK_GBS = 8000.0  # MI355X published HBM3E bandwidth
PROFILES = os.path.join(ROOT, "profiles")
# the sources of the dominant kernel (k_dslash); the committed byte counts
# are dropped as soon as any of them changes
KERNEL_SOURCES = ["paper_1010_5433_amd/csrc/dslash.hip", "paper_1010_5433_amd/csrc/common.h",
                  "paper_1010_5433_amd/csrc/links.h", "paper_1010_5433_amd/csrc/geom.h",
                  "paper_1010_5433_amd/csrc/internal.h"]


def log(msg):
    print(f"[bench] {msg}", file=sys.stderr, flush=True)


FMT_NROW = {"18": 3, "12": 2, "8": 1, "18p": 13, "12p": 12}   # "p": one field of float pairs


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


def kernel_source_hash() -> str:
    h = hashlib.sha256()
    for f in KERNEL_SOURCES:
        with open(os.path.join(ROOT, f), "rb") as fh:
            h.update(fh.read())
    return h.hexdigest()[:16]


def read_traffic(kernel: str):
    """HBM bytes per launch from the committed rocprofv3 counter summary,
    or None when the kernel sources changed since the counters were taken."""
    path = os.path.join(PROFILES, "dslash_traffic_32x32x32x32.txt")
    if not os.path.exists(path):
        return None
    vals = {}
    for line in open(path):
        if ":" in line and not line.startswith("#"):
            k, v = line.split(":", 1)
            vals[k.strip()] = v.strip()
    if vals.get("kernel_source_hash") != kernel_source_hash():
        return None
    key = f"traffic_bytes_per_launch[{kernel}]"
    return float(vals[key]) if key in vals else None


def time_dslash(lat, prec, n_warm=5, n_time=50):
    """Average duration of one half-Dslash launch, HIP events on the stream
    the library launches on (torch's current stream)."""
    import torch
    vh = lat.Vh
    dt = torch.float64 if prec == "f64" else torch.float32
    x = torch.randn((3, vh, 2), dtype=dt, device="cuda")
    y = torch.empty_like(x)
    for _ in range(n_warm):
        lat.dslash_eo(0, x, y)
        lat.dslash_eo(1, y, x)
    s = torch.cuda.current_stream()
    e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    e0.record(s)
    for k in range(n_time):
        if k & 1:
            lat.dslash_eo(1, y, x)
        else:
            lat.dslash_eo(0, x, y)
    e1.record(s)
    e1.synchronize()
    return e0.elapsed_time(e1) / n_time * 1e-3


def cpu_baseline(dims, U, b, mass, shifts, gpu_iters, sample_iters):
    """The FP64 oracle as it stands, on the host cores: the first
    `sample_iters` iterations of the same solve, scaled to the GPU's
    iteration count (every shift is still active in the sample, so the
    extrapolation is an upper bound of the oracle's time to solution)."""
    import oracle
    cores = len(os.sched_getaffinity(0))
    os.environ.setdefault("OMP_NUM_THREADS", str(cores))
    threads = int(os.environ["OMP_NUM_THREADS"])
    oracle.default()
    t0 = time.perf_counter()
    oracle.multishift_cg(dims, U, mass, shifts, b, tol=1e-10, max_iter=sample_iters)
    dt = time.perf_counter() - t0
    per_iter = dt / sample_iters
    return dict(value=round(per_iter * gpu_iters, 3), unit="s", cores=threads, kind="oracle",
                sample=f"first {sample_iters} multi-shift iterations of the same 32^4 solve "
                       f"({dt:.1f} s incl. 16 final true residuals), scaled by the GPU's "
                       f"{gpu_iters} iterations; {per_iter * 1e3:.1f} ms per iteration")


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
        log(f"batched {prec}: {t_b:.4f} s in one call vs {t_u:.4f} s one system after another "
            f"(first lattice's launch shape: block {block}, {rpt} right-hand sides per launch)")
        out[prec] = dict(batched_s=round(t_b, 4), sequential_s=round(t_u, 4), speedup=round(t_u / t_b, 3),
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
    unit weights): the whole call (one D_oe per shift, then the force
    launches of both parities) timed with events on the launch stream."""
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
    t_doe = time_dslash(lat, "f64")
    t_force = max(t - n * t_doe, 1e-9)
    b_force = force_bytes_per_site(nrow, n) * lat.V
    b_all = b_force + n * dslash_bytes_per_site(True, nrow) * lat.Vh
    return dict(shifts=n, call_ms=round(t * 1e3, 3), call_GBs=round(b_all / t / 1e9, 1),
                d_oe_us=round(t_doe * 1e6, 2), force_kernels_us_est=round(t_force * 1e6, 1),
                force_kernels_GBs_est=round(b_force / t_force / 1e9, 1),
                force_algorithmic_bytes=b_force, call_algorithmic_bytes=b_all,
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
    for phase in range(3):   # step size lr, lr/3, lr/10
        n = args.train_steps // 3 if phase < 2 else args.train_steps - 2 * (args.train_steps // 3)
        losses += learn.train(net, data, n, args.batch, lr, seed=phase, log=log)
        lr = args.lr / (3.0 if phase == 0 else 10.0)
    torch.cuda.synchronize()
    t_train = time.perf_counter() - t0
    log(f"learned: {args.train_steps} Adam steps of {args.batch} pairs in {t_train:.1f} s, "
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
        for name in res:
            if res[name]["status"] != 0 or res[name]["resid_true"] > tol:
                raise RuntimeError(f"learned evaluation failed: {name} {res[name]}")
        log(f"held-out field {seed}: " + ", ".join(
            f"{n} {res[n]['iters']} it {res[n]['seconds']:.4f} s" for n in res))
        evals.append(dict(field_seed=seed, **{f"{n}_{k2}": v for n in res
                                               for k2, v in res[n].items() if k2 != "status"}))
        del lat
    gains = {}
    for mode in ("bf16", "folded", "folded_bf16"):
        gains[mode] = dict(
            iteration_gain=round(float(np.mean([e["plain_iters"] / e[f"{mode}_iters"] for e in evals])), 3),
            tts_gain=round(float(np.mean([e["plain_seconds"] / e[f"{mode}_seconds"] for e in evals])), 3))
    return dict(train=dict(dims=list(c["train_dims"]), fields=nf, pairs_per_field=npairs, pairs=args.pairs,
                           steps=args.train_steps, batch=args.batch, lr=args.lr, mode="bf16",
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
    ap.add_argument("--cpu-sample-iters", type=int, default=40)
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
        print(f"bench.py runs on one GPU only (asked for --gpus {args.gpus}); "
              "the multi-GPU decomposition is a design, not part of this build", file=sys.stderr)
        sys.exit(2)

    import numpy as np
    import torch

    import paper_1010_5433_amd as stag
    import stag_synth as syn

    if args.batched_only:
        torch.cuda.set_device(0)
        print(json.dumps({"batched": batched_experiment(args)}), flush=True)
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
            time_dslash(lat, it_prec, n_warm=2, n_time=args.only_dslash)
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

    # ---- roofline of the dominant kernel: the half-Dslash in the step's precision
    dbl = it_prec == "f64"
    nrow = FMT_NROW[args.fmt]
    sec = time_dslash(lat, it_prec)
    algo = dslash_bytes_per_site(dbl, nrow) * lat.Vh
    achieved = algo / sec / 1e9
    kname = f"k_dslash<{'double' if dbl else 'float'},{nrow},PLAIN>"
    traffic = read_traffic(kname)
    roof = dict(bound="hbm", achieved=round(achieved, 1), peak=HBM_PEAK_GBS, unit="GB/s",
                frac=round(achieved / HBM_PEAK_GBS, 4), traffic=traffic,
                kernel=kname, bytes_per_launch=algo, avg_launch_us=round(sec * 1e6, 2))
    # every precision and link format, for the record (same field, repacked)
    dsl = {}
    for fmt in ("8", "12", "18", "12p", "18p"):
        if fmt != args.fmt:
            lat.set_links(torch.from_numpy(U).cuda(), fmt)
        for p in ("f64", "f32"):
            d = p == "f64"
            s = time_dslash(lat, p)
            gbs = dslash_bytes_per_site(d, FMT_NROW[fmt]) * lat.Vh / s / 1e9
            dsl[f"{p}_{fmt}"] = dict(us=round(s * 1e6, 2), GBs=round(gbs, 1), frac=round(gbs / HBM_PEAK_GBS, 4),
                                     traffic=read_traffic(f"k_dslash<{'double' if d else 'float'},{FMT_NROW[fmt]},PLAIN>"))
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
        extra["learned"] = learned_experiment(args, 1)

    cpu = None
    if not args.no_cpu_baseline:
        log(f"cpu baseline: oracle, first {args.cpu_sample_iters} iterations")
        cpu = cpu_baseline(dims, U, b, mass, shifts, st["iters"] + st["refine_iters"], args.cpu_sample_iters)

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
