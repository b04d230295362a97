"""Batched multi-shift CG (pseudo-fermions x shifts, uneven lattices) on
the GPU: every system against the oracle's operator, batched against
unbatched, every launch shape against every other, repeated calls bit for
bit."""
import numpy as np
import pytest

import stag_synth as syn
from tests.gpu_common import lattice_with_links, links_np, log, pack, rel, unpack

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module", autouse=True)
def _gpu():
    torch = pytest.importorskip("torch")
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    import paper_1010_5433_amd  # noqa: F401


def _setup(specs, fmt="18"):
    """specs: list of (dims, link_seed, mass, shifts, [source seeds])."""
    lats, systems, host = [], [], []
    for dims, lseed, mass, shifts, sseeds in specs:
        U = links_np(dims, "smooth", 0.5, lseed)
        lat = lattice_with_links(dims, U, fmt)
        lats.append(lat)
        for ss in sseeds:
            b = syn.gaussian_source(dims, ss)
            systems.append(dict(lat=lat, mass=mass, shifts=list(shifts), src=pack(lat, b)))
            host.append((dims, U, mass, shifts, b))
    return lats, systems, host


SMALL_BATCH = [
    ((8, 8, 8, 8), 41, 0.05, [1e-4, 0.01, 0.3, 1.0], [1, 2, 3]),
    ((6, 4, 4, 8), 42, 0.1, [0.0, 0.02, 0.5], [4]),
    ((4, 4, 4, 4), 43, 0.07, [2e-3, 0.2], [5, 6]),
]


@pytest.mark.parametrize("prec,fmt", [("f64", "18"), ("mixed", "18"), ("f64", "12p"), ("mixed", "12p")])
def test_batched_vs_oracle_and_unbatched(orc, prec, fmt):
    import torch
    import paper_1010_5433_amd as stag
    log(f"batched small prec={prec} fmt={fmt}")
    lats, systems, host = _setup(SMALL_BATCH, fmt)
    sols, rc, stats = stag.multishift_cg_batched(systems, prec=prec)
    torch.cuda.synchronize()
    assert rc == 0
    for k, (dims, U, mass, shifts, b) in enumerate(host):
        lat = systems[k]["lat"]
        ref, rc1, st1 = lat.multishift_cg(mass, shifts, systems[k]["src"], prec="f64")
        for i, s in enumerate(shifts):
            x = unpack(lat, sols[k][i])
            r = orc.true_residual(dims, U, mass, s, b, x)
            assert r <= 1e-10, (k, i, r)
            assert abs(stats[k]["resid_true"][i] - r) <= 1e-3 * r + 1e-16
            if prec == "f64":
                assert rel(x, unpack(lat, ref[i])) <= 1e-9
        if prec == "f64":
            assert abs(stats[k]["iters"] - st1["iters"]) <= 1


@pytest.mark.parametrize("max_iter", [13, 21])
def test_batched_stops_inside_a_block(orc, max_iter):
    """Multi-shift systems of a batch bring their shifted solutions up to date
    once per block of 16 iterations; a batch stopped by the iteration limit
    inside a block returns every system's iterates at that iteration (the
    oracle's, same limit).  A single-shift system (updated every iteration)
    rides in the same batch."""
    import torch
    import paper_1010_5433_amd as stag
    log(f"batched, stop at {max_iter}")
    specs = [((4, 4, 4, 4), 51, 0.1, [0.0, 0.05, 0.5], [7, 8]), ((6, 4, 2, 4), 52, 0.2, [0.01], [9])]
    lats, systems, host = _setup(specs)
    sols, rc, stats = stag.multishift_cg_batched(systems, prec="f64", max_iter=max_iter)
    torch.cuda.synchronize()
    assert rc == stag._abi.STAG_ENOCONV
    for k, (dims, U, mass, shifts, b) in enumerate(host):
        xo, rco, io = orc.multishift_cg(dims, U, mass, shifts, b, tol=1e-10, max_iter=max_iter)
        assert stats[k]["iters"] == io["iters"] == max_iter
        for i in range(len(shifts)):
            assert rel(unpack(systems[k]["lat"], sols[k][i]), xo[i]) <= 1e-12, (k, i)


def test_launch_shapes_agree():
    import torch
    import paper_1010_5433_amd as stag
    log("launch shapes")
    lats, systems, host = _setup(SMALL_BATCH)
    results = {}
    for rpt in (1, 2, 4, 8):
        for block in (64, 128, 256):
            sols, rc, stats = stag.multishift_cg_batched(systems, prec="f64", rpt=rpt, block=block)
            torch.cuda.synchronize()
            assert rc == 0
            assert stag.batch_last_config() == (block, rpt)
            results[(rpt, block)] = ([[x.clone() for x in s] for s in sols], [st["iters"] for st in stats])
    ref_sols, ref_its = results[(1, 256)]
    for key, (sols, its) in results.items():
        assert its == ref_its, key
        for a, b in zip(sols, ref_sols):
            for x, y in zip(a, b):
                d = float((x - y).abs().max()) / float(y.abs().max())
                assert d <= 1e-13, (key, d)
    # the autotuner picks one of the candidates
    stag.multishift_cg_batched(systems, prec="f64")
    block, rpt = stag.batch_last_config()
    assert block in (64, 128, 256) and rpt in (1, 2, 4, 8)


@pytest.mark.parametrize("prec", ["f64", "mixed"])
def test_repeated_calls_bit_identical(prec):
    """Graph replays against direct launches: a call that replays its
    captured block of 16 iterations (many replays per solve), one that
    launches every kernel, and a second replaying call, with eager work and
    synchronisations between them.  The reductions have a fixed order and
    the kernels are the same, so every result is equal bit for bit."""
    import torch
    import paper_1010_5433_amd as stag
    log(f"repeated batched calls prec={prec}")
    lats, systems, host = _setup(SMALL_BATCH)
    a, rca, sa = stag.multishift_cg_batched(systems, prec=prec, rpt=2, block=128)
    a = [[x.clone() for x in s] for s in a]
    junk = torch.randn(1 << 20, device="cuda").sum()
    torch.cuda.synchronize()
    b, rcb, sb = stag.multishift_cg_batched(systems, prec=prec, rpt=2, block=128, no_graph=True)
    b = [[x.clone() for x in s] for s in b]
    junk = junk + torch.randn(1 << 20, device="cuda").sum()
    torch.cuda.synchronize()
    c, rcc, sc = stag.multishift_cg_batched(systems, prec=prec, rpt=2, block=128)
    torch.cuda.synchronize()
    assert rca == rcb == rcc == 0
    for sa_, sb_, sc_ in zip(a, b, c):
        for x, y, z in zip(sa_, sb_, sc_):
            assert torch.equal(x, y) and torch.equal(x, z)
    assert [s["iters"] for s in sa] == [s["iters"] for s in sb]


@pytest.mark.parametrize("prec", ["f64", "mixed"])
def test_merged_launch_equals_per_lattice_launches(prec):
    """Three lattices of different sizes (one with three systems): the one
    multi-RHS launch per phase for all lattices, each group on its own range
    of workgroups, gives results bit-identical to one launch per lattice and
    group (same launch shape forced on both), with and without graphs."""
    import torch
    import paper_1010_5433_amd as stag
    log(f"merged vs per-lattice launches prec={prec}")
    lats, systems, host = _setup(SMALL_BATCH)
    runs = {}
    for name, kw in (("merged", {}), ("per_lattice", dict(per_lattice=True)),
                     ("merged_no_graph", dict(no_graph=True))):
        sols, rc, st = stag.multishift_cg_batched(systems, prec=prec, rpt=4, block=64, **kw)
        torch.cuda.synchronize()
        assert rc == 0, name
        runs[name] = ([[x.clone() for x in s] for s in sols], [t["iters"] for t in st])
    ref_sols, ref_its = runs["per_lattice"]
    for name, (sols, its) in runs.items():
        assert its == ref_its, name
        for a, b in zip(sols, ref_sols):
            for x, y in zip(a, b):
                assert torch.equal(x, y), name


def test_autotune_cache_file(tmp_path, monkeypatch):
    """STAG_AUTOTUNE_CACHE: a layout found in the file is used without
    timing; a layout timed in this process is appended to the file."""
    import torch
    import paper_1010_5433_amd as stag
    path = tmp_path / "shapes.txt"
    seeded = "f64 nrow3 6x6x6x6:2"
    path.write_text(f"garbage line\n{seeded}\t128\t2\n")
    monkeypatch.setenv("STAG_AUTOTUNE_CACHE", str(path))
    specs_seeded = [((6, 6, 6, 6), 44, 0.1, [0.0, 0.5], [7, 8])]
    _, systems, _ = _setup(specs_seeded)
    _, rc, _ = stag.multishift_cg_batched(systems, prec="f64")
    torch.cuda.synchronize()
    assert rc == 0 and stag.batch_last_config() == (128, 2)
    specs_new = [((6, 6, 4, 4), 45, 0.1, [0.0, 0.5], [9, 10, 11])]
    _, systems, _ = _setup(specs_new)
    _, rc, _ = stag.multishift_cg_batched(systems, prec="f64")
    torch.cuda.synchronize()
    assert rc == 0
    block, rpt = stag.batch_last_config()
    assert f"f64 nrow3 6x6x4x4:3\t{block}\t{rpt}" in path.read_text().splitlines()


def test_log_lines(capfd, monkeypatch):
    """STAG_LOG=1 prints one line per solve on stderr; unset, nothing."""
    import torch
    import paper_1010_5433_amd as stag
    _, systems, _ = _setup([((4, 4, 4, 4), 46, 0.1, [0.0, 0.3], [12])])
    y = systems[0]
    monkeypatch.setenv("STAG_LOG", "1")
    y["lat"].multishift_cg(y["mass"], y["shifts"], y["src"])
    torch.cuda.synchronize()
    err = capfd.readouterr().err
    assert "[stag] multishift_cg: 2 shifts, f64" in err
    monkeypatch.delenv("STAG_LOG")
    y["lat"].multishift_cg(y["mass"], y["shifts"], y["src"])
    torch.cuda.synchronize()
    assert "[stag]" not in capfd.readouterr().err


def test_batched_config4_full_size(orc):
    """8 pseudo-fermions x 16 shifts on 24^3x6 (m = 0.02) plus 8^4, 12^4 and
    16^3x8 (m = 0.05, 8 shifts each), FP32 with FP64 reliable updates and
    refinement, one batched call."""
    import torch
    import paper_1010_5433_amd as stag
    c = syn.config("c4_batched")
    log("config 4 batched")
    specs = []
    for y in c["systems"]:
        specs.append((y["dims"], y["links"][2], y["mass"], syn.logspace_shifts(*y["shifts"]),
                      list(y["source_seeds"])))
    lats, systems, host = _setup(specs)
    sols, rc, stats = stag.multishift_cg_batched(systems, prec="mixed")
    torch.cuda.synchronize()
    log(f"  seconds {stats[0]['seconds']:.3f} iters {[s['iters'] for s in stats]} "
        f"refine {[s['refine_iters'] for s in stats]} cfg {stag.batch_last_config()}")
    assert rc == 0
    for k, (dims, U, mass, shifts, b) in enumerate(host):
        assert max(stats[k]["resid_true"]) <= 1e-10
        lat = systems[k]["lat"]
        for i in (0, len(shifts) // 2, len(shifts) - 1):
            r = orc.true_residual(dims, U, mass, shifts[i], b, unpack(lat, sols[k][i]))
            assert r <= 1e-10, (k, i, r)


def test_batched_64_systems(orc):
    """The largest batch: 64 systems (two lattices, 8 groups of 8 on one of
    them), each against the oracle's operator; 65 are refused."""
    import torch
    import paper_1010_5433_amd as stag
    log("batched 64 systems")
    specs = [((4, 4, 4, 4), 61, 0.1, [0.0, 0.3], list(range(300, 348))),
             ((4, 2, 2, 4), 62, 0.2, [0.01], list(range(400, 416)))]
    lats, systems, host = _setup(specs)
    assert len(systems) == 64
    sols, rc, stats = stag.multishift_cg_batched(systems, prec="f64")
    torch.cuda.synchronize()
    assert rc == 0
    for k in (0, 17, 47, 48, 63):
        dims, U, mass, shifts, b = host[k]
        for i, s in enumerate(shifts):
            r = orc.true_residual(dims, U, mass, s, b, unpack(systems[k]["lat"], sols[k][i]))
            assert r <= 1e-10, (k, i, r)
            assert abs(stats[k]["resid_true"][i] - r) <= 1e-3 * r + 1e-16
    with pytest.raises(stag.StagError):
        stag.multishift_cg_batched(systems + systems[:1])


def test_batched_errors():
    import paper_1010_5433_amd as stag
    log("batched errors")
    lats, systems, host = _setup(SMALL_BATCH[:1])
    with pytest.raises(stag.StagError):
        stag.multishift_cg_batched(systems, rpt=3, block=64)
    bad = dict(systems[0])
    bad["mass"] = -1.0
    with pytest.raises(stag.StagError):
        stag.multishift_cg_batched([bad])
    sols, rc, st = stag.multishift_cg_batched(systems, max_iter=5)
    assert rc == stag._abi.STAG_ENOCONV
