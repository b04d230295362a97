"""Helpers shared by the GPU tests: input caching and host<->device moves."""
import functools

import numpy as np

import stag_synth as syn


@functools.lru_cache(maxsize=8)
def links_np(dims, kind="smooth", eps=0.5, seed=1):
    if kind == "haar":
        return syn.haar_links(dims, seed)
    return syn.smooth_links(dims, eps, seed)


def to_dev(a):
    import torch
    return torch.from_numpy(np.ascontiguousarray(a)).to("cuda")


def lattice_with_links(dims, links, fmt="18", antiperiodic=True):
    import paper_1010_5433_amd as stag
    lat = stag.Lattice(dims, antiperiodic)
    lat.set_links(to_dev(links), fmt)
    return lat


def pack(lat, v, prec="f64"):
    return lat.pack(to_dev(v), prec)


def unpack(lat, v):
    import torch
    torch.cuda.synchronize()
    return lat.unpack(v).cpu().numpy()


def rel(a, b):
    return float(np.linalg.norm(a - b) / max(np.linalg.norm(b), 1e-300))


def log(msg):
    print(msg, flush=True)
