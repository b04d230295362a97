"""The allocation-free normal operator (stag_normal_op_noalloc) against
stag_normal_op: the same kernels on the same inputs, so the results must be
bit-identical.  Two calls in a row, the second on a smaller lattice (the
static scratch keeps the first call's contents), and a lattice too large for
the scratch, which the host rejects before any device work."""
import ctypes

import numpy as np
import pytest

from tests.gpu_common import links_np, log, pack, to_dev
import stag_synth as syn

pytestmark = pytest.mark.gpu


def _lattice(dims, fmt, seed):
    import paper_1010_5433_amd as stag
    lat = stag.Lattice(dims)
    lat.set_links(to_dev(links_np(dims, "smooth", 0.5, seed)), fmt)
    return lat


def test_noalloc_matches_normal_op_on_two_calls():
    import torch
    import paper_1010_5433_amd as stag
    assert stag._L.stag_noalloc_scratch_bytes() == 32 << 20
    cases = [((16, 16, 16, 16), "8", "f64", 0.01, 1e-3, 31),
             ((4, 4, 4, 6), "18", "f64", 0.1, 0.0, 32),
             ((8, 6, 4, 10), "12", "f32", 0.05, 0.25, 33)]
    for n, (dims, fmt, prec, mass, shift, seed) in enumerate(cases):
        log(f"noalloc case {n}: dims={dims} fmt={fmt} prec={prec}")
        lat = _lattice(dims, fmt, seed)
        v = pack(lat, syn.gaussian_source(dims, seed + 100), prec)
        got = torch.empty_like(v)
        ref = torch.empty_like(v)
        torch.cuda.synchronize()
        free0 = torch.cuda.mem_get_info()[0]
        lat.normal_op_noalloc(mass, shift, v, got)
        torch.cuda.synchronize()
        free1 = torch.cuda.mem_get_info()[0]
        if n > 0:
            # the scratch was set up by the first call: later calls allocate nothing
            assert free1 == free0, (free0, free1)
        lat.normal_op(mass, shift, v, ref)
        torch.cuda.synchronize()
        g, r = got.cpu().numpy(), ref.cpu().numpy()
        assert np.isfinite(r).all()
        assert np.array_equal(g, r), float(np.max(np.abs(g - r)))
        lat.close()


def test_noalloc_rejects_a_lattice_beyond_the_scratch():
    import torch
    import paper_1010_5433_amd as stag
    from paper_1010_5433_amd._abi import STAG_EINVAL, F64, F32
    # 48^4: the odd temporary is 127 MB (F64) or 63.7 MB (F32); no links are set,
    # so the size check must come first
    lat = stag.Lattice((48, 48, 48, 48))
    dummy = torch.empty(16, dtype=torch.float64, device="cuda")
    for prec in (F64, F32):
        rc = stag._L.stag_normal_op_noalloc(lat._h, 0.1, 0.0, ctypes.c_void_p(dummy.data_ptr()),
                                            ctypes.c_void_p(dummy.data_ptr() + 64), prec, None)
        assert rc == STAG_EINVAL
        assert b"static scratch" in stag._L.stag_last_error()
    lat.close()
