// The normal operator without any device allocation: the odd-site
// temporary D_oe in lives in a file-scope device array instead of a work
// buffer of the lattice handle.  For callers that cannot allocate device
// memory (code under graph capture, tight serving loops).
//
// Every GPU the library runs on holds one copy of the array for the rest of
// the process; its device address is looked up once per device with
// hipGetSymbolAddress, with that device current, and only that address is
// ever handed to kernels (in host code the array's name is not a device
// address).  All calls on one GPU share the array: calls that overlap in
// time on one GPU (two streams, two host threads) race on it.
#include <cmath>
#include <cstring>
#include <mutex>
#include <string>

#include "internal.h"

namespace stag {

// 32 MiB: the double precision odd temporary of a 32^4 lattice (25.2 MB)
// fits, and single precision up to twice the volume.
constexpr size_t kNoAllocScratchBytes = size_t(32) << 20;

static __device__ __align__(256) char scratch[kNoAllocScratchBytes];

constexpr int kMaxDevices = 64;
static void *g_scratch_ptr[kMaxDevices];
static std::mutex g_scratch_mutex;

// Device address of this device's copy of the array (current device).
static stag_status scratch_address(int dev, void **out) {
    if (dev < 0 || dev >= kMaxDevices) return invalid("device index out of range for the static scratch table");
    std::lock_guard<std::mutex> lock(g_scratch_mutex);
    if (!g_scratch_ptr[dev]) {
        void *p = nullptr;
        STAG_HIP(hipGetSymbolAddress(&p, HIP_SYMBOL(scratch)));
        if (!p) return invalid("hipGetSymbolAddress returned no address for the static scratch");
        g_scratch_ptr[dev] = p;
    }
    *out = g_scratch_ptr[dev];
    return STAG_OK;
}

}  // namespace stag

using namespace stag;

extern "C" {

size_t stag_noalloc_scratch_bytes(void) { return kNoAllocScratchBytes; }

stag_status stag_normal_op_noalloc(stag_lattice *lat, double mass, double shift, const void *in, void *out,
                                   stag_prec prec, void *stream) {
    if (!lat) return invalid("null lattice handle");
    if (!in || !out) return invalid("null vector");
    if (!(mass > 0) || !std::isfinite(mass)) return invalid("mass must be > 0");
    if (!(shift >= 0) || !std::isfinite(shift)) return invalid("shift must be >= 0");
    if (prec != STAG_F64 && prec != STAG_F32) return invalid("precision must be STAG_F64 or STAG_F32");
    const bool dbl = prec == STAG_F64;
    const size_t need = (size_t)vec_bytes(lat, dbl);
    if (need > kNoAllocScratchBytes)
        return invalid("stag_normal_op_noalloc: the odd temporary needs " + std::to_string(need) +
                       " bytes, more than the " + std::to_string(kNoAllocScratchBytes) +
                       "-byte static scratch (use stag_normal_op)");
    if (!lat->nrow) return invalid("links not set (call stag_links_set first)");
    int dev = -1;
    STAG_HIP(hipGetDevice(&dev));
    if (dev != lat->device) {
        STAG_HIP(hipSetDevice(lat->device));
        dev = lat->device;
    }
    if (ranges_overlap({in, need}, {out, need})) return invalid("in and out must not overlap");
    void *t = nullptr;
    STAG_TRY(scratch_address(dev, &t));
    hipStream_t s = static_cast<hipStream_t>(stream);
    DslashArgs a;
    std::memset(&a, 0, sizeof(a));
    a.g = lat->g;
    a.links = dbl ? lat->links64 : lat->links32;
    a.link_cache = lat->link_cache;
    a.out_parity = 1;
    a.in = in;
    a.out = t;
    STAG_HIP(launch_dslash(dbl, lat->nrow, DS_PLAIN, a, s));
    a.out_parity = 0;
    a.in = t;
    a.out = out;
    a.aux = in;
    a.c = mass * mass + shift;
    STAG_HIP(launch_dslash(dbl, lat->nrow, DS_NORMAL, a, s));
    return STAG_OK;
}

}  // extern "C"
