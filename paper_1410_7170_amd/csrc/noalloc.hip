// (Q^2 + shift) in without a caller workspace and without any allocation:
// the intermediate field Q in lives in a file-scope device array of
// OVL_NOALLOC_SCRATCH_BYTES that every GPU the library runs on holds until
// the process ends.  For callers that cannot allocate device memory (code
// under HIP graph capture, tight serving loops).
//
// The array's name is a host-side stand-in in host code; its device address
// is taken once per device with hipGetSymbolAddress (on the first call on that
// device, with the device current) and only that address is used afterwards.
// All calls on one GPU share its array: calls that overlap on one GPU (other
// streams, other threads) race on it.  The kernels overwrite the whole part of
// the array they read, so nothing needs clearing between calls.
#include <mutex>

#include "internal.h"

namespace ovl {
int q2_apply_body(const ovl_lattice *lat, const ovl_gauge *U, double m0, double shift, const ovl_spinor *in,
                  ovl_spinor *out, char *ws, size_t ws_bytes, hipStream_t st);
}

namespace {

static __device__ __align__(256) unsigned char scratch[OVL_NOALLOC_SCRATCH_BYTES];

constexpr int kMaxDevices = 64;
std::mutex g_mu;
void *g_ptr[kMaxDevices];   // device address of `scratch` per device, once taken

// device address of this device's scratch array (taken on first use)
int scratch_ptr(void **out)
{
    int dev = -1;
    hipError_t e = hipGetDevice(&dev);
    if (e != hipSuccess) return ovl::hip_fail(e);
    if (dev < 0 || dev >= kMaxDevices) return OVL_ERR_INVALID;
    std::lock_guard<std::mutex> lk(g_mu);
    if (!g_ptr[dev]) {
        void *p = nullptr;
        e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
        if (e != hipSuccess) return ovl::hip_fail(e);
        if (!p) return OVL_ERR_HIP;
        g_ptr[dev] = p;
    }
    *out = g_ptr[dev];
    return OVL_OK;
}

}  // namespace

extern "C" {

int ovl_q2_apply_noalloc(const ovl_lattice *lat, const ovl_gauge *U, double m0, double shift, const ovl_spinor *in,
                         ovl_spinor *out, void *stream)
{
    // the size check first, so an oversized call fails before any device work
    if (!lat || !in) return OVL_ERR_INVALID;
    const size_t need = ovl_workspace_bytes(lat, OVL_OP_Q2, in->prec, in->nrhs, 0, nullptr);
    if (need == 0) return OVL_ERR_INVALID;
    if (need > OVL_NOALLOC_SCRATCH_BYTES) return OVL_ERR_WORKSPACE;
    void *p = nullptr;
    int rc = scratch_ptr(&p);
    if (rc) return rc;
    return ovl::q2_apply_body(lat, U, m0, shift, in, out, (char *)p, OVL_NOALLOC_SCRATCH_BYTES,
                              (hipStream_t)stream);
}

}  // extern "C"
