// lbm_step_noalloc: time steps of a caller-held state with no device
// allocation.  The spare distribution buffer, the density groups and the
// scalar planes of a step live in one file-scope device array, `scratch`,
// which every GPU the library runs on holds until the process ends.
#include <hip/hip_runtime.h>

#include <mutex>
#include <string>

#include "../../include/lbm.h"
#include "kernels.hpp"
#include "setup.hpp"

namespace {

// Largest mesh the allocation-free entry point takes (nx * ny nodes), and
// the planes of scratch it carves: the spare f (9), the density groups of
// both buffers (2 x 3), rho, the row part of mu, mu and F_y (4).
constexpr size_t kMaxNodes = LBM_NOALLOC_MAX_NODES;
constexpr size_t kPlaneBytes = kMaxNodes * sizeof(double);  // a multiple of 256
constexpr size_t kScratchPlanes = 9 + 6 + 4;
constexpr size_t kScratchBytes = kScratchPlanes * kPlaneBytes;
constexpr int kMaxDevices = 64;

}  // namespace

// 38 MiB per device.  In host code `scratch` names a host-side stand-in,
// not device memory: kernels receive the address hipGetSymbolAddress gives
// for the current device.
static __device__ __align__(256) unsigned char scratch[kScratchBytes];

namespace {

std::mutex g_scratch_mu;
void *g_scratch_ptr[kMaxDevices] = {};

size_t align256(size_t b) { return (b + 255) & ~size_t(255); }

lbm_status noalloc_fail(lbm_status s, const std::string &msg)
{
    cplbm::set_global_error(msg);
    return s;
}

// Device address of this device's copy of scratch (looked up once per
// device, with that device current).
hipError_t scratch_of_device(int dev, unsigned char **out)
{
    std::lock_guard<std::mutex> lock(g_scratch_mu);
    if (!g_scratch_ptr[dev]) {
        void *ptr = nullptr;
        hipError_t e = hipGetSymbolAddress(&ptr, HIP_SYMBOL(scratch));
        if (e != hipSuccess) return e;
        g_scratch_ptr[dev] = ptr;
    }
    *out = (unsigned char *)g_scratch_ptr[dev];
    return hipSuccess;
}

}  // namespace

extern "C" lbm_status lbm_step_noalloc(const lbm_params *p, double *f, int64_t nsteps,
                                       void *hip_stream)
{
    using namespace cplbm;
    KParams kp;
    std::string why;
    lbm_status st = setup_params(p, &kp, &why);
    if (st != LBM_OK) return noalloc_fail(st, why);
    const size_t N = (size_t)p->nx * p->ny;
    if (N > kMaxNodes)
        return noalloc_fail(LBM_E_INVALID, "lbm_step_noalloc takes meshes of at most " +
                                               std::to_string(kMaxNodes) + " nodes (got " +
                                               std::to_string(N) + ")");
    if (!f) return noalloc_fail(LBM_E_INVALID, "f is NULL");
    if (nsteps < 0) return noalloc_fail(LBM_E_INVALID, "nsteps must be >= 0");
    if (nsteps == 0) return LBM_OK;
    int dev = 0;
    hipError_t e = hipGetDevice(&dev);
    if (e == hipSuccess && (dev < 0 || dev >= kMaxDevices)) e = hipErrorInvalidDevice;
    unsigned char *base = nullptr;
    if (e == hipSuccess) e = scratch_of_device(dev, &base);
    if (e != hipSuccess)
        return noalloc_fail(LBM_E_DEVICE, std::string("scratch of the device: ") +
                                              hipGetErrorString(e));
    // carve the planes for this mesh
    const size_t plane = align256(N * sizeof(double));
    double *fs = (double *)base;
    double *g[2] = {(double *)(base + 9 * plane), (double *)(base + 12 * plane)};
    double *rho = (double *)(base + 15 * plane), *mux = (double *)(base + 16 * plane);
    double *mu = (double *)(base + 17 * plane), *fy = (double *)(base + 18 * plane);
    hipStream_t s = (hipStream_t)hip_stream;

    // the same sequence as lbm_step, the state alternating between the
    // caller's f and the spare buffer; the density groups of the caller's
    // state are formed first (everything in scratch is rewritten before it
    // is read, so nothing left by an earlier call is used)
    double *fb[2] = {f, fs};
    e = launch_density_groups(kp, f, g[0], s);
    int cur = 0;
    for (int64_t n = 0; n < nsteps && e == hipSuccess; ++n) {
        e = launch_rows_rho(kp, fb[cur], g[cur], rho, mux, s);
        if (e == hipSuccess) e = launch_cols_mu(kp, rho, mux, mu, fy, s);
        if (e == hipSuccess)
            e = launch_rows_collide(kp, fb[cur], mu, fy, fb[1 - cur], g[1 - cur], rho, s);
        cur = 1 - cur;
    }
    if (e == hipSuccess && cur == 1)
        e = hipMemcpyAsync(f, fs, 9 * N * sizeof(double), hipMemcpyDeviceToDevice, s);
    if (e != hipSuccess)
        return noalloc_fail(LBM_E_DEVICE, std::string("lbm_step_noalloc: ") + hipGetErrorString(e));
    return LBM_OK;
}
