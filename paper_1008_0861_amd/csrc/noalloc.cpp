// asd_step_semi_implicit_noalloc: the semi-implicit step loop of
// asd_step_semi_implicit for callers that cannot allocate device memory
// (code under stream capture, tight serving loops).  Its scratch - the
// intermediate state T*, the face coefficients, the reduction slots and the
// status word - lives in one file-scope device array, `scratch`, of
// kNoallocScratchBytes; each GPU the library runs on holds its own copy
// until the process ends.  The kernels are those of the workspace path, and
// the steps are launched directly (no graph is instantiated).
#include <hip/hip_runtime.h>

#include <mutex>

#include "../../include/asd.h"
#include "asd_internal.h"

using namespace asd;

static constexpr size_t kNoallocScratchBytes = (size_t)64 << 20;
static constexpr int kNoallocMaxDevices = 64;

static __device__ __align__(256) unsigned char scratch[kNoallocScratchBytes];

// Device address of `scratch` on each device, taken once per device with
// that device current (the array's name is only a host-side stand-in).
static std::mutex g_scratch_mu;
static void* g_scratch_ptr[kNoallocMaxDevices] = {};

static int scratch_on_current_device(void** out) {
    int dev = -1;
    hipError_t e = hipGetDevice(&dev);
    if (e != hipSuccess) return asd_fail(ASD_EHIP, "hipGetDevice: %s", hipGetErrorString(e));
    if (dev < 0 || dev >= kNoallocMaxDevices) return asd_fail(ASD_EUNSUPPORTED, "device %d out of range", dev);
    std::lock_guard<std::mutex> lock(g_scratch_mu);
    if (!g_scratch_ptr[dev]) {
        void* p = nullptr;
        e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
        if (e != hipSuccess || !p)
            return asd_fail(ASD_EHIP, "hipGetSymbolAddress(scratch): %s", hipGetErrorString(e));
        g_scratch_ptr[dev] = p;
    }
    *out = g_scratch_ptr[dev];
    return ASD_OK;
}

extern "C" size_t asd_noalloc_scratch_bytes(void) { return kNoallocScratchBytes; }

extern "C" int asd_step_semi_implicit_noalloc(const asd_desc* desc, void* dev_T, const void* dev_bx,
                                              const void* dev_by, const void* dev_bz, const void* dev_chi,
                                              double dt, int32_t nsteps, double* dev_energy, void* stream) {
    // all validation before any HIP call
    int rc = validate_desc(desc);
    if (rc) return rc;
    if (!dev_T || !dev_bx || !dev_by) return asd_fail(ASD_EINVAL, "T, bx and by must not be NULL");
    if (desc->ndim == 3 && !dev_bz) return asd_fail(ASD_EINVAL, "bz must not be NULL in 3-D");
    if ((desc->flags & ASD_FLAG_PER_CELL_CHI) && !dev_chi)
        return asd_fail(ASD_EINVAL, "chi must not be NULL with ASD_FLAG_PER_CELL_CHI");
    if (nsteps < 0) return asd_fail(ASD_EINVAL, "nsteps must be >= 0");
    const size_t need = grid_workspace_bytes(desc);
    if (need > kNoallocScratchBytes)
        return asd_fail(ASD_EUNSUPPORTED, "this grid needs %zu bytes of scratch; the static scratch holds %zu",
                        need, kNoallocScratchBytes);
    // the handle lives on the stack: nothing is allocated, host or device
    asd_grid_s g;
    g.d = *desc;
    rc = check_dt(&g, dt, false);
    if (rc) return rc;
    void* ws = nullptr;
    rc = scratch_on_current_device(&ws);
    if (rc) return rc;
    rc = init_grid_in_place(&g, desc, ws, kNoallocScratchBytes, stream);
    if (rc) return rc;
    g.graph_mode = ASD_GRAPHS_OFF;
    g.T = dev_T;
    g.b[0] = const_cast<void*>(dev_bx);
    g.b[1] = const_cast<void*>(dev_by);
    if (desc->ndim == 3) g.b[2] = const_cast<void*>(dev_bz);
    if (desc->flags & ASD_FLAG_PER_CELL_CHI) g.chi = const_cast<void*>(dev_chi);
    // face coefficients for dt and a cleared status word, then the steps
    rc = prepare(&g, dt);
    if (rc) return rc;
    StepOut o;
    o.energy = dev_energy;
    return enqueue_si_loop(&g, dt, nsteps, o);
}
