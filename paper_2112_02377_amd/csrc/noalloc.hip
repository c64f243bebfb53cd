// jac_sweep_noalloc: the fixed-count sweeps of jac_sweep with every scratch
// buffer of the call taken from one static device array, so that the call
// allocates nothing (for callers that cannot allocate: code being captured
// into a HIP graph, tight serving loops, harnesses that forbid it).
//
// The scratch of a sweep loop is the system descriptor the kernels read, the
// loop's control state and the per-tile norm partials (two sweeps' worth);
// the handle still owns the matrix, b and the iterates, allocated when it was
// created and split.  Each device holds its own copy of the array, at its own
// address, for the life of the process; every call on a device shares it, so
// calls that overlap on one device race (run them on one stream, or one at a
// time).  What must start clean is rewritten by every call: the descriptor is
// stored by a kernel, the state by the state-initialising kernel, and every
// partial is written by its sweep before the next launch reads it.
#include <hip/hip_runtime.h>

#include <cstdint>
#include <mutex>

#include "handle.h"
#include "launch.h"

namespace jac {
namespace {

constexpr size_t kScratchBytes = size_t(1) << 20;    // 1 MiB per device
constexpr size_t kDescBytes = 768;                   // SysDev
constexpr size_t kStateOff = kDescBytes;             // SysState
constexpr size_t kPartOff = 1024;                    // [2][ntiles][nrhs] doubles
static_assert(sizeof(SysDev) <= kDescBytes, "descriptor slot too small");
static_assert(kStateOff + sizeof(SysState) <= kPartOff, "state slot too small");

static __device__ __align__(256) unsigned char scratch[kScratchBytes];

constexpr int kMaxDevices = 64;
std::mutex g_mutex;
void* g_ptr[kMaxDevices] = {};

// Device address of this device's copy of `scratch`, looked up once per
// device with that device current.  In host code the array's name is only a
// host-side stand-in, never a device address.
void* scratch_ptr(int dev)
{
    if (dev < 0 || dev >= kMaxDevices) fail(JAC_E_INVALID, "device ordinal out of range");
    std::lock_guard<std::mutex> lock(g_mutex);
    if (!g_ptr[dev]) {
        int cur = 0;
        JAC_HIP(hipGetDevice(&cur));
        if (cur != dev) JAC_HIP(hipSetDevice(dev));
        void* p = nullptr;
        const hipError_t e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
        if (cur != dev) JAC_HIP(hipSetDevice(cur));
        JAC_HIP(e);
        if (!p) fail(JAC_E_HIP, "no device address for the scratch array");
        g_ptr[dev] = p;
    }
    return g_ptr[dev];
}

// Stores the descriptor (passed by value in the kernel arguments).
__global__ void k_put_desc(SysDev s, SysDev* dst)
{
    if (threadIdx.x == 0) *dst = s;
}

}  // namespace
}  // namespace jac

using namespace jac;

extern "C" jac_status jac_sweep_noalloc(jac_handle h, int32_t nsweeps, double* hist_dev)
{
    return guarded([&]() -> jac_status {
        if (!h) fail(JAC_E_INVALID, "NULL handle");
        h->require_plan();
        if (nsweeps < 0) fail(JAC_E_INVALID, "nsweeps must be >= 0");
        const int64_t part_bytes = 2 * (int64_t)std::max(h->plan.ntiles, 1) * h->nrhs * (int64_t)sizeof(double);
        if ((int64_t)kPartOff + part_bytes > (int64_t)kScratchBytes)
            fail(JAC_E_INVALID, "jac_sweep_noalloc: the split's norm partials (" + std::to_string(part_bytes) +
                                    " bytes: 2 x tiles x right-hand sides doubles) exceed the " +
                                    std::to_string(kScratchBytes - kPartOff) +
                                    "-byte scratch; use larger tiles or jac_sweep");
        if (nsweeps == 0) return JAC_OK;
        unsigned char* base = static_cast<unsigned char*>(scratch_ptr(h->device));
        ++h->state_gen;
        hipStream_t st = h->stream;
        SysDev s = h->sysdev(false);
        s.tile_part = reinterpret_cast<double*>(base + kPartOff);
        SysDev* d_sys = reinterpret_cast<SysDev*>(base);
        SysState* d_state = reinterpret_cast<SysState*>(base + kStateOff);
        k_put_desc<<<1, 64, 0, st>>>(s, d_sys);
        JAC_HIP(hipGetLastError());
        launch_init_state(d_state, 1, st);
        LoopParams p{};
        p.sys = d_sys;
        p.st = d_state;
        p.tile_base = nullptr;      // one system: the per-launch loop reads no tile prefix
        p.hist = hist_dev;
        p.bar = nullptr;            // no grid barrier: one launch per sweep
        p.nsys = 1;
        p.k0 = 0;
        p.kend = nsweeps;
        p.solve = 0;
        p.norm_inf = 0;
        const int fpb = h->lds_fp_bytes(false), tab = h->lds_tab();
        void* fn = sweep_kernel(false, h->nrhs, h->plan.colfmt, 0, s.keep != 0);
        const size_t lds = loop_lds_bytes(fpb, tab, 0);
        const int grid = sweep_grid(*h, fn, h->opt.block, lds);
        h->last_grid = grid;
        h->last_loop_sweeps = nsweeps;
        for (int32_t k = 0; k < nsweeps; ++k) launch_sweep1(fn, grid, h->opt.block, lds, st, p, k, fpb, tab);
        launch_decide(h->nrhs, st, p, nsweeps - 1);
        uint32_t which = 0;
        for (int c = 0; c < h->nrhs; ++c) which |= (uint32_t)(nsweeps % 3) << (2 * c);
        h->settle(which);
        JAC_HIP(hipGetLastError());
        return JAC_OK;
    });
}
