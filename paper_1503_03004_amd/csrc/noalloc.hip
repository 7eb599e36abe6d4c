// sfr_solve_noalloc: FR-ADM (Alg. 1 with the Alg. 2 L-step) for callers that
// cannot allocate device memory (code under graph capture, tight serving
// loops, hosts that forbid hipMalloc).  It runs the same engine and kernels
// as sfr_create + sfr_solve, with the whole device workspace carved from a
// file-scope array, `scratch`, and no pinned host memory or HIP events:
// progress is read back into per-device host mirrors in this file and
// waited for by synchronising the caller's stream.
//
// Each device holds its own copy of `scratch` for the life of the process.
// Its device address is taken once per device with hipGetSymbolAddress
// (with that device current) and kept in `g_dev`; host code uses only that
// address, never the array's name.  Every call on one device shares that
// device's array and host mirrors, so calls that overlap on one device race.
#include "engine.hpp"

#include <string.h>

#include <algorithm>
#include <mutex>

namespace sfr {
namespace {

constexpr size_t kScratchBytes = size_t(128) << 20;   // 128 MiB per device
constexpr size_t kScratchAlign = 256;
constexpr int kMaxDevices = 16;

static __device__ __align__(256) unsigned char scratch[kScratchBytes];

struct NoAllocDevice {
    unsigned char* ptr;        // device address of this device's `scratch`
    DevState host_state;       // readback of the solver state
    DevState host_poll[2];     // progress snapshots of a tolerance-driven solve
};

NoAllocDevice g_dev[kMaxDevices];
std::mutex g_mu;

// The device address of the current device's scratch (nullptr on error).
NoAllocDevice* device_slot()
{
    int dev = -1;
    if (hipGetDevice(&dev) != hipSuccess || dev < 0 || dev >= kMaxDevices) {
        (void)hipGetLastError();
        return nullptr;
    }
    std::lock_guard<std::mutex> lock(g_mu);
    NoAllocDevice& d = g_dev[dev];
    if (!d.ptr) {
        void* p = nullptr;
        if (hipGetSymbolAddress(&p, HIP_SYMBOL(scratch)) != hipSuccess || !p) {
            (void)hipGetLastError();
            return nullptr;
        }
        d.ptr = static_cast<unsigned char*>(p);
    }
    return &d;
}

}  // namespace
}  // namespace sfr

using namespace sfr;

extern "C" sfr_status sfr_solve_noalloc(int64_t m, int64_t n, int32_t r, double lambda, double mu, double tol,
                                        const sfr_options* opt, const void* M, int64_t ldm, void* U, double* B,
                                        void* V, void* S, int64_t lds, sfr_info* info, void* hip_stream)
{
    sfr_options o;
    const sfr_status vs = validate_create(m, n, r, lambda, mu, tol, opt, o);
    if (vs != SFR_OK) return vs;
    // FR-Nys keeps a second stream and host thread; profiling creates events;
    // the large-rank engine (r > 32) owns its own workspace
    if (o.nystrom_l != 0 || o.profile != 0 || r > kMaxR) return SFR_ERR_ARG;
    if (!M || !U || !B || !V) return SFR_ERR_ARG;
    if (ldm < n || (S && lds < n)) return SFR_ERR_ARG;
    Params prm;
    params_from(o, lambda, mu, tol, prm);
    const bool f64 = (o.precision == SFR_F64);
    const int hist = std::max(o.max_iter, o.fixed_iters);
    Engine e;
    sfr_status ps = engine_plan(e, (int)m, (int)n, r, f64, hist);
    if (ps != SFR_OK) return ps;
    if (prm.bf16 && !e.cfg[1].mfma) return SFR_ERR_ARG;
    // M is read in place when the sweeps can take it as it is, as in
    // engine_iterate; otherwise the padded copy is part of the workspace
    const bool aligned = ((uintptr_t)M % 16 == 0) && (ldm % e.vec == 0) && (e.ne == e.n);
    size_t need = 0;
    (void)engine_buffers(e, !aligned, [&](size_t sz) -> void* {
        need = (need + kScratchAlign - 1) / kScratchAlign * kScratchAlign + sz;
        return reinterpret_cast<void*>(kScratchAlign);   // placeholder, never dereferenced
    });
    if (need > kScratchBytes) return SFR_ERR_SCRATCH;
    NoAllocDevice* d = device_slot();
    if (!d) return SFR_ERR_DEVICE;
    size_t off = 0;
    const bool ok = engine_buffers(e, !aligned, [&](size_t sz) -> void* {
        off = (off + kScratchAlign - 1) / kScratchAlign * kScratchAlign;
        void* p = d->ptr + off;
        off += sz;
        return p;
    });
    if (!ok || off > kScratchBytes) return SFR_ERR_SCRATCH;
    e.host_state = &d->host_state;
    e.host_poll = d->host_poll;
    const bool mu_auto = !(mu > 0.0);
    return engine_solve(e, prm, mu_auto, M, ldm, U, B, V, S, lds, info, static_cast<hipStream_t>(hip_stream));
}
