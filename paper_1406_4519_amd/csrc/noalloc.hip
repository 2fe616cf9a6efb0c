// noalloc.hip -- dfacto_mttkrp_noalloc: the MTTKRP for callers that cannot
// allocate device memory (code under HIP graph capture, tight serving loops,
// harnesses that forbid it).
//
// Its buffers -- the carries of split output rows and, for a tensor built
// with relabeled gathers, the factor tables permuted into rank order -- live
// in `scratch`, a fixed device array of kScratchBytes that every GPU the
// library runs on holds until the process ends.  In host code the array's
// name is only a stand-in, not a device address: the entry point looks up
// the array's address on each device once, with that device current, and
// passes that address to the kernels.  Every call on a GPU shares its
// array, so calls that overlap on one GPU (two streams, two threads) race;
// nothing in it needs to start at zero (each call writes every carry and
// table entry it reads).
#include <hip/hip_runtime.h>

#include <mutex>

#include "internal.hpp"

namespace {

constexpr size_t kScratchBytes = (size_t)64 << 20;
constexpr int kMaxDevices = 64;

static __device__ __align__(256) unsigned char scratch[kScratchBytes];

std::mutex g_mu;
void *g_ptr[kMaxDevices] = {};  // the array's address on each device

// The array's address on `device` (the current device), looked up once.
void *scratch_on(int device) {
    if (device < 0 || device >= kMaxDevices)
        throw dfacto::Error{DFACTO_E_UNSUPPORTED, "device index beyond the scratch table"};
    std::lock_guard<std::mutex> lk(g_mu);
    if (!g_ptr[device]) {
        void *p = nullptr;
        const hipError_t e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
        if (e != hipSuccess || !p) {
            (void)hipGetLastError();
            throw dfacto::Error{DFACTO_E_DEVICE, "the fixed scratch array has no device address"};
        }
        g_ptr[device] = p;
    }
    return g_ptr[device];
}

}  // namespace

using namespace dfacto;

extern "C" dfacto_status dfacto_mttkrp_noalloc(dfacto_ctx *ctx, const dfacto_tensor *t, int mode,
                                               int R, dfacto_dtype dtype,
                                               const void *const d_F[3], float *d_out) {
    return guarded(ctx, [&] {
        check_common(t, R, dtype);
        if (mode < 0 || mode > 2) throw Error{DFACTO_E_INVALID, "mode must be 0, 1 or 2"};
        if (!d_F || !d_out) throw Error{DFACTO_E_INVALID, "factor array or output is NULL"};
        const ModeData &md = t->mode[mode];
        if (!d_F[md.leaf] || !d_F[md.mid]) throw Error{DFACTO_E_INVALID, "factor is NULL"};
        if ((uintptr_t)d_F[md.leaf] % elem_size(dtype) || (uintptr_t)d_F[md.mid] % elem_size(dtype))
            throw Error{DFACTO_E_INVALID, "factor is not aligned to its element size"};
        if ((uintptr_t)d_out % 4) throw Error{DFACTO_E_INVALID, "output is not 4-byte aligned"};
        if (t->device != ctx->device)
            throw Error{DFACTO_E_INVALID, "tensor built on another device"};
        size_t carry_bytes = 0;
        const size_t perm = mttkrp_buffers(t, mode, R, dtype, &carry_bytes);
        if (carry_bytes + perm > kScratchBytes)
            throw Error{DFACTO_E_UNSUPPORTED,
                        "this MTTKRP needs " + std::to_string(carry_bytes + perm) +
                            " bytes of scratch; the fixed scratch holds " +
                            std::to_string(kScratchBytes)};
        char *base = (char *)scratch_on(ctx->device);  // ctx's device is current (guarded)
        launch_mttkrp_in(ctx, t, mode, R, dtype, d_F[md.leaf], d_F[md.mid], d_out,
                         (float *)base, perm ? base + carry_bytes : nullptr);
    });
}
