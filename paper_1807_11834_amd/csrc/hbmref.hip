// hbmref.hip -- streaming reference kernels (read, write, copy), the practical
// HBM ceiling the coupling kernels are measured against (include/couple_hbmref.h).
// One 16-byte element per thread and one workgroup per 256 elements: on this
// chip these single-access threads stream faster than grid-stride loops or
// several accesses per thread; the loads are non-temporal (nothing reads the
// data again), the stores plain (faster here than non-temporal ones).  The read
// writes nothing unless it finds a non-finite value: per-wave or per-workgroup
// results written to neighbouring addresses cost it a fifth of its rate.
#include <hip/hip_runtime.h>

#include <cstdint>

#include "couple_hbmref.h"

namespace {

typedef float f4 __attribute__((ext_vector_type(4)));
constexpr int kRefBlock = 256;
constexpr int kRefWave = 64;

// A scan for non-finite values: x - x is 0 for a finite x and NaN otherwise,
// so a wave writes only when it holds one (the pass is a pure read stream).
__global__ __launch_bounds__(kRefBlock) void k_ref_read(const f4 *__restrict__ src, int64_t n,
                                                        int32_t *__restrict__ flag) {
    const int64_t i = (int64_t)blockIdx.x * kRefBlock + threadIdx.x;
    bool bad = false;
    if (i < n) {
        const f4 v = __builtin_nontemporal_load(src + i);
        const f4 z = v - v;
        bad = !(z.x == 0.f && z.y == 0.f && z.z == 0.f && z.w == 0.f);
    }
    if (__any(bad) && threadIdx.x % kRefWave == 0) *flag = 1;
}

__global__ __launch_bounds__(kRefBlock) void k_ref_write(f4 *__restrict__ dst, int64_t n, float value) {
    const int64_t i = (int64_t)blockIdx.x * kRefBlock + threadIdx.x;
    if (i < n) dst[i] = f4{value, value, value, value};
}

__global__ __launch_bounds__(kRefBlock) void k_ref_copy(const f4 *__restrict__ src, f4 *__restrict__ dst,
                                                        int64_t n) {
    const int64_t i = (int64_t)blockIdx.x * kRefBlock + threadIdx.x;
    if (i < n) dst[i] = __builtin_nontemporal_load(src + i);
}

bool aligned16(const void *p) { return (reinterpret_cast<uintptr_t>(p) & 15u) == 0; }

}  // namespace

extern "C" int couple_hbmref(int kind, const void *src, void *dst, int64_t n16, float value, void *stream) {
    if (kind < COUPLE_HBMREF_READ || kind > COUPLE_HBMREF_COPY || n16 < 0) return COUPLE_EINVAL;
    if (n16 == 0) return COUPLE_OK;
    const bool need_src = kind != COUPLE_HBMREF_WRITE;
    if (!dst || (need_src && !src)) return COUPLE_EINVAL;
    if ((kind != COUPLE_HBMREF_READ && !aligned16(dst)) || (need_src && !aligned16(src)) ||
        (kind == COUPLE_HBMREF_READ && (reinterpret_cast<uintptr_t>(dst) & 3u)))
        return COUPLE_EINVAL;
    const int64_t blocks = (n16 + kRefBlock - 1) / kRefBlock;
    if (blocks > 0x7fffffffLL) return COUPLE_EINVAL;
    hipStream_t st = static_cast<hipStream_t>(stream);
    switch (kind) {
    case COUPLE_HBMREF_READ:
        hipLaunchKernelGGL(k_ref_read, dim3((unsigned)blocks), dim3(kRefBlock), 0, st,
                           static_cast<const f4 *>(src), n16, static_cast<int32_t *>(dst));
        break;
    case COUPLE_HBMREF_WRITE:
        hipLaunchKernelGGL(k_ref_write, dim3((unsigned)blocks), dim3(kRefBlock), 0, st, static_cast<f4 *>(dst), n16,
                           value);
        break;
    default:
        hipLaunchKernelGGL(k_ref_copy, dim3((unsigned)blocks), dim3(kRefBlock), 0, st,
                           static_cast<const f4 *>(src), static_cast<f4 *>(dst), n16);
        break;
    }
    return hipGetLastError() == hipSuccess ? COUPLE_OK : COUPLE_EHIP;
}
