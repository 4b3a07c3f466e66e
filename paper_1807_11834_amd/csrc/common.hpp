// common.hpp -- device helpers shared by the coupling kernels (gfx950, wave64).
#pragma once
#include <type_traits>
#include <hip/hip_runtime.h>
#include <stdint.h>

namespace cpl {

constexpr int kBlock = 256;          // threads per workgroup for every kernel
constexpr int kWave = 64;            // CDNA wavefront width
constexpr int kWavesPerBlock = kBlock / kWave;
constexpr double kPi = 3.14159265358979323846;

// Diagnostic partial-sum slots: each kernel writes one FP64 value per slot per
// workgroup; the final reduction sums every slot in a fixed order.
enum Slot {
    SL_VTOT = 0, SL_PHISUM = 1, SL_FP = 2, SL_FB = 5, SL_FF = 8, SL_EPSF = 11,
    SL_NCLAMP = 12, SL_NOUT = 13, SL_MAXPHI = 14, SL_NFALL = 15,
    SL_MLPERR = 16, SL_MLPREF = 17, SL_MLPSAMP = 18,
    SL_KP = 19, SL_KUP = 20, SL_KB = 23, SL_KUB = 24, SL_KF = 27, SL_KUF = 28, SL_COUNT = 31
};

template <typename T> struct V4;
template <> struct V4<float> { using type = float4; };
template <> struct V4<double> { using type = double4; };
template <typename T> using vec4 = typename V4<T>::type;

// Geometry constants of the nested grid pair in the working precision.
template <typename T> struct Geo {
    int nb[3];          // bulk cells per axis
    int nf[3];          // fine cells per axis
    int64_t ncell;      // bulk cells
    int64_t nfine;      // fine cells
    T L[3];             // box lengths
    T sb[3];            // nb / L (bulk cells per unit length)
    T sf[3];            // nf / L
    T hb[3];            // bulk spacing
    T inv_vb;           // 1 / V_b
    double vb, vf;      // cell volumes (FP64, for the diagnostics)
};

// How the per-cell sums of a step accumulate (the FP32 precision modes):
// plainly in the storage type, with Kahan compensation in the storage type, or
// plainly in FP64 registers (rounded to the storage type once per cell).  The
// FP64 mode sums plainly in FP64.
enum SumMode : int { kSumPlain = 0, kSumKahan = 1, kSumWide = 2 };

// Compensated (Kahan) or plain running sum.
template <typename T, bool KAHAN> struct Acc {
    T s = T(0), c = T(0);
    __device__ __forceinline__ void add(T v) {
        if constexpr (KAHAN) {
            T y = v - c;
            T t = s + y;
            c = (t - s) - y;
            s = t;
        } else {
            s += v;
        }
    }
};

// A per-cell sum of values of type T under mode SM.
template <typename T, int SM> struct CellSum {
    using W = typename std::conditional<SM == kSumWide, double, T>::type;
    Acc<W, SM == kSumKahan> acc;
    __device__ __forceinline__ void add(T v) { acc.add(W(v)); }
    __device__ __forceinline__ T value() const { return T(acc.s); }
};

// A running sum of products w v under mode SM: Kahan in T with the product
// formed by an FMA against the running compensation (each term rounded once),
// plain FMAs in T, or plain FMAs in FP64 registers (rounded to T once, by
// value()).  Only the Kahan mode carries the compensation word (arrays of these
// accumulators must stay in registers).
template <typename W, bool KAHAN> struct FmaState {
    W s = W(0);
};
template <typename W> struct FmaState<W, true> {
    W s = W(0);
    W c = W(0);
};
template <typename T, int SM>
struct FmaSum : FmaState<typename std::conditional<SM == kSumWide, double, T>::type, SM == kSumKahan> {
    using W = typename std::conditional<SM == kSumWide, double, T>::type;
    __device__ __forceinline__ void add(W w, W v) {
        if constexpr (SM == kSumKahan) {
            const W y = fma(w, v, -this->c);
            const W t = this->s + y;
            this->c = (t - this->s) - y;
            this->s = t;
        } else {
            this->s = fma(w, v, this->s);
        }
    }
    __device__ __forceinline__ T value() const { return T(this->s); }
};

template <typename T> __device__ __forceinline__ T tmin(T a, T b) { return a < b ? a : b; }
template <typename T> __device__ __forceinline__ T tmax(T a, T b) { return a > b ? a : b; }

__device__ __forceinline__ float dfloor(float x) { return floorf(x); }
__device__ __forceinline__ double dfloor(double x) { return floor(x); }
__device__ __forceinline__ float dsqrt(float x) { return sqrtf(x); }
__device__ __forceinline__ double dsqrt(double x) { return sqrt(x); }
__device__ __forceinline__ float dexp(float x) { return expf(x); }
__device__ __forceinline__ double dexp(double x) { return exp(x); }
__device__ __forceinline__ float dlog10(float x) { return log10f(x); }
__device__ __forceinline__ double dlog10(double x) { return log10(x); }
__device__ __forceinline__ float dpow(float x, float y) { return powf(x, y); }
__device__ __forceinline__ double dpow(double x, double y) { return pow(x, y); }
__device__ __forceinline__ float dfma(float a, float b, float c) { return fmaf(a, b, c); }
__device__ __forceinline__ double dfma(double a, double b, double c) { return fma(a, b, c); }

__device__ __forceinline__ int clampi(int v, int n) { return v < 0 ? 0 : (v > n - 1 ? n - 1 : v); }

// Coordinate clamped into [0, L]; a NaN becomes 0 (fmax returns the other operand).
template <typename T> __device__ __forceinline__ T clamp_coord(T x, T L, int &outside) {
    if (!(x >= T(0) && x <= L)) outside = 1;
    return fmin(fmax(x, T(0)), L);
}

// One-axis CIC stencil: lower node, fraction, clamped node pair.
template <typename T> struct Axis {
    int lo, hi;   // clamped node indices (equal when folded at a wall)
    T t;          // weight of `hi`; `lo` has 1 - t
};
template <typename T> __device__ __forceinline__ Axis<T> cic_axis(T x, T s, int n) {
    T g = x * s - T(0.5);
    T jf = dfloor(g);
    int j = (int)jf;
    Axis<T> a;
    a.t = g - jf;
    a.lo = clampi(j, n);
    a.hi = clampi(j + 1, n);
    return a;
}
// Weight of axis stencil `a` on node `c` (folded corners add up).
template <typename T> __device__ __forceinline__ T axis_weight(const Axis<T> &a, int c) {
    T w = T(0);
    if (a.lo == c) w += T(1) - a.t;
    if (a.hi == c) w += a.t;
    return w;
}

// Containing-cell index along one axis: floor(x * s), clamped; x = L -> n - 1.
template <typename T> __device__ __forceinline__ int cell_axis(T x, T s, int n) {
    return clampi((int)dfloor(x * s), n);
}

// Bulk pressure gradient at cell c: central differences, one-sided at the
// walls, taken in FP64 of the compensated pressure hi + lo (differencing the
// rounded hi alone would lose ulp(P)/h).
template <typename T>
__device__ __forceinline__ void gradient_at(int64_t c, int cx, int cy, int cz, const int nb[3], const T hb[3],
                                            const T *__restrict__ P, const T *__restrict__ Plo, T out[3]) {
    const int idx[3] = {cx, cy, cz};
    const int64_t stride[3] = {1, nb[0], (int64_t)nb[0] * nb[1]};
    auto pv = [&](int64_t k) { return (double)P[k] + (double)Plo[k]; };
    for (int a = 0; a < 3; ++a) {
        double gr;
        const int nax = nb[a];
        const double h = (double)hb[a];
        if (nax == 1) gr = 0.0;
        else if (idx[a] == 0) gr = (pv(c + stride[a]) - pv(c)) / h;
        else if (idx[a] == nax - 1) gr = (pv(c) - pv(c - stride[a])) / h;
        else gr = (pv(c + stride[a]) - pv(c - stride[a])) / (2.0 * h);
        out[a] = (T)gr;
    }
}

// Segment bounds read from `start` (a prefix sum over [0, n]) clamped into
// [0, n]: a no-op for a consistent `start`, it keeps every load in bounds.
__device__ __forceinline__ int32_t seg_clamp(int32_t v, int64_t n) { return v < 0 ? 0 : (v > n ? (int32_t)n : v); }

__device__ __forceinline__ void decode_cell(int64_t c, const int nb[3], int &cx, int &cy, int &cz) {
    cx = (int)(c % nb[0]);
    cy = (int)((c / nb[0]) % nb[1]);
    cz = (int)(c / ((int64_t)nb[0] * nb[1]));
}

// LDS written by some lanes of a wave and read by other lanes of the same wave:
// order the accesses without a workgroup barrier.
__device__ __forceinline__ void wave_sync() {
    __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
    __builtin_amdgcn_wave_barrier();
    __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
}

// Workgroup -> logical tile.  Workgroups are dealt round-robin over the 8 XCDs
// (each with its own L2).  XCD x takes chunks of kXcdChunk consecutive tiles,
// and the chunks of the 8 XCDs interleave over the domain: neighbouring tiles
// share an L2, while a dense region (the packed bed) is spread over all XCDs.
// The final partial round of chunks keeps the identity mapping (a bijection).
constexpr int64_t kXcdChunk = 16;
__device__ __forceinline__ int64_t xcd_tile(int64_t b, int64_t nblk) {
    const int64_t nx = 8, round = nx * kXcdChunk;
    const int64_t full = (nblk / round) * round;
    if (b >= full) return b;
    const int64_t x = b % nx, k = b / nx;          // k-th workgroup dealt to XCD x
    const int64_t q = k / kXcdChunk, r = k % kXcdChunk;
    return (q * nx + x) * kXcdChunk + r;
}

// ---- wave / block reductions (fixed tree order -> deterministic) -----------
__device__ __forceinline__ double wave_sum(double v) {
    for (int o = kWave / 2; o > 0; o >>= 1) v += __shfl_xor(v, o, kWave);
    return v;
}
__device__ __forceinline__ double wave_max(double v) {
    for (int o = kWave / 2; o > 0; o >>= 1) v = fmax(v, __shfl_xor(v, o, kWave));
    return v;
}

// Block-wide sum of one double per thread; every thread receives the total.
__device__ __forceinline__ double block_sum(double v, double *lds /*[kWavesPerBlock]*/) {
    v = wave_sum(v);
    int lane = threadIdx.x % kWave, w = threadIdx.x / kWave;
    __syncthreads();
    if (lane == 0) lds[w] = v;
    __syncthreads();
    double t = 0.0;
    for (int i = 0; i < kWavesPerBlock; ++i) t += lds[i];
    return t;
}
__device__ __forceinline__ double block_max(double v, double *lds) {
    v = wave_max(v);
    int lane = threadIdx.x % kWave, w = threadIdx.x / kWave;
    __syncthreads();
    if (lane == 0) lds[w] = v;
    __syncthreads();
    double t = lds[0];
    for (int i = 1; i < kWavesPerBlock; ++i) t = fmax(t, lds[i]);
    return t;
}

}  // namespace cpl
