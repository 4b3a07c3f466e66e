// stages.hip -- restriction, particle sampling, drag, prolongation and the FP64
// conservation sums of one coupling step (deposition is in deposit.hip).
//
// Kernel order on the caller's stream (after binning/sorting, sort.hip):
//
//   k_gather       sorted copy sp = (x, y, z, d) of the particles: the packed
//                  input-order copy that binning wrote (clamped into the box),
//                  permuted, one 16-byte (FP32) read per particle.
//   deposit phi    (deposit.hip)
//   k_restrict     one thread per bulk cell streams its r^3 fine children of
//                  u, v, w, p (one 16-byte row load per (z, y) child row for
//                  r = 4) and writes the compensated averages U, P.
//   k_restrict_brick  the same restriction tiled in 8x4x2-cell bricks with the
//                  fine-grid lookup fused: the brick's fine u, v, w stay in LDS
//                  and its particles are sampled from there (fine trilinear
//                  velocity, void fraction from a haloed copy of phi), so the
//                  fine lookup costs no extra pass over the fine grid.
//   k_sample       the same sampling for the bulk and given velocity sources.
//   k_restrict_alpha  two-fluid drag: bulk liquid fraction, average of the fine
//                  children; k_pack_alpha8 then stores each cell's 2x2x2
//                  stencil corners as one record for the drag's lookups.
//   k_drag         drag and explicit Euler advection in input order (coalesced);
//                  with the semi-implicit split also (beta, beta u_p).
//   deposit force  (deposit.hip), with the bulk pressure gradient; then the
//                  semi-implicit K, KU when requested.
//   k_prolong      one thread per bulk cell writes its r^3 fine children of
//                  eps and F_fpi (a second launch: K and KU): conservative
//                  trilinear T_f + D_c with the 27-neighbour values in registers.
//   k_diag         fixed-order reduction of the per-workgroup FP64 partials.
#include <type_traits>

#include "common.hpp"
#include "launch.hpp"
#include "sample.hpp"

namespace cpl {

// ---------------------------------------------------------------------------
// Row loads of R consecutive fine values (16-byte vector loads where possible)
// ---------------------------------------------------------------------------
template <typename T, int R> struct Row { T v[R]; };

template <typename T, int N> using NtVec = T __attribute__((ext_vector_type(N)));

// STREAM: non-temporal loads, for fine rows that no later kernel of the step
// reads again (k_restrict, k_restrict_alpha); the brick kernel's rows use
// ordinary loads, since the stencils of its particles near a brick face read
// the neighbouring bricks' rows from the cache.
template <typename T, int N, bool STREAM> __device__ __forceinline__ NtVec<T, N> load_vec(const T *__restrict__ p) {
    const NtVec<T, N> *q = reinterpret_cast<const NtVec<T, N> *>(p);
    if constexpr (STREAM) return __builtin_nontemporal_load(q);
    else return *q;
}

template <typename T, int R, bool STREAM = false>
__device__ __forceinline__ Row<T, R> load_row(const T *__restrict__ p) {
    Row<T, R> r;
    if constexpr (std::is_same<T, float>::value && R == 4) {
        const NtVec<float, 4> q = load_vec<float, 4, STREAM>(p);
        r.v[0] = q.x; r.v[1] = q.y; r.v[2] = q.z; r.v[3] = q.w;
    } else if constexpr (std::is_same<T, float>::value && R == 2) {
        const NtVec<float, 2> q = load_vec<float, 2, STREAM>(p);
        r.v[0] = q.x; r.v[1] = q.y;
    } else if constexpr (std::is_same<T, double>::value && R == 4) {
        const NtVec<double, 2> a = load_vec<double, 2, STREAM>(p), b = load_vec<double, 2, STREAM>(p + 2);
        r.v[0] = a.x; r.v[1] = a.y; r.v[2] = b.x; r.v[3] = b.y;
    } else if constexpr (std::is_same<T, double>::value && R == 2) {
        const NtVec<double, 2> a = load_vec<double, 2, STREAM>(p);
        r.v[0] = a.x; r.v[1] = a.y;
    } else {
        for (int k = 0; k < R; ++k) r.v[k] = p[k];
    }
    return r;
}

// Fine-grid rows written once and not read again in the step: non-temporal
// stores, so that the 4 GB written per prolongation do not sit dirty in the
// caches and slow the next kernels while they are written back.
template <typename T, int R> __device__ __forceinline__ void store_row(T *__restrict__ p, const T *v) {
    if constexpr (std::is_same<T, float>::value && R == 4) {
        const NtVec<float, 4> q = {v[0], v[1], v[2], v[3]};
        __builtin_nontemporal_store(q, reinterpret_cast<NtVec<float, 4> *>(p));
    } else if constexpr (std::is_same<T, float>::value && R == 2) {
        const NtVec<float, 2> q = {v[0], v[1]};
        __builtin_nontemporal_store(q, reinterpret_cast<NtVec<float, 2> *>(p));
    } else if constexpr (std::is_same<T, double>::value && R == 4) {
        const NtVec<double, 2> q0 = {v[0], v[1]}, q1 = {v[2], v[3]};
        __builtin_nontemporal_store(q0, reinterpret_cast<NtVec<double, 2> *>(p));
        __builtin_nontemporal_store(q1, reinterpret_cast<NtVec<double, 2> *>(p) + 1);
    } else if constexpr (std::is_same<T, double>::value && R == 2) {
        const NtVec<double, 2> q = {v[0], v[1]};
        __builtin_nontemporal_store(q, reinterpret_cast<NtVec<double, 2> *>(p));
    } else {
        for (int k = 0; k < R; ++k) __builtin_nontemporal_store(v[k], p + k);
    }
}

// ---------------------------------------------------------------------------
// k_gather: sorted particle copies
// ---------------------------------------------------------------------------
template <typename T>
__global__ __launch_bounds__(kBlock) void k_gather(const int32_t *__restrict__ perm, const vec4<T> *__restrict__ pk,
                                                   int64_t n, vec4<T> *__restrict__ sp) {
    const int64_t i = (int64_t)blockIdx.x * kBlock + threadIdx.x;
    if (i < n) {
        int64_t p = perm[i];
        if (p < 0 || p >= n) p = 0;   // perm is a permutation of [0, n); guards the load
        sp[i] = pk[p];
    }
}

// ---------------------------------------------------------------------------
// Particle stage: void fraction and fluid velocity at the particle, drag
// (Eq. DragLaw with the Di Felice voidage function), optional Euler advection.
// ---------------------------------------------------------------------------
// Per particle in the sorted order: sample_one() with the handle's velocity
// source, written to uf4[id] = (u, v, w, eps_p) for the input-order drag kernel.
// KB particles per thread are sampled together so that all their gathers are in
// flight at once.
template <typename T, int KB>
__device__ __forceinline__ void sample_particles(const int64_t (&idx)[KB], const StepArgs<T> &a) {
    const vec4<T> *__restrict__ sp = a.sp;
    const int32_t *__restrict__ perm = a.perm;
    vec4<T> q[KB];
    int64_t p[KB];
#pragma unroll
    for (int k = 0; k < KB; ++k) {
        const int64_t i = idx[k] >= 0 ? idx[k] : 0;
        q[k] = sp[i];
        p[k] = perm[i];
        if (p[k] < 0 || p[k] >= a.n) p[k] = 0;   // perm is a permutation of [0, n)
    }
    vec4<T> s[KB];
#pragma unroll
    for (int k = 0; k < KB; ++k) s[k] = sample_one(q[k], a, a.vel_source);
#pragma unroll
    for (int k = 0; k < KB; ++k)
        if (idx[k] >= 0) a.uf4[p[k]] = s[k];
}

// ---------------------------------------------------------------------------
// Restriction fine -> bulk
// ---------------------------------------------------------------------------
// Sums of the r^3 fine children, per fine child plane and then the planes in
// order, under the step's sum mode.  Kahan (FP32): each plane is a Kahan sum and
// the planes are combined as s_0, -c_0, s_1, -c_1, ... in a Kahan sum; the
// average's residue lo = -c / r^3 carries the rest of the pressure for the
// gradient.  Wide (FP32 storage): the children are widened to FP64 and summed
// there; with at most 64 terms the sum is within 64 FP64 roundings of exact, so
// its FP32 rounding is the correctly rounded average in all but rare ties, and
// the FP32 residue lo = S - hi carries the rest of the pressure; one convert and
// one FP64 add per child instead of Kahan's four instructions.  Plain: the FP64
// mode and naive FP32 sum in their own type.
template <typename T, int SM> struct ChildSum {
    static constexpr bool kWide = std::is_same<T, float>::value && SM == kSumWide;
    using W = typename std::conditional<kWide, double, T>::type;
    static constexpr bool kComp = SM == kSumKahan;   // Kahan in T
    Acc<W, kComp> acc;
    __device__ __forceinline__ void add(T v) { acc.add(W(v)); }
    // a plane's sum (s, with its compensation c) added to the cell's
    __device__ __forceinline__ void add_plane(W ps, W pc) {
        acc.add(ps);
        if constexpr (kComp) acc.add(-pc);
    }
    // the average, and what its rounding leaves out (the scale 1/r^3 is a power
    // of two, so the scaling is exact)
    __device__ __forceinline__ T hi(T inv) const { return T(acc.s * W(inv)); }
    __device__ __forceinline__ T lo(T inv) const {
        if constexpr (kWide) return T(acc.s * W(inv) - W(hi(inv)));
        else return -acc.c * inv;
    }
};

// Fields F0 .. F1 - 1 of (u, v, w, p): all four for the bulk, given and learned
// velocity sources, the pressure alone beside the brick kernel (which restricts
// u, v, w).
template <typename T, int R, int SM, int F0, int F1>
__global__ __launch_bounds__(kBlock) void k_restrict(StepArgs<T> a) {
    const Geo<T> &g = a.g;
    const int64_t tile = xcd_tile(blockIdx.x, gridDim.x);
    const int64_t c = tile * kBlock + threadIdx.x;
    if (c < g.ncell) {
        int cx, cy, cz;
        decode_cell(c, g.nb, cx, cy, cz);
        const int64_t nfx = g.nf[0], nfxy = (int64_t)g.nf[0] * g.nf[1];
        const int64_t base = (int64_t)R * cz * nfxy + (int64_t)R * cy * nfx + (int64_t)R * cx;
        const T inv = T(1) / T(R * R * R);
#pragma unroll
        for (int f = F0; f < F1; ++f) {
            const T *__restrict__ q = a.fine[f] + base;
            Row<T, R> rows[R][R];
#pragma unroll
            for (int lz = 0; lz < R; ++lz)
#pragma unroll
                for (int ly = 0; ly < R; ++ly) rows[lz][ly] = load_row<T, R, true>(q + lz * nfxy + ly * nfx);
            // per fine child plane, then the planes in order (with a Kahan sum,
            // s_0, -c_0, s_1, ...): the same sums as the brick-tiled kernel
            ChildSum<T, SM> acc;
#pragma unroll
            for (int lz = 0; lz < R; ++lz) {
                ChildSum<T, SM> plane;
#pragma unroll
                for (int ly = 0; ly < R; ++ly)
#pragma unroll
                    for (int lx = 0; lx < R; ++lx) plane.add(rows[lz][ly].v[lx]);
                acc.add_plane(plane.acc.s, plane.acc.c);
            }
            const T val = acc.hi(inv);
            if (f < 3) {
                a.U[f * g.ncell + c] = val;
            } else {
                a.P[c] = val;
                // keep the rest of the average so that the pressure gradient can
                // difference (hi + lo) instead of the rounded hi
                a.Plo[c] = acc.lo(inv);
            }
        }
    }
}

// The same restrictions for r = 4 with four threads per bulk cell, one per fine
// child plane (64 cells per workgroup): a thread loads its plane's 4 x 4 child
// values of every field with streaming loads and sums them, and the cell's four
// plane sums are combined in order through cross-lane reads, the sums of the
// per-cell kernel above bit for bit.  A wave's row load covers 16 cells x 4
// planes, whole 128-byte lines, and each thread keeps a quarter of the per-cell
// kernel's loads in flight.  ALPHA: the liquid fraction instead of (u, v, w, p).
constexpr int kPlaneCells = kBlock / 4;   // bulk cells per workgroup

template <typename T, int SM, int F0, int F1, bool ALPHA>
__global__ __launch_bounds__(kBlock) void k_restrict_planes(StepArgs<T> a) {
    constexpr int R = 4, NF = ALPHA ? 1 : F1 - F0;
    const Geo<T> &g = a.g;
    const int t = (int)threadIdx.x, lane = t % kWave, rz = t & 3;
    const int64_t c = xcd_tile(blockIdx.x, gridDim.x) * kPlaneCells + (t >> 2);
    const bool inside = c < g.ncell;
    int cx, cy, cz;
    decode_cell(inside ? c : g.ncell - 1, g.nb, cx, cy, cz);   // every lane takes part in the cross-lane reads
    const int64_t nfx = g.nf[0], nfxy = (int64_t)g.nf[0] * g.nf[1];
    const int64_t base = ((int64_t)R * cz + rz) * nfxy + (int64_t)R * cy * nfx + (int64_t)R * cx;
    Row<T, R> rows[NF][R];
#pragma unroll
    for (int f = 0; f < NF; ++f) {
        const T *__restrict__ q = (ALPHA ? a.fine_alpha : a.fine[F0 + f]) + base;
#pragma unroll
        for (int ry = 0; ry < R; ++ry) rows[f][ry] = load_row<T, R, true>(q + ry * nfx);
    }
    const T inv = T(1) / T(R * R * R);
    const int l0 = lane & ~3;
#pragma unroll
    for (int f = 0; f < NF; ++f) {
        ChildSum<T, SM> plane;
#pragma unroll
        for (int ry = 0; ry < R; ++ry)
#pragma unroll
            for (int rx = 0; rx < R; ++rx) plane.add(rows[f][ry].v[rx]);
        ChildSum<T, SM> acc;
#pragma unroll
        for (int k = 0; k < R; ++k) {
            const auto sk = __shfl(plane.acc.s, l0 + k, kWave);
            const auto ck = ChildSum<T, SM>::kComp ? __shfl(plane.acc.c, l0 + k, kWave) : plane.acc.c;
            acc.add_plane(sk, ck);
        }
        if (inside && rz == 0) {
            if constexpr (ALPHA) {
                a.alpha[c] = acc.hi(inv);
            } else if (F0 + f < 3) {
                a.U[(F0 + f) * g.ncell + c] = acc.hi(inv);
            } else {
                a.P[c] = acc.hi(inv);
                a.Plo[c] = acc.lo(inv);
            }
        }
    }
}

// Restriction of the liquid volume fraction (two-fluid drag): the bulk alpha is
// the average of the r^3 fine children (the volume average that defines alpha),
// summed per fine child plane and then the planes in order, as for U and P.
template <typename T, int R, int SM>
__global__ __launch_bounds__(kBlock) void k_restrict_alpha(StepArgs<T> a) {
    const Geo<T> &g = a.g;
    const int64_t tile = xcd_tile(blockIdx.x, gridDim.x);
    const int64_t c = tile * kBlock + threadIdx.x;
    if (c >= g.ncell) return;
    int cx, cy, cz;
    decode_cell(c, g.nb, cx, cy, cz);
    const int64_t nfx = g.nf[0], nfxy = (int64_t)g.nf[0] * g.nf[1];
    const T *__restrict__ q = a.fine_alpha + (int64_t)R * cz * nfxy + (int64_t)R * cy * nfx + (int64_t)R * cx;
    Row<T, R> rows[R][R];
#pragma unroll
    for (int lz = 0; lz < R; ++lz)
#pragma unroll
        for (int ly = 0; ly < R; ++ly) rows[lz][ly] = load_row<T, R, true>(q + lz * nfxy + ly * nfx);
    ChildSum<T, SM> acc;
#pragma unroll
    for (int lz = 0; lz < R; ++lz) {
        ChildSum<T, SM> plane;
#pragma unroll
        for (int ly = 0; ly < R; ++ly)
#pragma unroll
            for (int lx = 0; lx < R; ++lx) plane.add(rows[lz][ly].v[lx]);
        acc.add_plane(plane.acc.s, plane.acc.c);
    }
    a.alpha[c] = acc.hi(T(1) / T(R * R * R));
}

// The bulk alpha at the eight cells cell + {0,1}^3 (clamped into the grid), as
// one 8-value record per cell: the drag kernel runs in input order, and a
// particle's trilinear stencil (whose lower corner is the record's cell) is
// then one 32-byte read instead of reads from four rows of the bulk grid.
template <typename T>
__global__ __launch_bounds__(kBlock) void k_pack_alpha8(StepArgs<T> a) {
    const Geo<T> &g = a.g;
    const int64_t c = (int64_t)blockIdx.x * kBlock + threadIdx.x;
    if (c >= g.ncell) return;
    int cx, cy, cz;
    decode_cell(c, g.nb, cx, cy, cz);
    const int64_t nx = g.nb[0], nxy = nx * g.nb[1];
    const int64_t xs[2] = {cx, cx + 1 < g.nb[0] ? cx + 1 : cx};
    const int64_t ys[2] = {cy * nx, (cy + 1 < g.nb[1] ? cy + 1 : cy) * nx};
    const int64_t zs[2] = {cz * nxy, (cz + 1 < g.nb[2] ? cz + 1 : cz) * nxy};
    vec4<T> r[2];
    for (int dz = 0; dz < 2; ++dz) {
        r[dz].x = a.alpha[zs[dz] + ys[0] + xs[0]];
        r[dz].y = a.alpha[zs[dz] + ys[0] + xs[1]];
        r[dz].z = a.alpha[zs[dz] + ys[1] + xs[0]];
        r[dz].w = a.alpha[zs[dz] + ys[1] + xs[1]];
    }
    vec4<T> *out = reinterpret_cast<vec4<T> *>(a.alpha8) + 2 * c;
    out[0] = r[0];
    out[1] = r[1];
}

// Trilinear alpha at a particle from its stencil record, in the arithmetic
// order of trilin() (the same value bit for bit).
template <typename T>
__device__ __forceinline__ T trilin_alpha8(const T *__restrict__ alpha8, const Axis<T> &ax, const Axis<T> &ay,
                                           const Axis<T> &az, const int nb[3]) {
    const vec4<T> *r = reinterpret_cast<const vec4<T> *>(alpha8) +
                       2 * (((int64_t)az.lo * nb[1] + ay.lo) * nb[0] + ax.lo);
    const vec4<T> lo = r[0];
    const vec4<T> hi = az.hi != az.lo ? r[1] : lo;
    const bool ox = ax.hi != ax.lo, oy = ay.hi != ay.lo;
    // corner [z][y][x] of the stencil: x, y offsets 0 at a folded wall
    const T z0y0x0 = lo.x, z0y0x1 = ox ? lo.y : lo.x, z0y1x0 = oy ? lo.z : lo.x,
            z0y1x1 = oy ? (ox ? lo.w : lo.z) : (ox ? lo.y : lo.x);
    const T z1y0x0 = hi.x, z1y0x1 = ox ? hi.y : hi.x, z1y1x0 = oy ? hi.z : hi.x,
            z1y1x1 = oy ? (ox ? hi.w : hi.z) : (ox ? hi.y : hi.x);
    const T sx = T(1) - ax.t, sy = T(1) - ay.t, sz = T(1) - az.t;
    const T c00 = sx * z0y0x0 + ax.t * z0y0x1;
    const T c01 = sx * z0y1x0 + ax.t * z0y1x1;
    const T c10 = sx * z1y0x0 + ax.t * z1y0x1;
    const T c11 = sx * z1y1x0 + ax.t * z1y1x1;
    const T c0 = sy * c00 + ay.t * c01;
    const T c1 = sy * c10 + ay.t * c11;
    return sz * c0 + az.t * c1;
}

// Restriction of the velocity with the fine-grid lookup, tiled in bricks of
// 8 x 4 x 2 bulk cells.  Filling a brick: 256 threads, four per cell (one per
// fine child plane z), each loads its plane's r x r rows of u, v, w, stores them
// in LDS and sums its plane (compensated); the four plane sums are combined in
// order through cross-lane reads (the pressure is restricted by k_restrict
// before this kernel).  The brick's particles (8 rows of up to 8 cells,
// contiguous in the sorted order, flattened over the threads) then take their
// trilinear fine velocity from LDS when all eight fine nodes lie in the brick
// (from global memory when the stencil crosses a brick face) and their void
// fraction from a haloed copy of phi in LDS.  The brick is 8r fine cells wide
// along x (one 128-byte line per row for r = 4 in FP32).
// One workgroup per brick: fill, then the particles.
constexpr int kBrickX = 8, kBrickY = 4, kBrickZ = 2;
constexpr int kBrickThreads = 4 * kBrickX * kBrickY * kBrickZ;
constexpr int kBrickRows = kBrickY * kBrickZ;                                     // particle rows of a brick
constexpr int kBrickHalo = (kBrickX + 2) * (kBrickY + 2) * (kBrickZ + 2);         // phi with a one-cell halo

template <typename T, int R> struct BrickLds {
    T sv[3][kBrickZ * R][kBrickY * R][kBrickX * R];
    T sphi[kBrickZ + 2][kBrickY + 2][kBrickX + 2];
    int32_t cnt[kBrickRows];   // particles of each row
    int32_t beg[kBrickRows];   // first sorted position of each row
};

template <typename T> struct BrickGrid {
    int bnx, bny;
    __device__ __forceinline__ void origin(int64_t brick, int &ox, int &oy, int &oz) const {
        ox = (int)(brick % bnx) * kBrickX;
        oy = (int)((brick / bnx) % bny) * kBrickY;
        oz = (int)(brick / ((int64_t)bnx * bny)) * kBrickZ;
    }
};

// Fill the brick at (ox, oy, oz) into L and write its U; thread t in [0, 256).
template <typename T, int R, int SM>
__device__ __forceinline__ void brick_fill(const StepArgs<T> &a, BrickLds<T, R> &L, int t, int ox, int oy, int oz) {
    constexpr int HX = kBrickX + 2, HY = kBrickY + 2;
    const Geo<T> &g = a.g;
    const int lane = t % kWave;
    const int cl = t >> 2, rz = t & 3;   // cell of the brick, fine child plane
    const int lx = cl % kBrickX, ly = (cl / kBrickX) % kBrickY, lz = cl / (kBrickX * kBrickY);
    const int cx = ox + lx, cy = oy + ly, cz = oz + lz;
    const bool inside = cx < g.nb[0] && cy < g.nb[1] && cz < g.nb[2];
    const int64_t nx = g.nb[0], nxy = (int64_t)g.nb[0] * g.nb[1];
    const int64_t nfx = g.nf[0], nfxy = (int64_t)g.nf[0] * g.nf[1];
    // Every load of the fill is issued before the first LDS write: the brick's
    // particle rows (their first sorted position and count), phi with its halo
    // (indices clamped at the walls) and the fine rows, so that a workgroup
    // waits for one memory round trip instead of three.
    static_assert(kBrickHalo <= kBrickThreads, "one halo value per thread");
    int32_t seg0 = 0, seg1 = 0;
    if (t < kBrickRows) {
        const int wx = (ox + kBrickX < g.nb[0]) ? kBrickX : g.nb[0] - ox;
        const int ry = oy + t % kBrickY, rzz = oz + t / kBrickY;
        if (ry < g.nb[1] && rzz < g.nb[2]) {
            const int64_t c0 = ox + nx * ry + nxy * rzz;
            seg0 = a.start[c0];
            seg1 = a.start[c0 + wx];
        }
    }
    const int hx = t % HX, hy = (t / HX) % HY, hz = t / (HX * HY);
    T ph = T(0);
    if (t < kBrickHalo) {
        const int gx = clampi(ox - 1 + hx, g.nb[0]), gy = clampi(oy - 1 + hy, g.nb[1]), gz = clampi(oz - 1 + hz, g.nb[2]);
        ph = a.phi[gx + nx * gy + nxy * gz];
    }
    const bool work = inside && rz < R;
    const int64_t base = ((int64_t)R * cz + rz) * nfxy + (int64_t)R * cy * nfx + (int64_t)R * cx;
    const T inv = T(1) / T(R * R * R);
    Row<T, R> rows[3][R];
    if (work) {
#pragma unroll
        for (int f = 0; f < 3; ++f)
#pragma unroll
            for (int ry = 0; ry < R; ++ry) rows[f][ry] = load_row<T, R>(a.fine[f] + base + ry * nfx);
    }
    if (t < kBrickRows) {
        const int32_t b0 = seg_clamp(seg0, a.n);
        L.beg[t] = b0;
        L.cnt[t] = seg_clamp(seg1, a.n) - b0;
    }
    if (t < kBrickHalo) L.sphi[hz][hy][hx] = ph;
#pragma unroll
    for (int f = 0; f < 3; ++f) {
        ChildSum<T, SM> plane;
        if (work) {
#pragma unroll
            for (int ry = 0; ry < R; ++ry)
#pragma unroll
                for (int rx = 0; rx < R; ++rx) plane.add(rows[f][ry].v[rx]);
#pragma unroll
            for (int ry = 0; ry < R; ++ry)
#pragma unroll
                for (int rx = 0; rx < R; ++rx) L.sv[f][lz * R + rz][ly * R + ry][lx * R + rx] = rows[f][ry].v[rx];
        }
        // the planes of this cell in order (with a Kahan sum, s_0, -c_0, s_1,
        // ...), read from the cell's four lanes; the plane-0 lane writes the
        // average
        ChildSum<T, SM> acc;
        const int l0 = lane & ~3;
#pragma unroll
        for (int k = 0; k < R; ++k) {
            const auto sk = __shfl(plane.acc.s, l0 + k, kWave);
            const auto ck = ChildSum<T, SM>::kComp ? __shfl(plane.acc.c, l0 + k, kWave) : plane.acc.c;
            acc.add_plane(sk, ck);
        }
        if (inside && rz == 0) a.U[f * g.ncell + (cx + nx * cy + nxy * cz)] = acc.hi(inv);
    }
}

// The particles of the filled brick at (ox, oy, oz): thread t of nt.
template <typename T, int R>
__device__ __forceinline__ void brick_particles(const StepArgs<T> &a, const BrickLds<T, R> &L, int t, int nt, int ox,
                                                int oy, int oz) {
    constexpr int FX = kBrickX * R, FY = kBrickY * R, FZ = kBrickZ * R;
    const Geo<T> &g = a.g;
    int32_t pre[kBrickRows + 1];   // particles before each row
    pre[0] = 0;
#pragma unroll
    for (int r = 0; r < kBrickRows; ++r) pre[r + 1] = pre[r] + L.cnt[r];
    const int total = pre[kBrickRows];
    const int fx0 = ox * R, fy0 = oy * R, fz0 = oz * R;
    // up to kPB particles per thread at a time: their loads are issued together
    constexpr int kPB = 2;
    for (int j0 = t; j0 < total; j0 += kPB * nt) {
        vec4<T> qs[kPB];
        int64_t ps[kPB];
#pragma unroll
        for (int k = 0; k < kPB; ++k) {
            const int j = j0 + k * nt;
            int64_t i = L.beg[0];
            if (j < total) {
                int r = 0;
#pragma unroll
                for (int q = 1; q < kBrickRows; ++q) r += (pre[q] <= j) ? 1 : 0;
                i = L.beg[r] + (j - pre[r]);
            }
            qs[k] = a.sp[i];
            ps[k] = a.perm[i];
        }
#pragma unroll
        for (int k = 0; k < kPB; ++k) {
            if (j0 + k * nt >= total) break;
            const vec4<T> q = qs[k];
            int64_t p = ps[k];
            if (p < 0 || p >= a.n) p = 0;   // perm is a permutation of [0, n)
            vec4<T> s;
            // fine trilinear velocity: from LDS when the eight nodes lie in the brick
            const Axis<T> ax = cic_axis(q.x, g.sf[0], g.nf[0]);
            const Axis<T> ay = cic_axis(q.y, g.sf[1], g.nf[1]);
            const Axis<T> az = cic_axis(q.z, g.sf[2], g.nf[2]);
            const int xl = ax.lo - fx0, xh = ax.hi - fx0, yl = ay.lo - fy0, yh = ay.hi - fy0, zl = az.lo - fz0,
                      zh = az.hi - fz0;
            if (xl >= 0 && xh < FX && yl >= 0 && yh < FY && zl >= 0 && zh < FZ) {
                const T sx = T(1) - ax.t, sy = T(1) - ay.t, sz = T(1) - az.t;
                T u[3];
#pragma unroll
                for (int f = 0; f < 3; ++f) {
                    const T e0 = sy * (sx * L.sv[f][zl][yl][xl] + ax.t * L.sv[f][zl][yl][xh]) +
                                 ay.t * (sx * L.sv[f][zl][yh][xl] + ax.t * L.sv[f][zl][yh][xh]);
                    const T e1 = sy * (sx * L.sv[f][zh][yl][xl] + ax.t * L.sv[f][zh][yl][xh]) +
                                 ay.t * (sx * L.sv[f][zh][yh][xl] + ax.t * L.sv[f][zh][yh][xh]);
                    u[f] = sz * e0 + az.t * e1;
                }
                s.x = u[0];
                s.y = u[1];
                s.z = u[2];
            } else {
                fine_velocity(q, a, s.x, s.y, s.z);
            }
            // void fraction at the particle from the haloed phi (its stencil is the
            // containing cell and a neighbour, always inside the halo)
            if (a.cic) {
                const Axis<T> bx = cic_axis(q.x, g.sb[0], g.nb[0]);
                const Axis<T> by = cic_axis(q.y, g.sb[1], g.nb[1]);
                const Axis<T> bz = cic_axis(q.z, g.sb[2], g.nb[2]);
                const int hxl = bx.lo - ox + 1, hxh = bx.hi - ox + 1, hyl = by.lo - oy + 1, hyh = by.hi - oy + 1,
                          hzl = bz.lo - oz + 1, hzh = bz.hi - oz + 1;
                const T f000 = L.sphi[hzl][hyl][hxl], f001 = L.sphi[hzl][hyl][hxh], f010 = L.sphi[hzl][hyh][hxl],
                        f011 = L.sphi[hzl][hyh][hxh], f100 = L.sphi[hzh][hyl][hxl], f101 = L.sphi[hzh][hyl][hxh],
                        f110 = L.sphi[hzh][hyh][hxl], f111 = L.sphi[hzh][hyh][hxh];
                const T sx = T(1) - bx.t, sy = T(1) - by.t, sz = T(1) - bz.t;
                const T phi_p = sz * (sy * (sx * f000 + bx.t * f001) + by.t * (sx * f010 + bx.t * f011)) +
                                bz.t * (sy * (sx * f100 + bx.t * f101) + by.t * (sx * f110 + bx.t * f111));
                if (std::is_same<T, float>::value && phi_p > (T)a.phi_fp64) {
                    // FP64 weights from the same positions; the cancellation in 1 - phi is exact
                    const double gx = (double)q.x * (double)g.sb[0] - 0.5, gy = (double)q.y * (double)g.sb[1] - 0.5,
                                 gz = (double)q.z * (double)g.sb[2] - 0.5;
                    const double tx = gx - floor(gx), ty = gy - floor(gy), tz = gz - floor(gz);
                    const double ux = 1.0 - tx, uy = 1.0 - ty, uz = 1.0 - tz;
                    const double ph =
                        uz * (uy * (ux * (double)f000 + tx * (double)f001) + ty * (ux * (double)f010 + tx * (double)f011)) +
                        tz * (uy * (ux * (double)f100 + tx * (double)f101) + ty * (ux * (double)f110 + tx * (double)f111));
                    s.w = (T)(1.0 - ph);
                } else {
                    s.w = T(1) - phi_p;
                }
            } else {
                const int ix = cell_axis(q.x, g.sb[0], g.nb[0]), iy = cell_axis(q.y, g.sb[1], g.nb[1]),
                          iz = cell_axis(q.z, g.sb[2], g.nb[2]);
                s.w = T(1) - L.sphi[iz - oz + 1][iy - oy + 1][ix - ox + 1];
            }
            a.uf4[p] = s;
        }
    }
}

template <typename T, int R, int SM>
__global__ __launch_bounds__(kBrickThreads) void k_restrict_brick(StepArgs<T> a, BrickGrid<T> bg) {
    static_assert(R <= 4, "one thread per fine child plane");
    static_assert(kBrickRows <= kBrickThreads, "one particle row per thread");
    __shared__ BrickLds<T, R> L;
    int ox, oy, oz;
    bg.origin(xcd_tile(blockIdx.x, gridDim.x), ox, oy, oz);
    brick_fill<T, R, SM>(a, L, threadIdx.x, ox, oy, oz);
    __syncthreads();
    brick_particles<T, R>(a, L, threadIdx.x, kBrickThreads, ox, oy, oz);
}

template <typename T, int R> int64_t brick_blocks(const Geo<T> &g) {
    return (int64_t)((g.nb[0] + kBrickX - 1) / kBrickX) * ((g.nb[1] + kBrickY - 1) / kBrickY) *
           ((g.nb[2] + kBrickZ - 1) / kBrickZ);
}

// Sampling for the bulk-velocity and given-velocity sources (sorted order).
template <typename T>
__global__ __launch_bounds__(kBlock) void k_sample(StepArgs<T> a) {
    const int64_t i = (int64_t)blockIdx.x * kBlock + threadIdx.x;
    if (i < a.n) {
        const int64_t idx[1] = {i};
        sample_particles<T, 1>(idx, a);
    }
}

// ---------------------------------------------------------------------------
// Drag and advection, one thread per particle in input order (coalesced).
//   F = beta (u_f - u_p), beta written as
//   1/2 rho_f (pi d^2/4) eps*^(2-chi) (0.63 sqrt|u_r| + 4.8 sqrt(mu_f/(rho_f eps* d)))^2
// which equals 1/2 C_D rho_f A eps*^(2-chi) |u_r| with C_D = (0.63 + 4.8/sqrt(Re))^2,
// Re = rho_f eps* d |u_r| / mu_f, chi = 3.7 - 0.65 exp(-(1.5 - log10 Re)^2 / 2), and
// stays finite as |u_r| -> 0 (where F = 0).
// ---------------------------------------------------------------------------
template <typename T>
__global__ __launch_bounds__(kBlock) void k_drag(StepArgs<T> a) {
    __shared__ double red[kWavesPerBlock];
    const Geo<T> &g = a.g;
    const int64_t p = (int64_t)blockIdx.x * kBlock + threadIdx.x;
    double acc[9] = {0.0, 0.0, 0.0, 0.0, 0.0, 0.0, 0.0, 0.0, 0.0};   // sum F (3), clamped, V_p, beta, beta u_p (3)
    if (p < a.n) {
        int o = 0;
        const T xs[3] = {clamp_coord(a.pos[3 * p + 0], g.L[0], o), clamp_coord(a.pos[3 * p + 1], g.L[1], o),
                         clamp_coord(a.pos[3 * p + 2], g.L[2], o)};
        const T us[3] = {a.vel[3 * p + 0], a.vel[3 * p + 1], a.vel[3 * p + 2]};
        const T d = a.diam[p];
        const vec4<T> s = a.uf4[p];
        T uf[3] = {s.x, s.y, s.z};
        if (a.vel_source == 2)
            for (int k = 0; k < 3; ++k) uf[k] = a.uf_given[3 * p + k];
        if (a.uf_out)
            for (int k = 0; k < 3; ++k) a.uf_out[3 * p + k] = uf[k];
        const T ur0 = uf[0] - us[0], ur1 = uf[1] - us[1], ur2 = uf[2] - us[2];
        const T mag = dsqrt(ur0 * ur0 + ur1 * ur1 + ur2 * ur2);
        T e = s.w;
        int clamped = 0;
        if (e < a.eps_min) {
            e = a.eps_min;
            clamped = 1;
        }
        // fluid density and viscosity at the particle: fluid 1's, or with the
        // two-fluid drag the mixture by the liquid fraction interpolated from
        // the restricted alpha
        T rho = a.rho_f, mu = a.mu_f;
        if (a.vof) {
            const Axis<T> bx = cic_axis(xs[0], g.sb[0], g.nb[0]);
            const Axis<T> by = cic_axis(xs[1], g.sb[1], g.nb[1]);
            const Axis<T> bz = cic_axis(xs[2], g.sb[2], g.nb[2]);
            const T al = trilin_alpha8(a.alpha8, bx, by, bz, g.nb);
            rho = a.rho_f * al + a.rho_f2 * (T(1) - al);
            mu = a.mu_f * al + a.mu_f2 * (T(1) - al);
        }
        T chi = T(3.7);
        if (mag > T(0)) {
            const T re = rho * e * d * mag / mu;
            const T l = T(1.5) - dlog10(re);
            chi = T(3.7) - T(0.65) * dexp(-l * l * T(0.5));
        }
        const T vfac = dpow(e, T(2) - chi);
        const T sq = T(0.63) * dsqrt(mag) + T(4.8) * dsqrt(mu / (rho * e * d));
        const T area = T(kPi / 4.0) * d * d;
        const T beta = T(0.5) * rho * area * vfac * (sq * sq);
        const T Fs[3] = {beta * ur0, beta * ur1, beta * ur2};
        for (int k = 0; k < 3; ++k) a.drag[3 * p + k] = Fs[k];
        if (a.beta) a.beta[p] = beta;
        for (int k = 0; k < 3; ++k) acc[k] = (double)Fs[k];
        acc[3] = clamped;
        const double dd = (double)d;
        acc[4] = kPi * dd * dd * dd / 6.0;
        if (a.semi) {
            // (beta, beta u_p) with the velocity the drag used, for the
            // semi-implicit deposition (this thread has read uf4[p] already)
            vec4<T> b;
            b.x = beta;
            b.y = beta * us[0];
            b.z = beta * us[1];
            b.w = beta * us[2];
            a.uf4[p] = b;
            acc[5] = (double)beta;
            acc[6] = (double)b.y;
            acc[7] = (double)b.z;
            acc[8] = (double)b.w;
        }

        if (a.advect) {
            // explicit Euler from the old state, specular reflection at the walls
            const T m = a.rho_p * (T(kPi / 6.0) * d * d * d);
            for (int k = 0; k < 3; ++k) {
                T xn = dfma(a.dt, us[k], xs[k]);
                T un = dfma(a.dt, Fs[k] / m, us[k]);
                const T L = g.L[k];
                if (xn < T(0)) {
                    xn = -xn;
                    un = -un;
                } else if (xn > L) {
                    xn = T(2) * L - xn;
                    un = -un;
                }
                xn = fmin(fmax(xn, T(0)), L);
                a.pos[3 * p + k] = xn;
                a.vel[3 * p + k] = un;
            }
        }
    }
    const int slots[9] = {SL_FP, SL_FP + 1, SL_FP + 2, SL_NCLAMP, SL_VTOT, SL_KP, SL_KUP, SL_KUP + 1, SL_KUP + 2};
    const int nsl = a.semi ? 9 : 5;   // uniform over the launch
    for (int k = 0; k < nsl; ++k) {
        const double t = block_sum(acc[k], red);
        if (threadIdx.x == 0) a.part[slots[k] * a.part_stride + blockIdx.x] = t;
    }
}

// ---------------------------------------------------------------------------
// Prolongation bulk -> fine (conservative trilinear)
// ---------------------------------------------------------------------------
// Child l of a parent cell sits at offset o = (l + 1/2)/R - 1/2 (in bulk cell
// units) from the parent centre; its 1-D trilinear weights on the nodes
// (c-1, c, c+1) are (max(-o,0), 1-|o|, max(o,0)).
template <int R> struct ChildW {
    static constexpr double off(int l) { return (l + 0.5) / R - 0.5; }
    static constexpr double w(int l, int k) {  // k = 0,1,2 for c-1, c, c+1
        return k == 0 ? (off(l) < 0 ? -off(l) : 0.0)
                      : (k == 1 ? 1.0 - (off(l) < 0 ? -off(l) : off(l)) : (off(l) > 0 ? off(l) : 0.0));
    }
    static constexpr double mean(int k) {       // (1/R) sum_l w(l, k)
        double s = 0.0;
        for (int l = 0; l < R; ++l) s += w(l, k);
        return s / R;
    }
};

template <typename T, int R>
__device__ __forceinline__ T wsum3(int l, T a0, T a1, T a2) {
    // sum_k w(l,k) a_k, skipping structurally zero weights
    T s = T(ChildW<R>::w(l, 1)) * a1;
    if (ChildW<R>::w(l, 0) != 0.0) s += T(ChildW<R>::w(l, 0)) * a0;
    if (ChildW<R>::w(l, 2) != 0.0) s += T(ChildW<R>::w(l, 2)) * a2;
    return s;
}

// The bulk fields a prolongation launch transfers (nf <= 4), their fine outputs
// and the diagnostic slots of their fine sums; field 0 is optionally
// complemented (the solid fraction phi is prolonged as the porosity 1 - phi).
template <typename T> struct ProlongSet {
    const T *B[4];
    T *out[4];
    int slot[4];
    int complement0;
    int nf;
};

// One workgroup per tile of kPTX x kPTY bulk cells of one layer (a wave per
// bulk row).  The bulk values of the tile's 3 x 3 x 3 neighbourhoods (the tile
// with a one-cell halo, indices clamped at the walls) are staged in LDS for all
// NF fields at once: one memory round trip per workgroup, and each cell reads
// its 27 values at fixed offsets from one LDS address.  Each thread then
// writes its cell's r^3 fine children of every field, one r-wide row at a
// time (a wave's store covers kPTX cells' children on one fine row).
constexpr int kPTX = kWave, kPTY = kBlock / kWave;
constexpr int kPHX = kPTX + 2, kPHY = kPTY + 2, kPHalo = 3 * kPHY * kPHX;   // staged values per field

int64_t prolong_tiles(const int nb[3]) {
    return (int64_t)((nb[0] + kPTX - 1) / kPTX) * ((nb[1] + kPTY - 1) / kPTY) * nb[2];
}

template <typename T, int R, int NF>
__global__ __launch_bounds__(kBlock) void k_prolong(StepArgs<T> a, ProlongSet<T> fs) {
    __shared__ T sb[NF][3][kPHY][kPHX];
    __shared__ double red[kWavesPerBlock];
    const Geo<T> &g = a.g;
    const int tnx = (g.nb[0] + kPTX - 1) / kPTX, tny = (g.nb[1] + kPTY - 1) / kPTY;
    const int64_t tile = xcd_tile(blockIdx.x, gridDim.x);
    const int cx0 = (int)(tile % tnx) * kPTX, cy0 = (int)((tile / tnx) % tny) * kPTY;
    const int cz = (int)(tile / ((int64_t)tnx * tny));
    const int64_t nx = g.nb[0], nxy = (int64_t)g.nb[0] * g.nb[1];
    // staging: every load is issued before the first LDS write
    constexpr int kIt = (kPHalo + kBlock - 1) / kBlock;
    T v[NF][kIt];
#pragma unroll
    for (int f = 0; f < NF; ++f)
#pragma unroll
        for (int it = 0; it < kIt; ++it) {
            const int e = it * kBlock + (int)threadIdx.x;
            v[f][it] = T(0);
            if (e < kPHalo) {
                const int i = e % kPHX, j = (e / kPHX) % kPHY, k = e / (kPHX * kPHY);
                const int gx = clampi(cx0 - 1 + i, g.nb[0]), gy = clampi(cy0 - 1 + j, g.nb[1]),
                          gz = clampi(cz - 1 + k, g.nb[2]);
                v[f][it] = fs.B[f][gz * nxy + gy * nx + gx];
            }
        }
#pragma unroll
    for (int f = 0; f < NF; ++f)
#pragma unroll
        for (int it = 0; it < kIt; ++it) {
            const int e = it * kBlock + (int)threadIdx.x;
            if (e < kPHalo) (&sb[f][0][0][0])[e] = (f == 0 && fs.complement0) ? T(1) - v[f][it] : v[f][it];
        }
    __syncthreads();

    const int lane = (int)threadIdx.x % kWave, w = (int)threadIdx.x / kWave;
    const int cx = cx0 + lane, cy = cy0 + w;
    const bool inside = cx < g.nb[0] && cy < g.nb[1];
    const int64_t c = cz * nxy + cy * nx + cx;
    const bool counted = inside && c >= a.own_c0 && c < a.own_c1;   // owned cells enter the fine-grid sums
    double sums[NF];
#pragma unroll
    for (int f = 0; f < NF; ++f) sums[f] = 0.0;
    if (inside) {
        const int64_t nfx = g.nf[0], nfxy = (int64_t)g.nf[0] * g.nf[1];
        const int64_t fbase = (int64_t)R * cz * nfxy + (int64_t)R * cy * nfx + (int64_t)R * cx;
#pragma unroll
        for (int f = 0; f < NF; ++f) {
            T *__restrict__ out = fs.out[f];
            T b[3][3][3];
#pragma unroll
            for (int k = 0; k < 3; ++k)
#pragma unroll
                for (int j = 0; j < 3; ++j)
#pragma unroll
                    for (int i = 0; i < 3; ++i) b[k][j][i] = sb[f][k][w + j][lane + i];
            // defect of the parent: B_c - (1/R^3) sum of the trilinear children
            T D = T(0);
            if constexpr (R > 1) {
                T mz[3];
#pragma unroll
                for (int k = 0; k < 3; ++k) {
                    T my[3];
#pragma unroll
                    for (int j = 0; j < 3; ++j)
                        my[j] = T(ChildW<R>::mean(0)) * b[k][j][0] + T(ChildW<R>::mean(1)) * b[k][j][1] +
                                T(ChildW<R>::mean(2)) * b[k][j][2];
                    mz[k] = T(ChildW<R>::mean(0)) * my[0] + T(ChildW<R>::mean(1)) * my[1] +
                            T(ChildW<R>::mean(2)) * my[2];
                }
                T mean = T(ChildW<R>::mean(0)) * mz[0] + T(ChildW<R>::mean(1)) * mz[1] +
                         T(ChildW<R>::mean(2)) * mz[2];
                D = b[1][1][1] - mean;
            }
            // separable trilinear: x, then y, then z
            T X[3][3][R];
#pragma unroll
            for (int k = 0; k < 3; ++k)
#pragma unroll
                for (int j = 0; j < 3; ++j)
#pragma unroll
                    for (int lx = 0; lx < R; ++lx) X[k][j][lx] = wsum3<T, R>(lx, b[k][j][0], b[k][j][1], b[k][j][2]);
            // one child row y at a time (its y-interpolated values only are
            // live), all its planes z
            double s = 0.0;
#pragma unroll
            for (int ly = 0; ly < R; ++ly) {
                T Y[3][R];
#pragma unroll
                for (int k = 0; k < 3; ++k)
#pragma unroll
                    for (int lx = 0; lx < R; ++lx) Y[k][lx] = wsum3<T, R>(ly, X[k][0][lx], X[k][1][lx], X[k][2][lx]);
#pragma unroll
                for (int lz = 0; lz < R; ++lz) {
                    T o[R];
#pragma unroll
                    for (int lx = 0; lx < R; ++lx) {
                        o[lx] = wsum3<T, R>(lz, Y[0][lx], Y[1][lx], Y[2][lx]) + D;
                        s += (double)o[lx];
                    }
                    store_row<T, R>(out + fbase + lz * nfxy + ly * nfx, o);
                    // keeps the scheduler from computing every row before the
                    // first store (all r^3 values live at once)
                    __builtin_amdgcn_sched_barrier(0);
                }
            }
            sums[f] = counted ? s : 0.0;
        }
    }
#pragma unroll
    for (int k = 0; k < NF; ++k) {
        const double t = block_sum(sums[k], red);
        if (threadIdx.x == 0) a.part[fs.slot[k] * a.part_stride + blockIdx.x] = t;
    }
}

// ---------------------------------------------------------------------------
// Final fixed-order reduction of the per-workgroup partials
// ---------------------------------------------------------------------------
struct DiagSpec {
    int nblk[SL_COUNT];
    double scale[SL_COUNT];
};

// Stage 1: workgroup (slot, chunk) sums a contiguous chunk of the slot's
// partials (thread t: elements t, t + kBlock, ... of the chunk, in order), then a
// fixed tree; stage 2: one workgroup per slot combines the kDiagChunks values in
// order.  Deterministic.
constexpr int kDiagChunks = 32;

__global__ __launch_bounds__(kBlock) void k_diag1(const double *__restrict__ part, int64_t ps, DiagSpec spec,
                                                  double *__restrict__ part2) {
    __shared__ double red[kWavesPerBlock];
    const int s = blockIdx.x / kDiagChunks, ch = blockIdx.x % kDiagChunks;
    const bool is_max = (s == SL_MAXPHI);
    const int nb = spec.nblk[s];
    const int per = (nb + kDiagChunks - 1) / kDiagChunks;
    const int j0 = ch * per, j1 = (j0 + per < nb) ? j0 + per : nb;
    const double *src = part + s * ps;
    double v = 0.0;
    for (int j = j0 + threadIdx.x; j < j1; j += kBlock) v = is_max ? fmax(v, src[j]) : v + src[j];
    const double t = is_max ? block_max(v, red) : block_sum(v, red);
    if (threadIdx.x == 0) part2[blockIdx.x] = t;
}

__global__ __launch_bounds__(kWave) void k_diag2(const double *__restrict__ part2, DiagSpec spec,
                                                 double *__restrict__ diag) {
    const int s = blockIdx.x;
    const bool is_max = (s == SL_MAXPHI);
    double v = 0.0;
    if (threadIdx.x < kDiagChunks) v = part2[s * kDiagChunks + threadIdx.x];
    v = is_max ? wave_max(v) : wave_sum(v);
    if (threadIdx.x == 0) diag[s] = v * spec.scale[s];
}

// ---------------------------------------------------------------------------
// Host dispatch
// ---------------------------------------------------------------------------
// Restriction of fields F0 .. F1 - 1: four threads per cell for r = 4, one
// otherwise.
template <typename T, int R, int SM, int F0, int F1> static void restrict_fields(const StepArgs<T> &a, hipStream_t st) {
    if constexpr (R == 4)
        hipLaunchKernelGGL((k_restrict_planes<T, SM, F0, F1, false>),
                           dim3((unsigned)((a.g.ncell + kPlaneCells - 1) / kPlaneCells)), dim3(kBlock), 0, st, a);
    else
        hipLaunchKernelGGL((k_restrict<T, R, SM, F0, F1>), dim3((unsigned)((a.g.ncell + kBlock - 1) / kBlock)),
                           dim3(kBlock), 0, st, a);
}

template <typename T, int R, int SM>
static void launch_grid_stages(const StepArgs<T> &a, hipStream_t st, int phases) {
    const int64_t cb = (a.g.ncell + kBlock - 1) / kBlock;
    const int64_t pb = (a.n + kBlock - 1) / kBlock;
    const int64_t nc = a.g.ncell, nf = a.g.nfine;
    const ProlongSet<T> eps{{a.phi, nullptr, nullptr, nullptr}, {a.fine_eps, nullptr, nullptr, nullptr},
                            {SL_EPSF, 0, 0, 0}, 1, 1};
    if (phases & kPhaseVelocity) {
    if (a.vel_source == 0) {
        // the pressure (for the gradient only), then u, v, w with the lookup
        a.mk->mark("restrict_p", st);
        restrict_fields<T, R, SM, 3, 4>(a, st);
        a.mk->mark("restrict_lookup", st);
        const int64_t nbk = brick_blocks<T, R>(a.g);
        const BrickGrid<T> bg{(a.g.nb[0] + kBrickX - 1) / kBrickX, (a.g.nb[1] + kBrickY - 1) / kBrickY};
        hipLaunchKernelGGL((k_restrict_brick<T, R, SM>), dim3((unsigned)nbk), dim3(kBrickThreads), 0, st, a, bg);
    } else if (a.vel_source == 3) {
        if constexpr (std::is_same<T, float>::value) {
            a.mk->mark("restrict", st);
            restrict_fields<T, R, SM, 0, 4>(a, st);
            a.mk->mark("mlp_pack", st);
            launch_mlp_pack(a, st);
            if (a.n > 0) {
                a.mk->mark("mlp_infer", st);
                launch_mlp_infer(a, st);
                a.mk->mark("mlp_check", st);
                launch_mlp_check(a, st);
            }
        }
    } else {
        a.mk->mark("restrict", st);
        restrict_fields<T, R, SM, 0, 4>(a, st);
        if (a.n > 0) a.mk->mark("sample", st);
        if (a.n > 0) hipLaunchKernelGGL(k_sample<T>, dim3(pb), dim3(kBlock), 0, st, a);
    }
    if (a.vof) {
        a.mk->mark("restrict_alpha", st);
        if constexpr (R == 4)
            hipLaunchKernelGGL((k_restrict_planes<T, SM, 0, 1, true>), dim3((unsigned)((nc + kPlaneCells - 1) / kPlaneCells)),
                               dim3(kBlock), 0, st, a);
        else
            hipLaunchKernelGGL((k_restrict_alpha<T, R, SM>), dim3(cb), dim3(kBlock), 0, st, a);
        if (a.n > 0) a.mk->mark("pack_alpha", st);
        if (a.n > 0) hipLaunchKernelGGL(k_pack_alpha8<T>, dim3(cb), dim3(kBlock), 0, st, a);
    }
    if (a.n > 0) a.mk->mark("drag", st);
    if (a.n > 0) hipLaunchKernelGGL(k_drag<T>, dim3(pb), dim3(kBlock), 0, st, a);
    }
    if (phases & kPhaseSource) {
    a.mk->mark("deposit_force", st);
    launch_deposit_force<T, SM>(a, st);
    if (a.semi) {
        a.mk->mark("deposit_semi", st);
        launch_deposit_semi<T, SM>(a, st);
    }
    }
    if (phases & kPhaseProlong) {
    const int64_t ptiles = prolong_tiles(a.g.nb);
    a.mk->mark("prolong_eps", st);
    hipLaunchKernelGGL((k_prolong<T, R, 1>), dim3(ptiles), dim3(kBlock), 0, st, a, eps);
    const ProlongSet<T> src{{a.F, a.F + nc, a.F + 2 * nc, nullptr},
                            {a.fine_F, a.fine_F + nf, a.fine_F + 2 * nf, nullptr},
                            {SL_FF, SL_FF + 1, SL_FF + 2, 0},
                            0, 3};
    a.mk->mark("prolong", st);
    hipLaunchKernelGGL((k_prolong<T, R, 3>), dim3(ptiles), dim3(kBlock), 0, st, a, src);
    if (a.semi) {
        const ProlongSet<T> semi{{a.K, a.KU, a.KU + nc, a.KU + 2 * nc},
                                 {a.fine_K, a.fine_KU, a.fine_KU + nf, a.fine_KU + 2 * nf},
                                 {SL_KF, SL_KUF, SL_KUF + 1, SL_KUF + 2},
                                 0, 4};
        a.mk->mark("prolong_semi", st);
        hipLaunchKernelGGL((k_prolong<T, R, 4>), dim3(ptiles), dim3(kBlock), 0, st, a, semi);
    }
    }
}

template <typename T, int SM> static void launch_by_ratio(const StepArgs<T> &a, hipStream_t st, int phases) {
    switch (a.ratio) {
    case 1: launch_grid_stages<T, 1, SM>(a, st, phases); break;
    case 2: launch_grid_stages<T, 2, SM>(a, st, phases); break;
    default: launch_grid_stages<T, 4, SM>(a, st, phases); break;
    }
}

template <typename T> hipError_t launch_stages(const StepArgs<T> &a, hipStream_t st, int phases) {
    const int64_t cb = (a.g.ncell + kBlock - 1) / kBlock;
    const int64_t pb = (a.n + kBlock - 1) / kBlock;
    const int sm = a.sum_mode;   // FP32 modes; the FP64 mode sums plainly

    // workgroups per diagnostic slot (each writes one partial per slot), checked
    // against the partials' stride before anything is launched
    DiagSpec spec;
    for (int s = 0; s < SL_COUNT; ++s) {
        spec.nblk[s] = (int)cb;
        spec.scale[s] = 1.0;
    }
    const int db = deposit_blocks(a.g.nb, a.g.ncell, a.cic);
    spec.nblk[SL_PHISUM] = db;
    spec.nblk[SL_MAXPHI] = db;
    for (int k = 0; k < 3; ++k) spec.nblk[SL_FB + k] = db;
    spec.nblk[SL_VTOT] = a.n > 0 ? (int)pb : 0;
    spec.nblk[SL_NOUT] = a.n > 0 ? sort_tiles(a.n) : 0;
    const int npart = a.n > 0 ? (int)pb : 0;   // k_drag
    for (int k = 0; k < 3; ++k) spec.nblk[SL_FP + k] = npart;
    spec.nblk[SL_NCLAMP] = npart;
    const int nmlp = (a.vel_source == 3 && a.n > 0) ? (int)mlp_check_blocks(a.n_bricks) : 0;
    spec.nblk[SL_NFALL] = nmlp;
    spec.nblk[SL_MLPERR] = nmlp;
    spec.nblk[SL_MLPREF] = nmlp;
    spec.nblk[SL_MLPSAMP] = nmlp;
    const int ptiles = (int)prolong_tiles(a.g.nb);   // k_prolong
    spec.nblk[SL_EPSF] = ptiles;
    for (int k = 0; k < 3; ++k) spec.nblk[SL_FF + k] = ptiles;
    for (int k = 0; k < 4; ++k) {
        spec.nblk[SL_KP + k] = a.semi ? npart : 0;   // k_drag
        spec.nblk[SL_KB + k] = a.semi ? db : 0;      // deposition
        spec.nblk[SL_KF + k] = a.semi ? ptiles : 0;  // prolongation
        spec.scale[SL_KB + k] = a.g.vb;
        spec.scale[SL_KF + k] = a.g.vf;
    }
    spec.scale[SL_PHISUM] = a.g.vb;
    for (int k = 0; k < 3; ++k) {
        spec.scale[SL_FB + k] = a.g.vb;
        spec.scale[SL_FF + k] = a.g.vf;
    }
    spec.scale[SL_EPSF] = a.g.vf;
    for (int s = 0; s < SL_COUNT; ++s)
        if (spec.nblk[s] > a.part_stride) return hipErrorInvalidValue;   // partials would not fit

    if (phases & kPhaseDeposit) {
        if (a.n > 0) a.mk->mark("gather", st);
        if (a.n > 0)
            hipLaunchKernelGGL(k_gather<T>, dim3(pb), dim3(kBlock), 0, st, a.perm, a.uf4, a.n, a.sp);
        a.mk->mark("deposit_phi", st);
        if constexpr (std::is_same<T, float>::value) {
            if (sm == kSumKahan) launch_deposit_phi<T, kSumKahan>(a, st);
            else if (sm == kSumWide) launch_deposit_phi<T, kSumWide>(a, st);
            else launch_deposit_phi<T, kSumPlain>(a, st);
        } else {
            launch_deposit_phi<T, kSumPlain>(a, st);
        }
    }
    if (phases & (kPhaseVelocity | kPhaseSource | kPhaseProlong)) {
        if constexpr (std::is_same<T, float>::value) {
            if (sm == kSumKahan) launch_by_ratio<T, kSumKahan>(a, st, phases);
            else if (sm == kSumWide) launch_by_ratio<T, kSumWide>(a, st, phases);
            else launch_by_ratio<T, kSumPlain>(a, st, phases);
        } else {
            launch_by_ratio<T, kSumPlain>(a, st, phases);
        }
    }
    if (phases & kPhaseDiag) {
        a.mk->mark("diag", st);
        double *part2 = a.part + (int64_t)SL_COUNT * a.part_stride;
        hipLaunchKernelGGL(k_diag1, dim3(SL_COUNT * kDiagChunks), dim3(kBlock), 0, st, a.part, a.part_stride, spec,
                           part2);
        hipLaunchKernelGGL(k_diag2, dim3(SL_COUNT), dim3(kWave), 0, st, part2, spec, a.diag);
        a.mk->mark(nullptr, st);
    }
    return hipGetLastError();
}

template hipError_t launch_stages<float>(const StepArgs<float> &, hipStream_t, int);
template hipError_t launch_stages<double>(const StepArgs<double> &, hipStream_t, int);

}  // namespace cpl
