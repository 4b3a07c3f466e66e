// deposit.hip -- particle -> bulk-cell deposition of the solid volume fraction
// and of the momentum source, deterministic and without atomics.
//
//   phi_c   = sum_p w_pc V_p / V_b                 (porosity eps = 1 - phi)
//   F_fpi,c = -(1/V_b) sum_p w_pc F_p              (counterpart of the drag)
//   K_c     = (1/V_b) sum_p w_pc beta_p            (semi-implicit split of F_fpi:
//   KU_c    = (1/V_b) sum_p w_pc beta_p u_p         F_fpi = -K u_f + KU in uniform flow)
//
// The particles are in the canonical (cell, id) order with CSR offsets `start`.
// CIC: two passes through partial sums per group of source rows (see below);
// every particle is staged once per pass.  NGP: one thread per cell sums its
// own segment.
#include <type_traits>

#include "common.hpp"
#include "launch.hpp"

namespace cpl {

constexpr int kChunk = 256;   // particles staged per wave and chunk
static_assert(kChunk % kWave == 0, "a chunk is staged in whole waves");

// What a deposition pass sums: V_p / V_b (phi), the drag F_p (source) or
// (beta_p, beta_p u_p) (semi-implicit split).
enum DepMode { kPhi = 0, kForce = 1, kSemi = 2 };
template <int MODE> struct DepNc { static constexpr int value = MODE == kPhi ? 1 : (MODE == kForce ? 3 : 4); };

template <typename T> __device__ __forceinline__ T vol_over_vb(T d, T inv_vb) {
    return (T(kPi / 6.0) * d * d * d) * inv_vb;
}

// Bulk pressure gradient of cell c written to G ([3][ncell]), in the arithmetic
// of gradient_at(): the cell's and its six neighbours' (hi, lo) pressure are
// loaded first, unconditionally (a neighbour beyond a wall is the cell itself),
// so that a kernel can issue these loads with its others and wait once.
template <typename T> struct GradLoads {
    T hi[7], lo[7];   // centre, then (low, high) neighbour per axis
};

template <typename T>
__device__ __forceinline__ GradLoads<T> load_gradient(int64_t c, int cx, int cy, int cz, const Geo<T> &g,
                                                      const T *__restrict__ P, const T *__restrict__ Plo) {
    const int idx[3] = {cx, cy, cz};
    const int64_t stride[3] = {1, g.nb[0], (int64_t)g.nb[0] * g.nb[1]};
    GradLoads<T> r;
    r.hi[0] = P[c];
    r.lo[0] = Plo[c];
#pragma unroll
    for (int a = 0; a < 3; ++a) {
        const int64_t kl = idx[a] > 0 ? c - stride[a] : c, kh = idx[a] < g.nb[a] - 1 ? c + stride[a] : c;
        r.hi[1 + 2 * a] = P[kl];
        r.lo[1 + 2 * a] = Plo[kl];
        r.hi[2 + 2 * a] = P[kh];
        r.lo[2 + 2 * a] = Plo[kh];
    }
    return r;
}

template <typename T>
__device__ __forceinline__ void write_gradient(const GradLoads<T> &v, int64_t c, int cx, int cy, int cz,
                                               const Geo<T> &g, T *__restrict__ G) {
    const int idx[3] = {cx, cy, cz};
    const double p0 = (double)v.hi[0] + (double)v.lo[0];
#pragma unroll
    for (int a = 0; a < 3; ++a) {
        const double pl = (double)v.hi[1 + 2 * a] + (double)v.lo[1 + 2 * a];
        const double ph = (double)v.hi[2 + 2 * a] + (double)v.lo[2 + 2 * a];
        const int nax = g.nb[a];
        const double h = (double)g.hb[a];
        double gr;
        if (nax == 1) gr = 0.0;
        else if (idx[a] == 0) gr = (ph - p0) / h;
        else if (idx[a] == nax - 1) gr = (p0 - pl) / h;
        else gr = (ph - pl) / (2.0 * h);
        G[a * g.ncell + c] = (T)gr;
    }
}

// ---------------------------------------------------------------------------
// NGP (containing cell)
// ---------------------------------------------------------------------------
template <typename T, int SM, int MODE>
__global__ __launch_bounds__(kBlock) void k_deposit_ngp(const int32_t *__restrict__ start,
                                                        const vec4<T> *__restrict__ sp,
                                                        const int32_t *__restrict__ perm,
                                                        const T *__restrict__ drag,
                                                        const vec4<T> *__restrict__ src4, int64_t n, Geo<T> g,
                                                        const T *__restrict__ P, const T *__restrict__ Plo,
                                                        T *__restrict__ out, T *__restrict__ out2, T *__restrict__ G,
                                                        double *__restrict__ part, int64_t ps) {
    __shared__ double red[kWavesPerBlock];
    const int64_t c = (int64_t)blockIdx.x * kBlock + threadIdx.x;
    double v[4] = {0.0, 0.0, 0.0, 0.0};
    if (c < g.ncell) {
        const int32_t s = seg_clamp(start[c], n), e = seg_clamp(start[c + 1], n);
        if constexpr (MODE == kSemi) {
            CellSum<T, SM> acc[4];
            for (int32_t p = s; p < e; ++p) {
                int64_t id = perm[p];
                if (id < 0 || id >= n) id = 0;
                const vec4<T> b = src4[id];
                acc[0].add(b.x);
                acc[1].add(b.y);
                acc[2].add(b.z);
                acc[3].add(b.w);
            }
            out[c] = acc[0].value() * g.inv_vb;
            for (int k = 0; k < 3; ++k) out2[k * g.ncell + c] = acc[k + 1].value() * g.inv_vb;
            for (int k = 0; k < 4; ++k) v[k] = (double)(acc[k].value() * g.inv_vb);
        } else if constexpr (MODE == kPhi) {
            CellSum<T, SM> acc;
            for (int32_t p = s; p < e; ++p) acc.add(vol_over_vb(sp[p].w, g.inv_vb));
            out[c] = acc.value();
            v[0] = (double)acc.value();
        } else {
            CellSum<T, SM> ax, ay, az;
            for (int32_t p = s; p < e; ++p) {
                int64_t id = perm[p];
                if (id < 0 || id >= n) id = 0;
                ax.add(drag[3 * id + 0]);
                ay.add(drag[3 * id + 1]);
                az.add(drag[3 * id + 2]);
            }
            const T fx = -ax.value() * g.inv_vb, fy = -ay.value() * g.inv_vb, fz = -az.value() * g.inv_vb;
            out[c] = fx;
            out[g.ncell + c] = fy;
            out[2 * g.ncell + c] = fz;
            v[0] = fx; v[1] = fy; v[2] = fz;
            int cx, cy, cz;
            decode_cell(c, g.nb, cx, cy, cz);
            write_gradient(load_gradient(c, cx, cy, cz, g, P, Plo), c, cx, cy, cz, g, G);
        }
    }
    if constexpr (MODE == kPhi) {
        const double t = block_sum(v[0], red);
        const double m = block_max(v[0], red);
        if (threadIdx.x == 0) {
            part[SL_PHISUM * ps + blockIdx.x] = t;
            part[SL_MAXPHI * ps + blockIdx.x] = m;
        }
    } else if constexpr (MODE == kForce) {
        for (int k = 0; k < 3; ++k) {
            const double t = block_sum(v[k], red);
            if (threadIdx.x == 0) part[(SL_FB + k) * ps + blockIdx.x] = t;
        }
    } else {
        const int slots[4] = {SL_KB, SL_KUB, SL_KUB + 1, SL_KUB + 2};
        for (int k = 0; k < 4; ++k) {
            const double t = block_sum(v[k], red);
            if (threadIdx.x == 0) part[slots[k] * ps + blockIdx.x] = t;
        }
    }
}

// ---------------------------------------------------------------------------
// CIC (trilinear to the 8 nearest bulk cell centres, folded at the walls)
// ---------------------------------------------------------------------------
// Pass 1, k_deposit_rows: one wave per (GS x GS group of source rows in y and
// z, 64-cell x segment), GS = 2 (or 1 on small grids, see deposit_group()).  For
// each source row of its group the wave stages the particles of the source
// cells x0-1 .. x0+64 once (in chunks), with their x-stencil, their weights on
// the three target y-rows and z-rows around the source row and the deposited
// value(s).  Lane x then accumulates, over the particles of source cells x-1,
// x, x+1 in canonical order, the contributions to target cell x of the
// (GS + 2) x (GS + 2) target rows the group reaches (y-rows GS gy - 1 ..
// GS gy + GS, likewise in z), and writes each to the partial slot of its
// (z-group, y-group) offset from the target.
// Pass 2, k_deposit_sum: per target cell, the <= 4 (GS = 2) or <= 9 (GS = 1)
// partials of the source groups it receives from, in ascending (z-group,
// y-group) order.
// With GS = 2 a target row receives from 2 x 2 groups rather than from 3 x 3
// source rows: the partial sums written and read back are 4/9 of one slot per
// source row; GS = 1 trades that for four times the waves.
template <typename T, int MODE> struct RowStage {
    int node[kWavesPerBlock][kChunk];                  // x-stencil nodes lo | hi << 16
    T tx[kWavesPerBlock][kChunk];                      // weight of hi
    T wy[3][kWavesPerBlock][kChunk];                   // weight on target rows y'-1, y', y'+1
    T wz[3][kWavesPerBlock][kChunk];                   // weight on target layers z'-1, z', z'+1
    T val[DepNc<MODE>::value][kWavesPerBlock][kChunk]; // V_p / V_b, F_p, or (beta_p, beta_p u_p)
};

// Row-pass sums s += w v under the step's sum mode: FP32 with Kahan
// compensation (the product w v formed by an FMA against the running
// compensation, so the term is rounded once), FP32 plainly, or widened to FP64
// registers with one FMA per term (both products exact in FP64: every term is
// rounded once at FP64 precision; FP64 FMAs issue at the rate of unpacked FP32
// ones on this chip).  The FP64 mode sums with plain FP64 FMAs (the at most ~100
// terms of a partial sum carry an error below 1e-14 of their magnitudes).
template <typename T, int SM> using RowSum = FmaSum<T, SM>;

template <typename T>
__device__ __forceinline__ void row_weights(const Axis<T> &a, int c, T w[3]) {
    for (int j = 0; j < 3; ++j) {
        const int t = c - 1 + j;
        T v = T(0);
        if (a.lo == t) v += T(1) - a.t;
        if (a.hi == t) v += a.t;
        w[j] = v;
    }
}

// Lowest source group (of G rows) that reaches target row t: floor((t - 1) / G)
// (-1 for t = 0).
template <int G> __device__ __forceinline__ int group_lo(int t) {
    if constexpr (G == 2) return ((t + 1) >> 1) - 1;
    else return t - 1;
}
// Source groups a target row receives from, per axis.
template <int G> struct GroupSlots { static constexpr int value = G == 1 ? 3 : 2; };

// One source row (ys, zs) of the wave's group: row JY, layer KZ of the group.
// Its contributions go to the accumulators [KZ + 0..2][JY + 0..2] (A = G + 2
// target rows per axis).
template <typename T, int SM, int MODE, int JY, int KZ, int A>
__device__ __forceinline__ void deposit_source_row(RowSum<T, SM> (&acc)[A][A][DepNc<MODE>::value],
                                                   RowStage<T, MODE> &st, int w, int lane, int x0, int ys, int zs,
                                                   const int32_t *__restrict__ start, const vec4<T> *__restrict__ sp,
                                                   const int32_t *__restrict__ perm, const T *__restrict__ drag,
                                                   const vec4<T> *__restrict__ src4, int64_t n, const Geo<T> &g) {
    constexpr int NC = DepNc<MODE>::value;
    using W = typename RowSum<T, SM>::W;
    const int nbx = g.nb[0], nby = g.nb[1], nbz = g.nb[2];
    const int x = x0 + lane;
    const int64_t srow = ((int64_t)zs * nby + ys) * nbx;
    const int xa = x0 > 0 ? x0 - 1 : 0;
    const int xb = (x0 + kWave < nbx ? x0 + kWave : nbx - 1);
    const int32_t rs = seg_clamp(start[srow + xa], n), re = seg_clamp(start[srow + xb + 1], n);
    int32_t ls = 0, le = 0;
    if (x < nbx) {
        ls = seg_clamp(start[srow + (x > 0 ? x - 1 : 0)], n);
        le = seg_clamp(start[srow + (x < nbx - 1 ? x + 1 : nbx - 1) + 1], n);
    }
    for (int32_t cs = rs; cs < re; cs += kChunk) {       // wave-uniform loop
        const int32_t m = ((cs + kChunk < re) ? cs + kChunk : re) - cs;
        const int32_t ce = cs + m;
        // Staging: every load of the chunk is issued before any is used, so the
        // random-access value gather through perm costs one round trip per
        // chunk rather than one per 64 particles.
        constexpr int KS = kChunk / kWave;
        vec4<T> q[KS];
        int64_t id[KS];
#pragma unroll
        for (int u = 0; u < KS; ++u) {
            const int k = lane + u * kWave;
            id[u] = 0;
            if (k < m) {
                q[u] = sp[cs + k];
                if constexpr (MODE != kPhi) {
                    const int64_t i = perm[cs + k];
                    id[u] = (i < 0 || i >= n) ? 0 : i;   // perm is a permutation of [0, n)
                }
            }
        }
        T val[KS][NC];
#pragma unroll
        for (int u = 0; u < KS; ++u) {
            if (lane + u * kWave < m) {
                if constexpr (MODE == kForce) {
                    for (int c = 0; c < 3; ++c) val[u][c] = drag[3 * id[u] + c];
                } else if constexpr (MODE == kSemi) {
                    const vec4<T> b = src4[id[u]];
                    val[u][0] = b.x;
                    val[u][1] = b.y;
                    val[u][2] = b.z;
                    val[u][3] = b.w;
                } else {
                    val[u][0] = vol_over_vb(q[u].w, g.inv_vb);
                }
            }
        }
#pragma unroll
        for (int u = 0; u < KS; ++u) {
            const int k = lane + u * kWave;
            if (k < m) {
                const Axis<T> ax = cic_axis(q[u].x, g.sb[0], nbx);
                const Axis<T> ay = cic_axis(q[u].y, g.sb[1], nby);
                const Axis<T> az = cic_axis(q[u].z, g.sb[2], nbz);
                st.node[w][k] = ax.lo | (ax.hi << 16);
                st.tx[w][k] = ax.t;
                T wy[3], wz[3];
                row_weights(ay, ys, wy);
                row_weights(az, zs, wz);
                for (int j = 0; j < 3; ++j) {
                    st.wy[j][w][k] = wy[j];
                    st.wz[j][w][k] = wz[j];
                }
                for (int c = 0; c < NC; ++c) st.val[c][w][k] = val[u][c];
            }
        }
        wave_sync();
        const int32_t b0 = (ls > cs ? ls : cs) - cs, b1 = (le < ce ? le : ce) - cs;
        // Branch-free: the lanes of a wave hold different particles, so a skip
        // of the zero weights (5 of the 9 target rows, a third of the x
        // visits) would diverge and save nothing; their terms add zeros.
        for (int32_t k = b0; k < b1; ++k) {
            const int nd = st.node[w][k];
            const T t = st.tx[w][k];
            T wx = T(0);
            if ((nd & 0xffff) == x) wx += T(1) - t;
            if ((nd >> 16) == x) wx += t;
            W v[NC];
#pragma unroll
            for (int c = 0; c < NC; ++c) v[c] = W(wx) * W(st.val[c][w][k]);
            W wy[3], wz[3];
#pragma unroll
            for (int j = 0; j < 3; ++j) {
                wy[j] = W(st.wy[j][w][k]);
                wz[j] = W(st.wz[j][w][k]);
            }
#pragma unroll
            for (int kz = 0; kz < 3; ++kz) {
#pragma unroll
                for (int jy = 0; jy < 3; ++jy) {
                    const W wyz = wy[jy] * wz[kz];
#pragma unroll
                    for (int c = 0; c < NC; ++c) acc[KZ + kz][JY + jy][c].add(wyz, v[c]);
                }
            }
        }
        wave_sync();
    }
}

template <typename T, int SM, int MODE, int GS>
__global__ __launch_bounds__(kBlock) void k_deposit_rows(const int32_t *__restrict__ start,
                                                         const vec4<T> *__restrict__ sp,
                                                         const int32_t *__restrict__ perm,
                                                         const T *__restrict__ drag,
                                                         const vec4<T> *__restrict__ src4, int64_t n, Geo<T> g,
                                                         T *__restrict__ partial) {
    constexpr int NC = DepNc<MODE>::value, A = GS + 2, S = GroupSlots<GS>::value;
    __shared__ RowStage<T, MODE> st;
    const int w = threadIdx.x / kWave, lane = threadIdx.x % kWave;
    const int nbx = g.nb[0], nby = g.nb[1], nbz = g.nb[2];
    const int nseg = (nbx + kWave - 1) / kWave;
    const int ngy = (nby + GS - 1) / GS, ngz = (nbz + GS - 1) / GS;
    const int64_t nwave = (int64_t)ngy * ngz * nseg;
    const int64_t tile = xcd_tile(blockIdx.x, gridDim.x);
    const int64_t gw = tile * kWavesPerBlock + w;        // (source group, segment)
    if (gw >= nwave) return;                             // wave-uniform; no block barriers below
    const int64_t grp = gw / nseg;
    const int x0 = (int)(gw % nseg) * kWave;
    const int gy = (int)(grp % ngy), gz = (int)(grp / ngy);
    const int x = x0 + lane;
    const int y0 = GS * gy, z0 = GS * gz;
    RowSum<T, SM> acc[A][A][NC];   // [target z - (z0 - 1)][target y - (y0 - 1)][component]
    deposit_source_row<T, SM, MODE, 0, 0, A>(acc, st, w, lane, x0, y0, z0, start, sp, perm, drag, src4, n, g);
    if constexpr (GS == 2) {
        if (y0 + 1 < nby)
            deposit_source_row<T, SM, MODE, 1, 0, A>(acc, st, w, lane, x0, y0 + 1, z0, start, sp, perm, drag, src4, n,
                                                     g);
        if (z0 + 1 < nbz) {
            deposit_source_row<T, SM, MODE, 0, 1, A>(acc, st, w, lane, x0, y0, z0 + 1, start, sp, perm, drag, src4, n,
                                                     g);
            if (y0 + 1 < nby)
                deposit_source_row<T, SM, MODE, 1, 1, A>(acc, st, w, lane, x0, y0 + 1, z0 + 1, start, sp, perm, drag,
                                                         src4, n, g);
        }
    }
    if (x >= nbx) return;
#pragma unroll
    for (int kz = 0; kz < A; ++kz) {
        const int tz = z0 - 1 + kz;
        if (tz < 0 || tz >= nbz) continue;
        const int sz = gz - group_lo<GS>(tz);             // 0 .. S - 1
#pragma unroll
        for (int jy = 0; jy < A; ++jy) {
            const int ty = y0 - 1 + jy;
            if (ty < 0 || ty >= nby) continue;
            const int slot = sz * S + (gy - group_lo<GS>(ty));
            const int64_t tc = ((int64_t)tz * nby + ty) * nbx + x;
#pragma unroll
            for (int c = 0; c < NC; ++c) partial[((int64_t)slot * NC + c) * g.ncell + tc] = T(acc[kz][jy][c].s);
        }
    }
}

template <typename T, int SM, int MODE, int GS>
__global__ __launch_bounds__(kBlock) void k_deposit_sum(const T *__restrict__ partial, Geo<T> g,
                                                        const T *__restrict__ P, const T *__restrict__ Plo,
                                                        T *__restrict__ out, T *__restrict__ out2, T *__restrict__ G,
                                                        double *__restrict__ part, int64_t ps) {
    constexpr int NC = DepNc<MODE>::value, S = GroupSlots<GS>::value;
    __shared__ double red[kWavesPerBlock];
    const int64_t c = (int64_t)blockIdx.x * kBlock + threadIdx.x;
    double v[4] = {0.0, 0.0, 0.0, 0.0};
    if (c < g.ncell) {
        int cx, cy, cz;
        decode_cell(c, g.nb, cx, cy, cz);
        CellSum<T, SM> acc[NC];
        const int gzl = group_lo<GS>(cz), gyl = group_lo<GS>(cy);
        const int ngy = (g.nb[1] + GS - 1) / GS, ngz = (g.nb[2] + GS - 1) / GS;
        GradLoads<T> gl;
        if constexpr (MODE == kForce) gl = load_gradient(c, cx, cy, cz, g, P, Plo);
        // all S x S slots loaded at once (in the partial buffer whether or not
        // their source group exists), then the existing ones summed in order
        T pv[S * S][NC];
#pragma unroll
        for (int slot = 0; slot < S * S; ++slot)
#pragma unroll
            for (int k = 0; k < NC; ++k) pv[slot][k] = partial[((int64_t)slot * NC + k) * g.ncell + c];
#pragma unroll
        for (int sz = 0; sz < S; ++sz)
#pragma unroll
            for (int sy = 0; sy < S; ++sy) {
                const bool has = gzl + sz >= 0 && gzl + sz < ngz && gyl + sy >= 0 && gyl + sy < ngy;
                if (has)
#pragma unroll
                    for (int k = 0; k < NC; ++k) acc[k].add(pv[sz * S + sy][k]);
            }
        if constexpr (MODE == kForce) {
            const T fx = -acc[0].value() * g.inv_vb, fy = -acc[1].value() * g.inv_vb, fz = -acc[2].value() * g.inv_vb;
            out[c] = fx;
            out[g.ncell + c] = fy;
            out[2 * g.ncell + c] = fz;
            v[0] = fx; v[1] = fy; v[2] = fz;
            write_gradient(gl, c, cx, cy, cz, g, G);
        } else if constexpr (MODE == kSemi) {
            out[c] = acc[0].value() * g.inv_vb;
            for (int k = 0; k < 3; ++k) out2[k * g.ncell + c] = acc[k + 1].value() * g.inv_vb;
            for (int k = 0; k < 4; ++k) v[k] = (double)(acc[k].value() * g.inv_vb);
        } else {
            out[c] = acc[0].value();
            v[0] = (double)acc[0].value();
        }
    }
    if constexpr (MODE == kPhi) {
        const double t = block_sum(v[0], red);
        const double m = block_max(v[0], red);
        if (threadIdx.x == 0) {
            part[SL_PHISUM * ps + blockIdx.x] = t;
            part[SL_MAXPHI * ps + blockIdx.x] = m;
        }
    } else if constexpr (MODE == kForce) {
        for (int k = 0; k < 3; ++k) {
            const double t = block_sum(v[k], red);
            if (threadIdx.x == 0) part[(SL_FB + k) * ps + blockIdx.x] = t;
        }
    } else {
        const int slots[4] = {SL_KB, SL_KUB, SL_KUB + 1, SL_KUB + 2};
        for (int k = 0; k < 4; ++k) {
            const double t = block_sum(v[k], red);
            if (threadIdx.x == 0) part[slots[k] * ps + blockIdx.x] = t;
        }
    }
}

// ---------------------------------------------------------------------------
// Host side
// ---------------------------------------------------------------------------
int deposit_blocks(const int nb[3], int64_t ncell, int cic) {
    (void)nb;
    (void)cic;
    return (int)((ncell + kBlock - 1) / kBlock);   // NGP kernel and CIC pass 2
}

static int64_t row_waves(const int nb[3], int G) {
    const int64_t nseg = (nb[0] + kWave - 1) / kWave;
    return (int64_t)((nb[1] + G - 1) / G) * ((nb[2] + G - 1) / G) * nseg;
}

// Source rows per group of the CIC row pass: 2 x 2 (each target row receives 4
// partials) unless that leaves fewer than 4096 waves (four per SIMD of the
// chip), then single rows (9 partials per target, four times the waves).
int deposit_group(const int nb[3]) { return row_waves(nb, 2) < 4096 ? 1 : 2; }

static int row_blocks(const int nb[3], int G) {
    return (int)((row_waves(nb, G) + kWavesPerBlock - 1) / kWavesPerBlock);
}

template <typename T, int SM, int MODE>
static int launch_deposit(const StepArgs<T> &a, T *out, T *out2, hipStream_t st, const char *sum_mark) {
    const int nblk = deposit_blocks(a.g.nb, a.g.ncell, a.cic);
    const vec4<T> *src4 = a.uf4;   // (beta, beta u_p) per particle once the drag has run
    if (a.cic) {
        auto rows_and_sums = [&](auto gc) {
            constexpr int GS = decltype(gc)::value;
            hipLaunchKernelGGL((k_deposit_rows<T, SM, MODE, GS>), dim3(row_blocks(a.g.nb, GS)), dim3(kBlock), 0, st,
                               a.start, a.sp, a.perm, a.drag, src4, a.n, a.g, a.dep_partial);
            a.mk->mark(sum_mark, st);
            hipLaunchKernelGGL((k_deposit_sum<T, SM, MODE, GS>), dim3(nblk), dim3(kBlock), 0, st, a.dep_partial, a.g,
                               a.P, a.Plo, out, out2, a.G, a.part, a.part_stride);
        };
        if (deposit_group(a.g.nb) == 1) rows_and_sums(std::integral_constant<int, 1>{});
        else rows_and_sums(std::integral_constant<int, 2>{});
    } else {
        hipLaunchKernelGGL((k_deposit_ngp<T, SM, MODE>), dim3(nblk), dim3(kBlock), 0, st, a.start, a.sp, a.perm,
                           a.drag, src4, a.n, a.g, a.P, a.Plo, out, out2, a.G, a.part, a.part_stride);
    }
    return nblk;
}

template <typename T, int SM> int launch_deposit_phi(const StepArgs<T> &a, hipStream_t st) {
    return launch_deposit<T, SM, kPhi>(a, a.phi, nullptr, st, "deposit_phi_sum");
}

template <typename T, int SM> int launch_deposit_force(const StepArgs<T> &a, hipStream_t st) {
    return launch_deposit<T, SM, kForce>(a, a.F, nullptr, st, "deposit_force_sum");
}

template <typename T, int SM> int launch_deposit_semi(const StepArgs<T> &a, hipStream_t st) {
    return launch_deposit<T, SM, kSemi>(a, a.K, a.KU, st, "deposit_semi_sum");
}

template int launch_deposit_phi<float, kSumPlain>(const StepArgs<float> &, hipStream_t);
template int launch_deposit_phi<float, kSumKahan>(const StepArgs<float> &, hipStream_t);
template int launch_deposit_phi<float, kSumWide>(const StepArgs<float> &, hipStream_t);
template int launch_deposit_phi<double, kSumPlain>(const StepArgs<double> &, hipStream_t);
template int launch_deposit_force<float, kSumPlain>(const StepArgs<float> &, hipStream_t);
template int launch_deposit_force<float, kSumKahan>(const StepArgs<float> &, hipStream_t);
template int launch_deposit_force<float, kSumWide>(const StepArgs<float> &, hipStream_t);
template int launch_deposit_force<double, kSumPlain>(const StepArgs<double> &, hipStream_t);
template int launch_deposit_semi<float, kSumPlain>(const StepArgs<float> &, hipStream_t);
template int launch_deposit_semi<float, kSumKahan>(const StepArgs<float> &, hipStream_t);
template int launch_deposit_semi<float, kSumWide>(const StepArgs<float> &, hipStream_t);
template int launch_deposit_semi<double, kSumPlain>(const StepArgs<double> &, hipStream_t);

}  // namespace cpl
