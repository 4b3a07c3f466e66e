// stages.hip -- deposition, restriction, particle gather + drag, momentum
// source, prolongation and the FP64 conservation sums of one coupling step.
//
// Kernel order on the caller's stream (after binning/sorting, sort.hip):
//
//   k_gather       sorted copies of the particle data: sp = (x,y,z,d) clamped
//                  into the box, sv = velocity; FP64 partial sums of V_p.
//   k_deposit_phi  one thread per bulk cell gathers the particles of the 27
//                  (CIC) or 1 (NGP) neighbouring cells from the sorted order, in
//                  ascending (cell, id), into a compensated FP32 (or FP64) sum:
//                  phi_c = sum_p w_pc V_p / V_b.  Deterministic, no atomics.
//   k_restrict     one thread per bulk cell streams its r^3 fine children of
//                  u, v, w, p (one 16-byte row load per (z, y) child row for
//                  r = 4) and writes the compensated averages U, P.  With the
//                  fine-grid velocity source the same wave then evaluates the
//                  drag of the particles in its 64 cells while their fine rows
//                  are still in L2 (the fine lookup costs no extra HBM pass).
//   k_particles    drag for the bulk-velocity and given-velocity sources.
//   k_deposit_force F_fpi,c = -(1/V_b) sum_p w_pc F_p (same gather as phi) and
//                  the bulk pressure gradient.
//   k_prolong      one thread per bulk cell writes its r^3 fine children of
//                  eps and F_fpi: conservative trilinear T_f + D_c with the
//                  27-neighbour values held in registers.
//   k_diag         fixed-order reduction of the per-workgroup FP64 partials.
#include <type_traits>

#include "common.hpp"
#include "launch.hpp"

namespace cpl {

// ---------------------------------------------------------------------------
// Row loads of R consecutive fine values (16-byte vector loads where possible)
// ---------------------------------------------------------------------------
template <typename T, int R> struct Row { T v[R]; };

template <typename T, int R> __device__ __forceinline__ Row<T, R> load_row(const T *__restrict__ p) {
    Row<T, R> r;
    if constexpr (std::is_same<T, float>::value && R == 4) {
        float4 q = *reinterpret_cast<const float4 *>(p);
        r.v[0] = q.x; r.v[1] = q.y; r.v[2] = q.z; r.v[3] = q.w;
    } else if constexpr (std::is_same<T, float>::value && R == 2) {
        float2 q = *reinterpret_cast<const float2 *>(p);
        r.v[0] = q.x; r.v[1] = q.y;
    } else if constexpr (std::is_same<T, double>::value && R == 4) {
        double2 a = reinterpret_cast<const double2 *>(p)[0];
        double2 b = reinterpret_cast<const double2 *>(p)[1];
        r.v[0] = a.x; r.v[1] = a.y; r.v[2] = b.x; r.v[3] = b.y;
    } else if constexpr (std::is_same<T, double>::value && R == 2) {
        double2 a = *reinterpret_cast<const double2 *>(p);
        r.v[0] = a.x; r.v[1] = a.y;
    } else {
        for (int k = 0; k < R; ++k) r.v[k] = p[k];
    }
    return r;
}

template <typename T, int R> __device__ __forceinline__ void store_row(T *__restrict__ p, const T *v) {
    if constexpr (std::is_same<T, float>::value && R == 4) {
        *reinterpret_cast<float4 *>(p) = make_float4(v[0], v[1], v[2], v[3]);
    } else if constexpr (std::is_same<T, float>::value && R == 2) {
        *reinterpret_cast<float2 *>(p) = make_float2(v[0], v[1]);
    } else if constexpr (std::is_same<T, double>::value && R == 4) {
        reinterpret_cast<double2 *>(p)[0] = make_double2(v[0], v[1]);
        reinterpret_cast<double2 *>(p)[1] = make_double2(v[2], v[3]);
    } else if constexpr (std::is_same<T, double>::value && R == 2) {
        *reinterpret_cast<double2 *>(p) = make_double2(v[0], v[1]);
    } else {
        for (int k = 0; k < R; ++k) p[k] = v[k];
    }
}

// ---------------------------------------------------------------------------
// k_gather: sorted particle copies
// ---------------------------------------------------------------------------
template <typename T>
__global__ __launch_bounds__(kBlock) void k_gather(const int32_t *__restrict__ perm, const T *__restrict__ pos,
                                                   const T *__restrict__ vel, const T *__restrict__ diam,
                                                   int64_t n, Geo<T> g, vec4<T> *__restrict__ sp,
                                                   vec4<T> *__restrict__ sv, double *__restrict__ part_vtot) {
    __shared__ double red[kWavesPerBlock];
    int64_t i = (int64_t)blockIdx.x * kBlock + threadIdx.x;
    double vp = 0.0;
    if (i < n) {
        int64_t p = perm[i];
        if (p < 0 || p >= n) p = 0;   // perm is a permutation of [0, n); guards the loads
        int o = 0;
        vec4<T> q;
        q.x = clamp_coord(pos[3 * p + 0], g.L[0], o);
        q.y = clamp_coord(pos[3 * p + 1], g.L[1], o);
        q.z = clamp_coord(pos[3 * p + 2], g.L[2], o);
        q.w = diam[p];
        sp[i] = q;
        vec4<T> v;
        v.x = vel[3 * p + 0];
        v.y = vel[3 * p + 1];
        v.z = vel[3 * p + 2];
        v.w = T(0);
        sv[i] = v;
        double d = (double)q.w;
        vp = kPi * d * d * d / 6.0;
    }
    double t = block_sum(vp, red);
    if (threadIdx.x == 0) part_vtot[blockIdx.x] = t;
}

// ---------------------------------------------------------------------------
// Deposition gathers.  The particles that can touch bulk cell c sit in the 27
// cells c + {-1,0,1}^3 (a CIC particle reaches its containing cell and one
// neighbour per axis).  For each (dz, dy) the 1-3 cells along x are adjacent in
// the sorted order, so the thread walks 9 contiguous runs in ascending cell
// order, each in ascending id: the canonical (cell, id) order.
// ---------------------------------------------------------------------------
// Segment bounds read from `start` (a prefix sum over [0, n]) clamped into
// [0, n]: a no-op for a consistent `start`, it keeps every load in bounds.
__device__ __forceinline__ int32_t seg_lo(int32_t v, int64_t n) { return v < 0 ? 0 : (v > n ? (int32_t)n : v); }
__device__ __forceinline__ int32_t seg_hi(int32_t v, int64_t n) { return v < 0 ? 0 : (v > n ? (int32_t)n : v); }

template <typename T>
__device__ __forceinline__ T cic_weight_to(const vec4<T> &q, const Geo<T> &g, int cx, int cy, int cz) {
    Axis<T> ax = cic_axis(q.x, g.sb[0], g.nb[0]);
    Axis<T> ay = cic_axis(q.y, g.sb[1], g.nb[1]);
    Axis<T> az = cic_axis(q.z, g.sb[2], g.nb[2]);
    return axis_weight(ax, cx) * axis_weight(ay, cy) * axis_weight(az, cz);
}

template <typename T> __device__ __forceinline__ T vol_over_vb(T d, T inv_vb) {
    return (T(kPi / 6.0) * d * d * d) * inv_vb;
}

__device__ __forceinline__ void decode_cell(int64_t c, const int nb[3], int &cx, int &cy, int &cz) {
    cx = (int)(c % nb[0]);
    cy = (int)((c / nb[0]) % nb[1]);
    cz = (int)(c / ((int64_t)nb[0] * nb[1]));
}

template <typename T, bool CIC, bool KAHAN>
__global__ __launch_bounds__(kBlock) void k_deposit_phi(const int32_t *__restrict__ start,
                                                        const vec4<T> *__restrict__ sp, int64_t n, Geo<T> g,
                                                        T *__restrict__ phi, double *__restrict__ part,
                                                        int64_t ps) {
    __shared__ double red[kWavesPerBlock];
    int64_t c = (int64_t)blockIdx.x * kBlock + threadIdx.x;
    double v = 0.0;
    if (c < g.ncell) {
        int cx, cy, cz;
        decode_cell(c, g.nb, cx, cy, cz);
        Acc<T, KAHAN> acc;
        if constexpr (!CIC) {
            const int32_t s = seg_lo(start[c], n), e = seg_hi(start[c + 1], n);
            for (int32_t p = s; p < e; ++p) acc.add(vol_over_vb(sp[p].w, g.inv_vb));
        } else {
            int xl = cx > 0 ? cx - 1 : 0, xh = cx < g.nb[0] - 1 ? cx + 1 : cx;
            for (int dz = -1; dz <= 1; ++dz) {
                int z = cz + dz;
                if (z < 0 || z >= g.nb[2]) continue;
                for (int dy = -1; dy <= 1; ++dy) {
                    int y = cy + dy;
                    if (y < 0 || y >= g.nb[1]) continue;
                    int64_t row = (int64_t)g.nb[0] * (y + (int64_t)g.nb[1] * z);
                    int32_t s = seg_lo(start[row + xl], n), e = seg_hi(start[row + xh + 1], n);
                    for (int32_t p = s; p < e; ++p) {
                        vec4<T> q = sp[p];
                        T w = cic_weight_to(q, g, cx, cy, cz);
                        if (w != T(0)) acc.add(w * vol_over_vb(q.w, g.inv_vb));
                    }
                }
            }
        }
        phi[c] = acc.s;
        v = (double)acc.s;
    }
    double t = block_sum(v, red);
    double m = block_max(v, red);
    if (threadIdx.x == 0) {
        part[SL_PHISUM * ps + blockIdx.x] = t;
        part[SL_MAXPHI * ps + blockIdx.x] = m;
    }
}

template <typename T, bool CIC, bool KAHAN>
__global__ __launch_bounds__(kBlock) void k_deposit_force(const int32_t *__restrict__ start,
                                                          const vec4<T> *__restrict__ sp,
                                                          const vec4<T> *__restrict__ sf, int64_t n, Geo<T> g,
                                                          const T *__restrict__ P, const T *__restrict__ Plo,
                                                          T *__restrict__ F, T *__restrict__ G,
                                                          double *__restrict__ part, int64_t ps) {
    __shared__ double red[kWavesPerBlock];
    int64_t c = (int64_t)blockIdx.x * kBlock + threadIdx.x;
    double fb[3] = {0.0, 0.0, 0.0};
    if (c < g.ncell) {
        int cx, cy, cz;
        decode_cell(c, g.nb, cx, cy, cz);
        Acc<T, KAHAN> ax, ay, az;
        if constexpr (!CIC) {
            const int32_t s = seg_lo(start[c], n), e = seg_hi(start[c + 1], n);
            for (int32_t p = s; p < e; ++p) {
                vec4<T> f = sf[p];
                ax.add(f.x);
                ay.add(f.y);
                az.add(f.z);
            }
        } else {
            int xl = cx > 0 ? cx - 1 : 0, xh = cx < g.nb[0] - 1 ? cx + 1 : cx;
            for (int dz = -1; dz <= 1; ++dz) {
                int z = cz + dz;
                if (z < 0 || z >= g.nb[2]) continue;
                for (int dy = -1; dy <= 1; ++dy) {
                    int y = cy + dy;
                    if (y < 0 || y >= g.nb[1]) continue;
                    int64_t row = (int64_t)g.nb[0] * (y + (int64_t)g.nb[1] * z);
                    int32_t s = seg_lo(start[row + xl], n), e = seg_hi(start[row + xh + 1], n);
                    for (int32_t p = s; p < e; ++p) {
                        T w = cic_weight_to(sp[p], g, cx, cy, cz);
                        if (w != T(0)) {
                            vec4<T> f = sf[p];
                            ax.add(w * f.x);
                            ay.add(w * f.y);
                            az.add(w * f.z);
                        }
                    }
                }
            }
        }
        T fx = -ax.s * g.inv_vb, fy = -ay.s * g.inv_vb, fz = -az.s * g.inv_vb;
        F[c] = fx;
        F[g.ncell + c] = fy;
        F[2 * g.ncell + c] = fz;
        fb[0] = fx;
        fb[1] = fy;
        fb[2] = fz;
        // bulk pressure gradient: central differences, one-sided at the walls.
        // The difference is taken in FP64 of the compensated pressure hi + lo:
        // differencing the rounded FP32 values alone would lose ulp(P)/h.
        int idx[3] = {cx, cy, cz};
        int64_t stride[3] = {1, g.nb[0], (int64_t)g.nb[0] * g.nb[1]};
        auto pv = [&](int64_t k) { return (double)P[k] + (double)Plo[k]; };
        for (int a = 0; a < 3; ++a) {
            double gr;
            const int nax = g.nb[a];
            const double h = (double)g.hb[a];
            if (nax == 1) gr = 0.0;
            else if (idx[a] == 0) gr = (pv(c + stride[a]) - pv(c)) / h;
            else if (idx[a] == nax - 1) gr = (pv(c) - pv(c - stride[a])) / h;
            else gr = (pv(c + stride[a]) - pv(c - stride[a])) / (2.0 * h);
            G[a * g.ncell + c] = (T)gr;
        }
    }
    for (int a = 0; a < 3; ++a) {
        double t = block_sum(fb[a], red);
        if (threadIdx.x == 0) part[(SL_FB + a) * ps + blockIdx.x] = t;
    }
}

// ---------------------------------------------------------------------------
// Particle stage: void fraction and fluid velocity at the particle, drag
// (Eq. DragLaw with the Di Felice voidage function), optional Euler advection.
// ---------------------------------------------------------------------------
template <typename T>
__device__ __forceinline__ T trilin(const T *__restrict__ f, const Axis<T> &ax, const Axis<T> &ay,
                                    const Axis<T> &az, int64_t nx, int64_t nxy) {
    const int64_t zl = az.lo * nxy, zh = az.hi * nxy, yl = ay.lo * nx, yh = ay.hi * nx;
    const T sx = T(1) - ax.t, sy = T(1) - ay.t, sz = T(1) - az.t;
    T c00 = sx * f[zl + yl + ax.lo] + ax.t * f[zl + yl + ax.hi];
    T c01 = sx * f[zl + yh + ax.lo] + ax.t * f[zl + yh + ax.hi];
    T c10 = sx * f[zh + yl + ax.lo] + ax.t * f[zh + yl + ax.hi];
    T c11 = sx * f[zh + yh + ax.lo] + ax.t * f[zh + yh + ax.hi];
    T c0 = sy * c00 + ay.t * c01;
    T c1 = sy * c10 + ay.t * c11;
    return sz * c0 + az.t * c1;
}

// FP64 re-evaluation of the particle's solid fraction (near close packing).
template <typename T>
__device__ __forceinline__ double phi_at_fp64(const T *__restrict__ phi, const vec4<T> &q, const Geo<T> &g, int cic) {
    if (!cic) {
        int ix = cell_axis(q.x, g.sb[0], g.nb[0]);
        int iy = cell_axis(q.y, g.sb[1], g.nb[1]);
        int iz = cell_axis(q.z, g.sb[2], g.nb[2]);
        return (double)phi[ix + (int64_t)g.nb[0] * (iy + (int64_t)g.nb[1] * iz)];
    }
    double xs[3] = {(double)q.x, (double)q.y, (double)q.z};
    int lo[3], hi[3];
    double t[3];
    for (int a = 0; a < 3; ++a) {
        double gg = xs[a] * (double)g.sb[a] - 0.5;
        double jf = floor(gg);
        t[a] = gg - jf;
        lo[a] = clampi((int)jf, g.nb[a]);
        hi[a] = clampi((int)jf + 1, g.nb[a]);
    }
    double s = 0.0;
    for (int dz = 0; dz < 2; ++dz)
        for (int dy = 0; dy < 2; ++dy)
            for (int dx = 0; dx < 2; ++dx) {
                double w = (dx ? t[0] : 1.0 - t[0]) * (dy ? t[1] : 1.0 - t[1]) * (dz ? t[2] : 1.0 - t[2]);
                int64_t c = (dx ? hi[0] : lo[0]) + (int64_t)g.nb[0] * ((dy ? hi[1] : lo[1]) +
                                                                        (int64_t)g.nb[1] * (dz ? hi[2] : lo[2]));
                s += w * (double)phi[c];
            }
    return s;
}

template <typename T>
__device__ __forceinline__ void particle_step(int64_t i, const StepArgs<T> &a, double acc[4]) {
    const Geo<T> &g = a.g;
    const vec4<T> q = a.sp[i];
    const vec4<T> v = a.sv[i];
    int64_t p = a.perm[i];
    if (p < 0 || p >= a.n) p = 0;   // perm is a permutation of [0, n); guards the stores
    const T d = q.w;

    // solid fraction at the particle: transpose of the deposition weights
    T phi_p;
    if (a.cic) {
        Axis<T> bx = cic_axis(q.x, g.sb[0], g.nb[0]);
        Axis<T> by = cic_axis(q.y, g.sb[1], g.nb[1]);
        Axis<T> bz = cic_axis(q.z, g.sb[2], g.nb[2]);
        phi_p = trilin(a.phi, bx, by, bz, g.nb[0], (int64_t)g.nb[0] * g.nb[1]);
    } else {
        int ix = cell_axis(q.x, g.sb[0], g.nb[0]);
        int iy = cell_axis(q.y, g.sb[1], g.nb[1]);
        int iz = cell_axis(q.z, g.sb[2], g.nb[2]);
        phi_p = a.phi[ix + (int64_t)g.nb[0] * (iy + (int64_t)g.nb[1] * iz)];
    }

    // fluid velocity at the particle
    T uf[3];
    if (a.vel_source == 0) {
        Axis<T> fx = cic_axis(q.x, g.sf[0], g.nf[0]);
        Axis<T> fy = cic_axis(q.y, g.sf[1], g.nf[1]);
        Axis<T> fz = cic_axis(q.z, g.sf[2], g.nf[2]);
        const int64_t nx = g.nf[0], nxy = (int64_t)g.nf[0] * g.nf[1];
        for (int k = 0; k < 3; ++k) uf[k] = trilin(a.fine[k], fx, fy, fz, nx, nxy);
    } else if (a.vel_source == 1) {
        Axis<T> bx = cic_axis(q.x, g.sb[0], g.nb[0]);
        Axis<T> by = cic_axis(q.y, g.sb[1], g.nb[1]);
        Axis<T> bz = cic_axis(q.z, g.sb[2], g.nb[2]);
        const int64_t nx = g.nb[0], nxy = (int64_t)g.nb[0] * g.nb[1];
        for (int k = 0; k < 3; ++k) uf[k] = trilin(a.U + k * g.ncell, bx, by, bz, nx, nxy);
    } else {
        for (int k = 0; k < 3; ++k) uf[k] = a.uf_given[3 * p + k];
    }

    // drag: F = beta (u_f - u_p); beta in the form
    //   1/2 rho_f (pi d^2/4) eps*^(2-chi) (0.63 sqrt|u_r| + 4.8 sqrt(mu_f/(rho_f eps* d)))^2
    // which equals 1/2 C_D rho_f A eps*^(2-chi) |u_r| with C_D = (0.63 + 4.8/sqrt(Re))^2
    // and stays finite as |u_r| -> 0.
    const T ur0 = uf[0] - v.x, ur1 = uf[1] - v.y, ur2 = uf[2] - v.z;
    const T mag = dsqrt(ur0 * ur0 + ur1 * ur1 + ur2 * ur2);
    const bool wide = std::is_same<T, float>::value && phi_p > (T)a.phi_fp64;
    double eps_w = 0.0;
    T e;
    int clamped = 0;
    if (wide) {
        eps_w = 1.0 - phi_at_fp64(a.phi, q, g, a.cic);
        if (eps_w < (double)a.eps_min) {
            eps_w = (double)a.eps_min;
            clamped = 1;
        }
        e = (T)eps_w;
    } else {
        e = T(1) - phi_p;
        if (e < a.eps_min) {
            e = a.eps_min;
            clamped = 1;
        }
    }
    T chi = T(3.7);
    if (mag > T(0)) {
        T re = a.rho_f * e * d * mag / a.mu_f;
        T l = T(1.5) - dlog10(re);
        chi = T(3.7) - T(0.65) * dexp(-l * l * T(0.5));
    }
    T vfac = wide ? (T)pow(eps_w, 2.0 - (double)chi) : dpow(e, T(2) - chi);
    T sq = T(0.63) * dsqrt(mag) + T(4.8) * dsqrt(a.mu_f / (a.rho_f * e * d));
    T area = T(kPi / 4.0) * d * d;
    T beta = T(0.5) * a.rho_f * area * vfac * (sq * sq);
    T F0 = beta * ur0, F1 = beta * ur1, F2 = beta * ur2;

    a.drag[3 * p + 0] = F0;
    a.drag[3 * p + 1] = F1;
    a.drag[3 * p + 2] = F2;
    if (a.beta) a.beta[p] = beta;
    vec4<T> f;
    f.x = F0; f.y = F1; f.z = F2; f.w = T(0);
    a.sf[i] = f;
    acc[0] += (double)F0;
    acc[1] += (double)F1;
    acc[2] += (double)F2;
    acc[3] += clamped;

    if (a.advect) {
        // explicit Euler from the old state, specular reflection at the walls
        const T m = a.rho_p * (T(kPi / 6.0) * d * d * d);
        const T xs[3] = {q.x, q.y, q.z};
        const T us[3] = {v.x, v.y, v.z};
        const T Fs[3] = {F0, F1, F2};
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

template <typename T>
__device__ __forceinline__ void write_particle_partials(const double acc[4], double *part, int64_t ps, double *red) {
    for (int k = 0; k < 3; ++k) {
        double t = block_sum(acc[k], red);
        if (threadIdx.x == 0) part[(SL_FP + k) * ps + blockIdx.x] = t;
    }
    double t = block_sum(acc[3], red);
    if (threadIdx.x == 0) part[SL_NCLAMP * ps + blockIdx.x] = t;
}

// ---------------------------------------------------------------------------
// Restriction fine -> bulk (+ fused fine lookup and drag)
// ---------------------------------------------------------------------------
template <typename T, int R, bool KAHAN, bool FUSED>
__global__ __launch_bounds__(kBlock) void k_restrict(StepArgs<T> a) {
    __shared__ double red[kWavesPerBlock];
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
        for (int f = 0; f < 4; ++f) {
            const T *__restrict__ q = a.fine[f] + base;
            Row<T, R> rows[R][R];
#pragma unroll
            for (int lz = 0; lz < R; ++lz)
#pragma unroll
                for (int ly = 0; ly < R; ++ly) rows[lz][ly] = load_row<T, R>(q + lz * nfxy + ly * nfx);
            Acc<T, KAHAN> acc;
#pragma unroll
            for (int lz = 0; lz < R; ++lz)
#pragma unroll
                for (int ly = 0; ly < R; ++ly)
#pragma unroll
                    for (int lx = 0; lx < R; ++lx) acc.add(rows[lz][ly].v[lx]);
            T val = acc.s * inv;   // 1/R^3 is a power of two: the scaling is exact
            if (f < 3) {
                a.U[f * g.ncell + c] = val;
            } else {
                a.P[c] = val;
                // the compensated sum is s - c: keep -c/R^3 so that the pressure
                // gradient can difference (hi + lo) instead of the rounded hi
                a.Plo[c] = -acc.c * inv;
            }
        }
    }
    if constexpr (FUSED) {
        double acc[4] = {0.0, 0.0, 0.0, 0.0};
        const int w = threadIdx.x / kWave, lane = threadIdx.x % kWave;
        const int64_t c0 = tile * kBlock + (int64_t)w * kWave;
        if (c0 < g.ncell) {
            const int64_t c1 = (c0 + kWave < g.ncell) ? c0 + kWave : g.ncell;
            const int64_t s = seg_lo(a.start[c0], a.n), e = seg_hi(a.start[c1], a.n);
            for (int64_t i = s + lane; i < e; i += kWave) particle_step(i, a, acc);
        }
        write_particle_partials<T>(acc, a.part, a.part_stride, red);
    }
}

template <typename T>
__global__ __launch_bounds__(kBlock) void k_particles(StepArgs<T> a) {
    __shared__ double red[kWavesPerBlock];
    double acc[4] = {0.0, 0.0, 0.0, 0.0};
    const int64_t i = (int64_t)blockIdx.x * kBlock + threadIdx.x;
    if (i < a.n) particle_step(i, a, acc);
    write_particle_partials<T>(acc, a.part, a.part_stride, red);
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

template <typename T, int R>
__global__ __launch_bounds__(kBlock) void k_prolong(StepArgs<T> a) {
    __shared__ double red[kWavesPerBlock];
    const Geo<T> &g = a.g;
    const int64_t tile = xcd_tile(blockIdx.x, gridDim.x);
    const int64_t c = tile * kBlock + threadIdx.x;
    double sums[4] = {0.0, 0.0, 0.0, 0.0};
    if (c < g.ncell) {
        int cx, cy, cz;
        decode_cell(c, g.nb, cx, cy, cz);
        const int64_t nx = g.nb[0], nxy = (int64_t)g.nb[0] * g.nb[1];
        int64_t ox[3] = {(cx > 0 ? cx - 1 : 0), cx, (cx < g.nb[0] - 1 ? cx + 1 : cx)};
        int64_t oy[3] = {(cy > 0 ? cy - 1 : 0) * nx, cy * nx, (cy < g.nb[1] - 1 ? cy + 1 : cy) * nx};
        int64_t oz[3] = {(cz > 0 ? cz - 1 : 0) * nxy, cz * nxy, (cz < g.nb[2] - 1 ? cz + 1 : cz) * nxy};
        const int64_t nfx = g.nf[0], nfxy = (int64_t)g.nf[0] * g.nf[1];
        const int64_t fbase = (int64_t)R * cz * nfxy + (int64_t)R * cy * nfx + (int64_t)R * cx;
#pragma unroll
        for (int f = 0; f < 4; ++f) {
            const T *__restrict__ B = (f == 0) ? a.phi : a.F + (int64_t)(f - 1) * g.ncell;
            T *__restrict__ out = (f == 0) ? a.fine_eps : a.fine_F + (int64_t)(f - 1) * g.nfine;
            T b[3][3][3];
#pragma unroll
            for (int k = 0; k < 3; ++k)
#pragma unroll
                for (int j = 0; j < 3; ++j)
#pragma unroll
                    for (int i = 0; i < 3; ++i) {
                        T v = B[oz[k] + oy[j] + ox[i]];
                        b[k][j][i] = (f == 0) ? T(1) - v : v;
                    }
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
            T Y[3][R][R];
#pragma unroll
            for (int k = 0; k < 3; ++k)
#pragma unroll
                for (int ly = 0; ly < R; ++ly)
#pragma unroll
                    for (int lx = 0; lx < R; ++lx) Y[k][ly][lx] = wsum3<T, R>(ly, X[k][0][lx], X[k][1][lx], X[k][2][lx]);
            double s = 0.0;
#pragma unroll
            for (int lz = 0; lz < R; ++lz)
#pragma unroll
                for (int ly = 0; ly < R; ++ly) {
                    T o[R];
#pragma unroll
                    for (int lx = 0; lx < R; ++lx) {
                        o[lx] = wsum3<T, R>(lz, Y[0][ly][lx], Y[1][ly][lx], Y[2][ly][lx]) + D;
                        s += (double)o[lx];
                    }
                    store_row<T, R>(out + fbase + lz * nfxy + ly * nfx, o);
                }
            sums[f] = s;
        }
    }
    {
        double t = block_sum(sums[0], red);
        if (threadIdx.x == 0) a.part[SL_EPSF * a.part_stride + blockIdx.x] = t;
    }
    for (int k = 0; k < 3; ++k) {
        double t = block_sum(sums[k + 1], red);
        if (threadIdx.x == 0) a.part[(SL_FF + k) * a.part_stride + blockIdx.x] = t;
    }
}

// ---------------------------------------------------------------------------
// Final fixed-order reduction of the per-workgroup partials
// ---------------------------------------------------------------------------
struct DiagSpec {
    int nblk[SL_COUNT];
    double scale[SL_COUNT];
};

__global__ __launch_bounds__(kBlock) void k_diag(const double *__restrict__ part, int64_t ps, DiagSpec spec,
                                                 double *__restrict__ diag) {
    __shared__ double red[kWavesPerBlock];
    for (int s = 0; s < SL_COUNT; ++s) {
        const bool is_max = (s == SL_MAXPHI);
        double v = 0.0;
        for (int j = threadIdx.x; j < spec.nblk[s]; j += kBlock) {
            double x = part[s * ps + j];
            v = is_max ? fmax(v, x) : v + x;
        }
        double t = is_max ? block_max(v, red) : block_sum(v, red);
        if (threadIdx.x == 0) diag[s] = t * spec.scale[s];
        __syncthreads();
    }
}

// ---------------------------------------------------------------------------
// Host dispatch
// ---------------------------------------------------------------------------
template <typename T, int R, bool KAHAN>
static void launch_grid_stages(const StepArgs<T> &a, hipStream_t st) {
    const int64_t cb = (a.g.ncell + kBlock - 1) / kBlock;
    const int64_t pb = (a.n + kBlock - 1) / kBlock;
    const bool fused = (a.vel_source == 0);
    if (fused) {
        a.mk->mark("restrict_lookup_drag", st);
        hipLaunchKernelGGL((k_restrict<T, R, KAHAN, true>), dim3(cb), dim3(kBlock), 0, st, a);
    } else {
        a.mk->mark("restrict", st);
        hipLaunchKernelGGL((k_restrict<T, R, KAHAN, false>), dim3(cb), dim3(kBlock), 0, st, a);
        if (a.n > 0) a.mk->mark("particles", st);
        if (a.n > 0) hipLaunchKernelGGL(k_particles<T>, dim3(pb), dim3(kBlock), 0, st, a);
    }
    a.mk->mark("deposit_force", st);
    if (a.cic)
        hipLaunchKernelGGL((k_deposit_force<T, true, KAHAN>), dim3(cb), dim3(kBlock), 0, st, a.start, a.sp, a.sf,
                           a.n, a.g, a.P, a.Plo, a.F, a.G, a.part, a.part_stride);
    else
        hipLaunchKernelGGL((k_deposit_force<T, false, KAHAN>), dim3(cb), dim3(kBlock), 0, st, a.start, a.sp, a.sf,
                           a.n, a.g, a.P, a.Plo, a.F, a.G, a.part, a.part_stride);
    a.mk->mark("prolong", st);
    hipLaunchKernelGGL((k_prolong<T, R>), dim3(cb), dim3(kBlock), 0, st, a);
}

template <typename T, bool KAHAN> static void launch_by_ratio(const StepArgs<T> &a, hipStream_t st) {
    switch (a.ratio) {
    case 1: launch_grid_stages<T, 1, KAHAN>(a, st); break;
    case 2: launch_grid_stages<T, 2, KAHAN>(a, st); break;
    default: launch_grid_stages<T, 4, KAHAN>(a, st); break;
    }
}

template <typename T> hipError_t launch_stages(const StepArgs<T> &a, hipStream_t st) {
    const int64_t cb = (a.g.ncell + kBlock - 1) / kBlock;
    const int64_t pb = (a.n + kBlock - 1) / kBlock;
    const bool kahan = std::is_same<T, float>::value && a.kahan;
    if (a.n > 0) a.mk->mark("gather", st);
    if (a.n > 0)
        hipLaunchKernelGGL(k_gather<T>, dim3(pb), dim3(kBlock), 0, st, a.perm, a.pos, a.vel, a.diam, a.n, a.g, a.sp,
                           a.sv, a.part + SL_VTOT * a.part_stride);
    a.mk->mark("deposit_phi", st);
    if (a.cic) {
        if (kahan)
            hipLaunchKernelGGL((k_deposit_phi<T, true, true>), dim3(cb), dim3(kBlock), 0, st, a.start, a.sp, a.n, a.g,
                               a.phi, a.part, a.part_stride);
        else
            hipLaunchKernelGGL((k_deposit_phi<T, true, false>), dim3(cb), dim3(kBlock), 0, st, a.start, a.sp, a.n, a.g,
                               a.phi, a.part, a.part_stride);
    } else {
        if (kahan)
            hipLaunchKernelGGL((k_deposit_phi<T, false, true>), dim3(cb), dim3(kBlock), 0, st, a.start, a.sp, a.n, a.g,
                               a.phi, a.part, a.part_stride);
        else
            hipLaunchKernelGGL((k_deposit_phi<T, false, false>), dim3(cb), dim3(kBlock), 0, st, a.start, a.sp, a.n, a.g,
                               a.phi, a.part, a.part_stride);
    }
    if (kahan) launch_by_ratio<T, true>(a, st);
    else launch_by_ratio<T, false>(a, st);

    DiagSpec spec;
    for (int s = 0; s < SL_COUNT; ++s) {
        spec.nblk[s] = (int)cb;
        spec.scale[s] = 1.0;
    }
    spec.nblk[SL_VTOT] = a.n > 0 ? (int)pb : 0;
    spec.nblk[SL_NOUT] = a.n > 0 ? sort_tiles(a.n) : 0;
    const int npart = (a.vel_source == 0) ? (int)cb : (a.n > 0 ? (int)pb : 0);
    for (int k = 0; k < 3; ++k) spec.nblk[SL_FP + k] = npart;
    spec.nblk[SL_NCLAMP] = npart;
    spec.nblk[SL_NFALL] = 0;
    spec.scale[SL_PHISUM] = a.g.vb;
    for (int k = 0; k < 3; ++k) {
        spec.scale[SL_FB + k] = a.g.vb;
        spec.scale[SL_FF + k] = a.g.vf;
    }
    spec.scale[SL_EPSF] = a.g.vf;
    a.mk->mark("diag", st);
    hipLaunchKernelGGL(k_diag, dim3(1), dim3(kBlock), 0, st, a.part, a.part_stride, spec, a.diag);
    a.mk->mark(nullptr, st);
    return hipGetLastError();
}

template hipError_t launch_stages<float>(const StepArgs<float> &, hipStream_t);
template hipError_t launch_stages<double>(const StepArgs<double> &, hipStream_t);

}  // namespace cpl
