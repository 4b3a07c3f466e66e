// sample.hpp -- interpolation of bulk and fine fields at a particle (internal).
#pragma once
#include <type_traits>

#include "common.hpp"
#include "launch.hpp"

namespace cpl {

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

// Values at x-nodes lo and hi (hi == lo + 1, or hi == lo at a wall) of one row
// of n >= 2 values, from one 8-byte load of the pair that contains them.
template <typename T> struct Pair2;
template <> struct Pair2<float> { typedef float __attribute__((ext_vector_type(2), aligned(4))) type; };
template <> struct Pair2<double> { typedef double __attribute__((ext_vector_type(2), aligned(8))) type; };

template <typename T>
__device__ __forceinline__ void load_pair(const T *__restrict__ row, int lo, int hi, T &vlo, T &vhi) {
    const int base = (hi != lo) ? lo : (lo == 0 ? 0 : lo - 1);
    const typename Pair2<T>::type v = *reinterpret_cast<const typename Pair2<T>::type *>(row + base);
    vlo = (lo == base) ? v.x : v.y;
    vhi = (hi == base) ? v.x : v.y;
}

// Trilinear value of a cell-centred field from its 4 (y, z) rows of x-pairs.
template <typename T>
__device__ __forceinline__ T trilin_pairs(const T *__restrict__ f, const Axis<T> &ax, const Axis<T> &ay,
                                          const Axis<T> &az, int nx, int64_t nxy) {
    if (nx == 1) return trilin(f, ax, ay, az, nx, nxy);
    const int64_t zl = az.lo * nxy, zh = az.hi * nxy, yl = (int64_t)ay.lo * nx, yh = (int64_t)ay.hi * nx;
    T a0, a1, b0, b1, c0, c1, d0, d1;
    load_pair(f + zl + yl, ax.lo, ax.hi, a0, a1);
    load_pair(f + zl + yh, ax.lo, ax.hi, b0, b1);
    load_pair(f + zh + yl, ax.lo, ax.hi, c0, c1);
    load_pair(f + zh + yh, ax.lo, ax.hi, d0, d1);
    const T sx = T(1) - ax.t, sy = T(1) - ay.t, sz = T(1) - az.t;
    const T e0 = sy * (sx * a0 + ax.t * a1) + ay.t * (sx * b0 + ax.t * b1);
    const T e1 = sy * (sx * c0 + ax.t * c1) + ay.t * (sx * d0 + ax.t * d1);
    return sz * e0 + az.t * e1;
}

// Trilinear interpolation of the fine-grid velocity at the clamped position q.
template <typename T>
__device__ __forceinline__ void fine_velocity(const vec4<T> &q, const StepArgs<T> &a, T &ux, T &uy, T &uz) {
    const Geo<T> &g = a.g;
    const Axis<T> fx = cic_axis(q.x, g.sf[0], g.nf[0]);
    const Axis<T> fy = cic_axis(q.y, g.sf[1], g.nf[1]);
    const Axis<T> fz = cic_axis(q.z, g.sf[2], g.nf[2]);
    const int nx = g.nf[0];
    const int64_t nxy = (int64_t)g.nf[0] * g.nf[1];
    ux = trilin_pairs(a.fine[0], fx, fy, fz, nx, nxy);
    uy = trilin_pairs(a.fine[1], fx, fy, fz, nx, nxy);
    uz = trilin_pairs(a.fine[2], fx, fy, fz, nx, nxy);
}

// Void fraction at one particle (clamped position q.xyz): eps_p = sum_c w_pc
// (1 - phi_c), the transpose of the deposition weights.  In the FP32 modes,
// where the particle solid fraction exceeds phi_fp64 (near close packing), phi_p
// and 1 - phi_p are formed in FP64 from the same eight bulk values.
template <typename T> __device__ __forceinline__ T eps_at(const vec4<T> &q, const StepArgs<T> &a) {
    const Geo<T> &g = a.g;
    const T *__restrict__ phi = a.phi;
    T eps;
    if (a.cic) {
        const Axis<T> bx = cic_axis(q.x, g.sb[0], g.nb[0]);
        const Axis<T> by = cic_axis(q.y, g.sb[1], g.nb[1]);
        const Axis<T> bz = cic_axis(q.z, g.sb[2], g.nb[2]);
        const int nx = g.nb[0];
        const int64_t nxy = (int64_t)g.nb[0] * g.nb[1];
        T f000, f001, f010, f011, f100, f101, f110, f111;
        if (nx >= 2) {
            const int64_t zl = bz.lo * nxy, zh = bz.hi * nxy, yl = (int64_t)by.lo * nx, yh = (int64_t)by.hi * nx;
            load_pair(phi + zl + yl, bx.lo, bx.hi, f000, f001);
            load_pair(phi + zl + yh, bx.lo, bx.hi, f010, f011);
            load_pair(phi + zh + yl, bx.lo, bx.hi, f100, f101);
            load_pair(phi + zh + yh, bx.lo, bx.hi, f110, f111);
        } else {
            const int64_t zl = bz.lo * nxy, zh = bz.hi * nxy, yl = (int64_t)by.lo * nx, yh = (int64_t)by.hi * nx;
            f000 = f001 = phi[zl + yl];
            f010 = f011 = phi[zl + yh];
            f100 = f101 = phi[zh + yl];
            f110 = f111 = phi[zh + yh];
        }
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
            eps = (T)(1.0 - ph);
        } else {
            eps = T(1) - phi_p;
        }
    } else {
        const int ix = cell_axis(q.x, g.sb[0], g.nb[0]);
        const int iy = cell_axis(q.y, g.sb[1], g.nb[1]);
        const int iz = cell_axis(q.z, g.sb[2], g.nb[2]);
        eps = T(1) - phi[ix + (int64_t)g.nb[0] * (iy + (int64_t)g.nb[1] * iz)];  // exact for phi in [1/2, 1]
    }
    return eps;
}

// Void fraction and fluid velocity at one particle: eps_at() and u_f by source
// src (0: trilinear on the fine grid, 1: trilinear on the restricted bulk
// velocity, otherwise 0).
template <typename T>
__device__ __forceinline__ vec4<T> sample_one(const vec4<T> &q, const StepArgs<T> &a, int src) {
    const Geo<T> &g = a.g;
    vec4<T> s;
    s.w = eps_at(q, a);
    if (src == 0) {
        fine_velocity(q, a, s.x, s.y, s.z);
    } else if (src == 1) {
        const Axis<T> bx = cic_axis(q.x, g.sb[0], g.nb[0]);
        const Axis<T> by = cic_axis(q.y, g.sb[1], g.nb[1]);
        const Axis<T> bz = cic_axis(q.z, g.sb[2], g.nb[2]);
        const int nx = g.nb[0];
        const int64_t nxy = (int64_t)g.nb[0] * g.nb[1];
        s.x = trilin_pairs(a.U, bx, by, bz, nx, nxy);
        s.y = trilin_pairs(a.U + g.ncell, bx, by, bz, nx, nxy);
        s.z = trilin_pairs(a.U + 2 * g.ncell, bx, by, bz, nx, nxy);
    } else {
        s.x = s.y = s.z = T(0);   // the drag kernel takes u_f from uf_given
    }
    return s;
}

}  // namespace cpl
