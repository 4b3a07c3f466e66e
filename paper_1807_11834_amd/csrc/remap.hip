// remap.hip -- volume-weighted transfer between two rectilinear grids that need
// not be nested (see include/couple_remap.h).
//
// The overlap map |f intersect c| / |c| factors over the axes, so it is kept as
// three 1-D factors: for receiver index i along axis a, the overlapping sender
// indices are the contiguous range first_a[i] .. first_a[i] + cnt_a[i] - 1 with
// weights w_a[off_a[i] + k] = overlap length / receiver cell length.  Built on
// the host in FP64 once per grid pair.  Applied on the device by one of three
// kernels: for a receiver finer than the sender in y and z, tiles of receiver
// rows over an LDS-staged sender slab (k_remap_tile); otherwise receiver rows
// per workgroup (k_remap_rows: the y, z part of the sum over whole sender rows
// with coalesced loads, then the x part from LDS); for sender rows too long for
// LDS, one thread per receiver cell (k_remap: raster order z, y, x).
// In the compensated FP32 mode the tile and per-cell kernels sum in FP64
// registers (each weight x value product of FP32 operands is exact there; one
// FMA per term); the row kernel keeps Kahan-compensated FP32 sums (an FP64
// variant of it, with its partial sums in LDS, measured slower).
// Storing the 3-D map as CSR
// would read more bytes of indices and weights than of field values; the
// factors are a few KB and stay in cache.
#include <algorithm>
#include <type_traits>
#include <cstdint>
#include <cmath>
#include <cstring>
#include <string>
#include <vector>

#include "common.hpp"
#include "couple_remap.h"

using namespace cpl;

namespace {

struct Axis1D {
    int32_t *first = nullptr;   // [nd] first overlapping sender index
    int32_t *cnt = nullptr;     // [nd] number of overlapping sender cells
    int32_t *off = nullptr;     // [nd] offset of the weights
    void *w = nullptr;          // [nnz] T weights
    int64_t nnz = 0;
};

template <typename T> struct RemapArgs {
    const int32_t *first[3], *cnt[3], *off[3];
    const T *w[3];
    int ns[3], nd[3];
    int64_t nsrc, ndst;
};

// Sums of weight x value under the map's sum mode (SumMode): W is the type the
// weights and values are widened to.
template <typename T, int SM> using SumT = typename FmaSum<T, SM>::W;

template <typename T, int SM>
__global__ __launch_bounds__(kBlock) void k_remap(RemapArgs<T> r, const T *__restrict__ src, T *__restrict__ dst) {
    const int64_t nblk = gridDim.x;
    const int64_t c = xcd_tile(blockIdx.x, nblk) * kBlock + threadIdx.x;
    if (c >= r.ndst) return;
    const T *__restrict__ s = src + (int64_t)blockIdx.y * r.nsrc;
    const int i = (int)(c % r.nd[0]), j = (int)((c / r.nd[0]) % r.nd[1]),
              k = (int)(c / ((int64_t)r.nd[0] * r.nd[1]));
    const int fx = r.first[0][i], nx = r.cnt[0][i], ox = r.off[0][i];
    const int fy = r.first[1][j], ny = r.cnt[1][j], oy = r.off[1][j];
    const int fz = r.first[2][k], nz = r.cnt[2][k], oz = r.off[2][k];
    const int64_t sx = r.ns[0], sxy = (int64_t)r.ns[0] * r.ns[1];
    using W = SumT<T, SM>;
    FmaSum<T, SM> acc;
    for (int kz = 0; kz < nz; ++kz) {
        const T wz = r.w[2][oz + kz];
        for (int ky = 0; ky < ny; ++ky) {
            const T wyz = wz * r.w[1][oy + ky];
            const T *__restrict__ row = s + (int64_t)(fz + kz) * sxy + (int64_t)(fy + ky) * sx + fx;
            for (int kx = 0; kx < nx; ++kx) acc.add(W(wyz * r.w[0][ox + kx]), W(row[kx]));
        }
    }
    dst[(int64_t)blockIdx.y * r.ndst + c] = acc.value();
}

// Receiver rows (y, z) of one field per workgroup, grid-strided over the rows.
// A row's y and z factors are the same for the whole workgroup: the (z, y)
// sender rows it overlaps and their weights wz * wy are tabulated in LDS (up to
// kMaxQ at a time), then every sender x of the slab is summed over those rows
// -- each thread issues its kMaxQ loads together -- giving r(x_s) in LDS; then
// each receiver x sums its overlapping r values with the x weights.  Sum
// order: (z, y) in raster order, then x.
constexpr int kMaxQ = 16;

template <typename T, int SM>
__global__ __launch_bounds__(kBlock) void k_remap_rows(RemapArgs<T> r, const T *__restrict__ src,
                                                       T *__restrict__ dst) {
    // both compensated modes run Kahan in T here: FP64 sums of the sixteen
    // rows in flight per thread ran three times slower
    constexpr int SMR = SM == kSumWide ? (int)kSumKahan : SM;
    extern __shared__ __align__(16) unsigned char lds_raw[];
    T *row = reinterpret_cast<T *>(lds_raw);
    __shared__ int64_t qoff[kMaxQ];
    __shared__ T qw[kMaxQ];
    const int64_t nrow = (int64_t)r.nd[1] * r.nd[2];
    const T *__restrict__ s = src + (int64_t)blockIdx.y * r.nsrc;
    const int nsx = r.ns[0];
    const int64_t sxy = (int64_t)r.ns[0] * r.ns[1];
    const int64_t first_row = xcd_tile(blockIdx.x, gridDim.x);
    for (int64_t rr = first_row; rr < nrow; rr += gridDim.x) {    // uniform over the workgroup
        const int j = (int)(rr % r.nd[1]), k = (int)(rr / r.nd[1]);
        const int fy = r.first[1][j], ny = r.cnt[1][j], oy = r.off[1][j];
        const int fz = r.first[2][k], nz = r.cnt[2][k], oz = r.off[2][k];
        const int nq = ny * nz;
        for (int q0 = 0; q0 < nq; q0 += kMaxQ) {
            const int mq = nq - q0 < kMaxQ ? nq - q0 : kMaxQ;
            if (threadIdx.x < mq) {
                const int q = q0 + threadIdx.x, kz = q / ny, ky = q % ny;
                qoff[threadIdx.x] = (int64_t)(fz + kz) * sxy + (int64_t)(fy + ky) * nsx;
                qw[threadIdx.x] = r.w[2][oz + kz] * r.w[1][oy + ky];
            }
            __syncthreads();
            for (int xs = threadIdx.x; xs < nsx; xs += kBlock) {
                T v[kMaxQ];
#pragma unroll
                for (int q = 0; q < kMaxQ; ++q) v[q] = q < mq ? s[qoff[q] + xs] : T(0);
                using W = SumT<T, SMR>;
                FmaSum<T, SMR> acc;
                if (q0 > 0) acc.s = W(row[xs]);   // continue the partial sum of earlier rows
#pragma unroll
                for (int q = 0; q < kMaxQ; ++q)
                    if (q < mq) acc.add(W(qw[q]), W(v[q]));
                row[xs] = acc.value();
            }
            __syncthreads();
        }
        T *__restrict__ out = dst + (int64_t)blockIdx.y * r.ndst + rr * r.nd[0];
        for (int xd = threadIdx.x; xd < r.nd[0]; xd += kBlock) {
            const int fx = r.first[0][xd], nx = r.cnt[0][xd], ox = r.off[0][xd];
            using W = SumT<T, SMR>;
            FmaSum<T, SMR> acc;
            for (int kx = 0; kx < nx; ++kx) acc.add(W(r.w[0][ox + kx]), W(row[fx + kx]));
            out[xd] = acc.value();
        }
        __syncthreads();   // the row buffer is reused by the next row
    }
}

// A tile of kTileJ x kTileK receiver rows (y, z) of one field per workgroup,
// for receivers finer than the sender in y and z.  The sender slab under the
// tile (its overlapping y and z rows, whole x extent) is staged in LDS with
// coalesced loads; every slab row is then transferred along x into a second LDS
// buffer (rx, receiver x resolution); finally each receiver cell sums its
// (z, y) overlaps of rx, whose offsets and weights are tabulated per receiver
// row of the tile.  Sum order: x within each sender row, then (z, y) in raster
// order.  Loop positions advance incrementally: no integer divisions per
// element.
constexpr int kTileJ = 8, kTileK = 8;
constexpr int kTileRows = kTileJ * kTileK;
constexpr int kMaxX = 4;       // x factors held in registers (longer ranges read them in the loop)
constexpr int kMaxTerms = 4;   // (z, y) terms of a receiver row in the table: a receiver cell no
                               // larger than the sender cells it meets overlaps at most 2 x 2
                               // sender rows; rows with more terms read the factors directly

template <typename T> using Vec4NT = T __attribute__((ext_vector_type(4)));

template <typename T, int SM>
__global__ __launch_bounds__(kBlock) void k_remap_tile(RemapArgs<T> r, const T *__restrict__ src,
                                                       T *__restrict__ dst, bool vec4) {
    using W = SumT<T, SM>;
    extern __shared__ __align__(16) unsigned char lds_raw[];
    __shared__ int32_t toff[kTileRows][kMaxTerms];   // rx offset of each term of a receiver row
    __shared__ W tw[kTileRows][kMaxTerms];           // its weight wz * wy
    __shared__ int32_t tn[kTileRows];                // number of terms
    __shared__ int32_t tjk[kTileRows][2];            // the row's receiver (j, k)
    __shared__ int64_t orow[kTileRows];              // the row's offset in the receiver field
    const int tny = (r.nd[1] + kTileJ - 1) / kTileJ;
    const int64_t t = xcd_tile(blockIdx.x, gridDim.x);
    const int j0 = (int)(t % tny) * kTileJ, k0 = (int)(t / tny) * kTileK;
    const int j1 = j0 + kTileJ < r.nd[1] ? j0 + kTileJ : r.nd[1];
    const int k1 = k0 + kTileK < r.nd[2] ? k0 + kTileK : r.nd[2];
    const int nj = j1 - j0, nk = k1 - k0;
    const int ys0 = r.first[1][j0], ys1 = r.first[1][j1 - 1] + r.cnt[1][j1 - 1];
    const int zs0 = r.first[2][k0], zs1 = r.first[2][k1 - 1] + r.cnt[2][k1 - 1];
    const int Ys = ys1 - ys0, nsx = r.ns[0], ndx = r.nd[0];
    const int nrows = (zs1 - zs0) * Ys;   // sender rows of the slab
    T *slab = reinterpret_cast<T *>(lds_raw);
    T *rx = slab + (((size_t)nrows * nsx + 3) & ~(size_t)3);   // 16-byte aligned
    const int64_t sxy = (int64_t)r.ns[0] * r.ns[1];
    const T *__restrict__ s = src + (int64_t)blockIdx.y * r.nsrc;
    // the term table, one thread per receiver row of the tile (row = kk * nj + jj)
    if (threadIdx.x < nj * nk) {
        const int jj = threadIdx.x % nj, kk = threadIdx.x / nj;
        const int j = j0 + jj, k = k0 + kk;
        const int fz = r.first[2][k], nz = r.cnt[2][k], oz = r.off[2][k];
        const int fy = r.first[1][j], ny = r.cnt[1][j], oy = r.off[1][j];
        tn[threadIdx.x] = nz * ny;
        tjk[threadIdx.x][0] = j;
        tjk[threadIdx.x][1] = k;
        orow[threadIdx.x] = ((int64_t)k * r.nd[1] + j) * ndx;
        if (nz * ny <= kMaxTerms) {
            int q = 0;
            for (int kz = 0; kz < nz; ++kz)
                for (int ky = 0; ky < ny; ++ky, ++q) {
                    toff[threadIdx.x][q] = ((fz + kz - zs0) * Ys + (fy + ky - ys0)) * ndx;
                    tw[threadIdx.x][q] = W(r.w[2][oz + kz] * r.w[1][oy + ky]);
                }
        }
    }
    // stage the slab, x fastest, then slab rows (y fastest, then z)
    {
        int x = threadIdx.x % nsx, row = threadIdx.x / nsx;
        int yy = row % Ys, zz = row / Ys;
        const int dx = kBlock % nsx, drow = kBlock / nsx;
        while (row < nrows) {
            slab[(size_t)row * nsx + x] = s[(int64_t)(zs0 + zz) * sxy + (int64_t)(ys0 + yy) * nsx + x];
            x += dx;
            int d = drow;
            if (x >= nsx) {
                x -= nsx;
                ++d;
            }
            row += d;
            yy += d;
            if (yy >= Ys) {
                zz += yy / Ys;
                yy %= Ys;
            }
        }
    }
    __syncthreads();
    // x transfer of every slab row; each thread keeps the x factor of its
    // receiver columns in registers
    for (int xd = threadIdx.x; xd < ndx; xd += kBlock) {
        const int fx = r.first[0][xd], nx = r.cnt[0][xd], ox = r.off[0][xd];
        W wx[kMaxX];
#pragma unroll
        for (int q = 0; q < kMaxX; ++q) wx[q] = q < nx ? W(r.w[0][ox + q]) : W(0);
        for (int row = 0; row < nrows; ++row) {
            const T *sr = slab + (size_t)row * nsx + fx;
            FmaSum<T, SM> acc;
            if (nx <= kMaxX) {
#pragma unroll
                for (int q = 0; q < kMaxX; ++q)
                    if (q < nx) acc.add(wx[q], W(sr[q]));
            } else {
                for (int kx = 0; kx < nx; ++kx) acc.add(W(r.w[0][ox + kx]), W(sr[kx]));
            }
            rx[(size_t)row * ndx + xd] = acc.value();
        }
    }
    __syncthreads();
    // (z, y) overlaps of each receiver cell; the (large, write-once) receiver
    // field is stored non-temporally.  With vec4 set (receiver rows a multiple
    // of 4 long, 16-byte aligned output) a thread forms 4 neighbouring cells of
    // a row and stores them with one vector store.  Work items run over
    // (tile row, x / width).
    T *__restrict__ out = dst + (int64_t)blockIdx.y * r.ndst;
    const int Wd = vec4 ? 4 : 1, nxw = ndx / Wd;
    const int ntr = nj * nk;
    int xw = threadIdx.x % nxw, tr = threadIdx.x / nxw;
    const int dxw = kBlock % nxw, dtr = kBlock / nxw;
    while (tr < ntr) {
        const int xd = xw * Wd;
        const int n = tn[tr];
        FmaSum<T, SM> acc[4];
        auto term = [&](W w, const T *p) {
            if (vec4) {
                const Vec4NT<T> v = *reinterpret_cast<const Vec4NT<T> *>(p);
                acc[0].add(w, W(v.x));
                acc[1].add(w, W(v.y));
                acc[2].add(w, W(v.z));
                acc[3].add(w, W(v.w));
            } else {
                acc[0].add(w, W(p[0]));
            }
        };
        if (n <= kMaxTerms) {
            for (int q = 0; q < n; ++q) term(tw[tr][q], rx + toff[tr][q] + xd);
        } else {
            const int j = tjk[tr][0], k = tjk[tr][1];
            const int fz = r.first[2][k], nz = r.cnt[2][k], oz = r.off[2][k];
            const int fy = r.first[1][j], ny = r.cnt[1][j], oy = r.off[1][j];
            for (int kz = 0; kz < nz; ++kz)
                for (int ky = 0; ky < ny; ++ky)
                    term(W(r.w[2][oz + kz] * r.w[1][oy + ky]), rx + ((fz + kz - zs0) * Ys + (fy + ky - ys0)) * ndx + xd);
        }
        T *o = out + orow[tr] + xd;
        if (vec4) {
            const Vec4NT<T> v = {acc[0].value(), acc[1].value(), acc[2].value(), acc[3].value()};
            __builtin_nontemporal_store(v, reinterpret_cast<Vec4NT<T> *>(o));
        } else {
            __builtin_nontemporal_store(acc[0].value(), o);
        }
        xw += dxw;
        int d = dtr;
        if (xw >= nxw) {
            xw -= nxw;
            ++d;
        }
        tr += d;
    }
}

// Tiles whose sender slab and x-transferred rows take up to this many bytes of
// LDS use k_remap_tile when the receiver is finer than the sender in y and z.
constexpr size_t kTileLdsBytes = 96 * 1024;

// Sender rows up to this many bytes are staged whole in LDS by k_remap_rows;
// longer rows take k_remap.
constexpr size_t kRowLdsBytes = 60 * 1024;

}  // namespace

struct couple_remap {
    int32_t ns[3], nd[3];
    int32_t precision;
    size_t tile_slab_rows;   // most sender (y, z) rows under one receiver tile (0: tile kernel not used)
    Axis1D ax[3];
    std::string err;
};

static thread_local std::string g_remap_init_err;

static int rfail(couple_remap *r, int code, const std::string &msg) {
    if (r) r->err = msg;
    else g_remap_init_err = msg;
    return code;
}

static void remap_release(couple_remap *r) {
    for (int a = 0; a < 3; ++a) {
        void *p[] = {r->ax[a].first, r->ax[a].cnt, r->ax[a].off, r->ax[a].w};
        for (void *q : p)
            if (q) (void)hipFree(q);
        r->ax[a] = Axis1D{};
    }
}

static std::string check_grid(const int32_t n[3], const double *nodes, const char *name) {
    int64_t cells = 1;
    const double *x = nodes;
    for (int a = 0; a < 3; ++a) {
        if (n[a] < 1) return std::string(name) + ": cells per axis must be >= 1";
        cells *= n[a];
        if (cells >= (int64_t(1) << 31)) return std::string(name) + ": too many cells (must be < 2^31)";
        for (int i = 0; i <= n[a]; ++i)
            if (!std::isfinite(x[i])) return std::string(name) + ": node coordinates must be finite";
        for (int i = 0; i < n[a]; ++i)
            if (!(x[i + 1] > x[i])) return std::string(name) + ": node coordinates must increase strictly";
        x += n[a] + 1;
    }
    return "";
}

// 1-D factor along one axis: receiver cells [xd_i, xd_{i+1}] against sender
// cells [xs_j, xs_{j+1}], weights = overlap length / receiver length.
static void build_axis(const double *xs, int ns, const double *xd, int nd, std::vector<int32_t> &first,
                       std::vector<int32_t> &cnt, std::vector<int32_t> &off, std::vector<double> &w) {
    first.assign(nd, 0);
    cnt.assign(nd, 0);
    off.assign(nd, 0);
    w.clear();
    int j = 0;
    for (int i = 0; i < nd; ++i) {
        const double lo = xd[i], hi = xd[i + 1], len = hi - lo;
        while (j < ns - 1 && xs[j + 1] <= lo) ++j;   // first sender cell ending after lo
        off[i] = (int32_t)w.size();
        first[i] = j;
        int c = 0;
        for (int jj = j; jj < ns && xs[jj] < hi; ++jj) {
            const double ov = std::fmin(hi, xs[jj + 1]) - std::fmax(lo, xs[jj]);
            if (ov <= 0.0) {
                if (c == 0) first[i] = jj + 1;   // touches only: not part of the range
                continue;
            }
            w.push_back(ov / len);
            ++c;
        }
        cnt[i] = c;
    }
}

template <typename X> static bool dalloc_copy(X **p, const void *host, size_t bytes) {
    void *q = nullptr;
    if (hipMalloc(&q, bytes ? bytes : 16) != hipSuccess) {
        (void)hipGetLastError();
        *p = nullptr;
        return false;
    }
    if (bytes && hipMemcpy(q, host, bytes, hipMemcpyHostToDevice) != hipSuccess) {
        (void)hipGetLastError();
        (void)hipFree(q);
        *p = nullptr;
        return false;
    }
    *p = static_cast<X *>(q);
    return true;
}

extern "C" int couple_remap_init(const int32_t src_n[3], const double *src_nodes, const int32_t dst_n[3],
                                 const double *dst_nodes, int32_t precision, couple_remap **out) {
    if (!out) return rfail(nullptr, COUPLE_EINVAL, "couple_remap_init: NULL output");
    *out = nullptr;
    if (!src_n || !src_nodes || !dst_n || !dst_nodes) return rfail(nullptr, COUPLE_EINVAL, "couple_remap_init: NULL grid");
    if (!(precision == COUPLE_FP64 || precision == COUPLE_FP32_WIDE || precision == COUPLE_FP32_NAIVE ||
          precision == COUPLE_FP32_KAHAN))
        return rfail(nullptr, COUPLE_EINVAL, "couple_remap_init: unknown precision");
    std::string e = check_grid(src_n, src_nodes, "sender grid");
    if (e.empty()) e = check_grid(dst_n, dst_nodes, "receiver grid");
    if (!e.empty()) return rfail(nullptr, COUPLE_EINVAL, "couple_remap_init: " + e);
    const double *xs = src_nodes, *xd = dst_nodes;
    for (int a = 0; a < 3; ++a) {
        // a 1-D factor has at most src_n + dst_n - 1 entries (one per interval
        // of the merged node sequence); its offsets are 32-bit
        if ((int64_t)src_n[a] + dst_n[a] >= (int64_t(1) << 31))
            return rfail(nullptr, COUPLE_EINVAL, "couple_remap_init: too many cells along an axis");
        const double L = xs[src_n[a]] - xs[0], tol = 1e-12 * L;
        if (std::fabs(xs[0] - xd[0]) > tol || std::fabs(xs[src_n[a]] - xd[dst_n[a]]) > tol)
            return rfail(nullptr, COUPLE_EINVAL, "couple_remap_init: the grids must span the same box");
        xs += src_n[a] + 1;
        xd += dst_n[a] + 1;
    }
    couple_remap *r = new (std::nothrow) couple_remap();
    if (!r) return rfail(nullptr, COUPLE_ENOMEM, "couple_remap_init: host allocation failed");
    for (int a = 0; a < 3; ++a) {
        r->ns[a] = src_n[a];
        r->nd[a] = dst_n[a];
    }
    r->precision = precision;
    xs = src_nodes;
    xd = dst_nodes;
    bool ok = true;
    size_t span[3] = {0, 0, 0};   // most sender indices under kTileJ (y) / kTileK (z) receiver indices
    bool finer[3] = {true, true, true};
    for (int a = 0; a < 3 && ok; ++a) {
        std::vector<int32_t> first, cnt, off;
        std::vector<double> w;
        build_axis(xs, src_n[a], xd, dst_n[a], first, cnt, off, w);
        const int tile = a == 2 ? kTileK : kTileJ;
        for (int i0 = 0; i0 < dst_n[a]; i0 += tile) {
            const int i1 = std::min(i0 + tile, dst_n[a]);
            span[a] = std::max(span[a], (size_t)(first[i1 - 1] + cnt[i1 - 1] - first[i0]));
        }
        finer[a] = dst_n[a] > src_n[a];
        r->ax[a].nnz = (int64_t)w.size();
        const size_t nd = (size_t)dst_n[a];
        ok = dalloc_copy(&r->ax[a].first, first.data(), nd * 4) && dalloc_copy(&r->ax[a].cnt, cnt.data(), nd * 4) &&
             dalloc_copy(&r->ax[a].off, off.data(), nd * 4);
        if (ok) {
            if (precision == COUPLE_FP64) {
                ok = dalloc_copy(&r->ax[a].w, w.data(), w.size() * sizeof(double));
            } else {
                std::vector<float> wf(w.begin(), w.end());
                ok = dalloc_copy(&r->ax[a].w, wf.data(), wf.size() * sizeof(float));
            }
        }
        xs += src_n[a] + 1;
        xd += dst_n[a] + 1;
    }
    r->tile_slab_rows = (finer[1] && finer[2]) ? span[1] * span[2] : 0;
    if (!ok) {
        remap_release(r);
        delete r;
        return rfail(nullptr, COUPLE_ENOMEM, "couple_remap_init: device allocation failed");
    }
    *out = r;
    return COUPLE_OK;
}

template <typename T, int SM>
static hipError_t launch_remap(const couple_remap *r, const void *src, void *dst, int nfields, hipStream_t st) {
    RemapArgs<T> a;
    a.nsrc = a.ndst = 1;
    for (int k = 0; k < 3; ++k) {
        a.first[k] = r->ax[k].first;
        a.cnt[k] = r->ax[k].cnt;
        a.off[k] = r->ax[k].off;
        a.w[k] = static_cast<const T *>(r->ax[k].w);
        a.ns[k] = r->ns[k];
        a.nd[k] = r->nd[k];
        a.nsrc *= r->ns[k];
        a.ndst *= r->nd[k];
    }
    const size_t lds = sizeof(T) * (size_t)r->ns[0];
    const size_t tile_lds =
        sizeof(T) * (((r->tile_slab_rows * (size_t)r->ns[0] + 3) & ~(size_t)3) + r->tile_slab_rows * r->nd[0]);   // slab + rx
    bool tile_ok = r->tile_slab_rows > 0 && tile_lds <= kTileLdsBytes;
    if (tile_ok && tile_lds > 64 * 1024) {
        // more than 64 KB of dynamic LDS per workgroup must be allowed explicitly
        tile_ok = hipFuncSetAttribute(reinterpret_cast<const void *>(&k_remap_tile<T, SM>),
                                      hipFuncAttributeMaxDynamicSharedMemorySize, (int)tile_lds) == hipSuccess;
        if (!tile_ok) (void)hipGetLastError();
    }
    if (tile_ok) {
        const int64_t ntile = (int64_t)((r->nd[1] + kTileJ - 1) / kTileJ) * ((r->nd[2] + kTileK - 1) / kTileK);
        const bool vec4 = r->nd[0] % 4 == 0 && reinterpret_cast<uintptr_t>(dst) % (4 * sizeof(T)) == 0;
        hipLaunchKernelGGL((k_remap_tile<T, SM>), dim3((unsigned)ntile, (unsigned)nfields), dim3(kBlock), tile_lds,
                           st, a, static_cast<const T *>(src), static_cast<T *>(dst), vec4);
    } else if (lds <= kRowLdsBytes) {
        // enough workgroups to fill the chip several times over, each looping
        // over rows (a row is a small amount of work when the receiver is finer)
        const int64_t nrow = (int64_t)r->nd[1] * r->nd[2];
        const int64_t per_field = std::max<int64_t>(1, std::min<int64_t>(nrow, 8192 / nfields + 1));
        hipLaunchKernelGGL((k_remap_rows<T, SM>), dim3((unsigned)per_field, (unsigned)nfields), dim3(kBlock), lds,
                           st, a, static_cast<const T *>(src), static_cast<T *>(dst));
    } else {
        const int64_t nblk = (a.ndst + kBlock - 1) / kBlock;
        hipLaunchKernelGGL((k_remap<T, SM>), dim3((unsigned)nblk, (unsigned)nfields), dim3(kBlock), 0, st, a,
                           static_cast<const T *>(src), static_cast<T *>(dst));
    }
    return hipGetLastError();
}

extern "C" int couple_remap_apply(couple_remap *r, const void *src, void *dst, int32_t nfields, void *stream) {
    if (!r) return rfail(nullptr, COUPLE_EINVAL, "couple_remap_apply: NULL map");
    if (!src || !dst) return rfail(r, COUPLE_EINVAL, "couple_remap_apply: NULL field");
    if (nfields < 1 || nfields > 64) return rfail(r, COUPLE_EINVAL, "couple_remap_apply: nfields must be in [1, 64]");
    const size_t fsz = r->precision == COUPLE_FP64 ? 8 : 4;
    const size_t bs = fsz * (size_t)nfields * (size_t)r->ns[0] * r->ns[1] * r->ns[2];
    const size_t bd = fsz * (size_t)nfields * (size_t)r->nd[0] * r->nd[1] * r->nd[2];
    const char *ps = static_cast<const char *>(src), *pd = static_cast<const char *>(dst);
    if (ps < pd + bd && pd < ps + bs) return rfail(r, COUPLE_EINVAL, "couple_remap_apply: src and dst overlap");
    (void)hipGetLastError();
    hipStream_t st = static_cast<hipStream_t>(stream);
    hipError_t e;
    if (r->precision == COUPLE_FP64) e = launch_remap<double, kSumPlain>(r, src, dst, nfields, st);
    else if (r->precision == COUPLE_FP32_WIDE) e = launch_remap<float, kSumWide>(r, src, dst, nfields, st);
    else if (r->precision == COUPLE_FP32_KAHAN) e = launch_remap<float, kSumKahan>(r, src, dst, nfields, st);
    else e = launch_remap<float, kSumPlain>(r, src, dst, nfields, st);
    if (e != hipSuccess) return rfail(r, COUPLE_EHIP, std::string("couple_remap_apply: launch failed: ") + hipGetErrorString(e));
    return COUPLE_OK;
}

extern "C" int couple_remap_info(const couple_remap *r, int64_t nnz_axis[3], int64_t *nnz_total) {
    if (!r) return COUPLE_EINVAL;
    if (nnz_axis)
        for (int a = 0; a < 3; ++a) nnz_axis[a] = r->ax[a].nnz;
    if (nnz_total) {
        // the 3-D map has, per receiver cell, the product of its three ranges
        *nnz_total = r->ax[0].nnz * r->ax[1].nnz * r->ax[2].nnz;
    }
    return COUPLE_OK;
}

extern "C" int couple_remap_free(couple_remap *r) {
    if (!r) return COUPLE_OK;
    remap_release(r);
    delete r;
    return COUPLE_OK;
}

extern "C" const char *couple_remap_last_error(const couple_remap *r) {
    return r ? r->err.c_str() : g_remap_init_err.c_str();
}
