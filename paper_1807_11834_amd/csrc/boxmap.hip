// boxmap.hip -- transfer between grids of arbitrary axis-aligned cells through a
// CSR overlap map built once on the host (see include/couple_boxmap.h).
//
//   k_boxmap   one thread per receiver row, fields in groups of four: the row's
//              (column, weight) pairs are read once per group and the sender
//              values gathered (neighbouring rows touch neighbouring senders, so
//              the gathers mostly hit the caches); rows dealt to the XCDs in
//              chunks so that neighbouring rows share an L2.
#include <algorithm>
#include <cmath>
#include <string>
#include <thread>
#include <type_traits>
#include <vector>

#include "common.hpp"
#include "couple_boxmap.h"

namespace cpl {

// One thread per receiver row: sum_j w_j src[col_j] for up to NF fields at a
// time, under the map's sum mode (SumMode).
template <typename T, int SM, int NF>
__global__ __launch_bounds__(kBlock) void k_boxmap(const int64_t *__restrict__ rowptr, const int32_t *__restrict__ col,
                                                   const T *__restrict__ w, int64_t nr, int64_t ns,
                                                   const T *__restrict__ src, T *__restrict__ dst, int nfields) {
    using S = typename FmaSum<T, SM>::W;
    const int64_t tile = xcd_tile(blockIdx.x, gridDim.x);
    const int64_t r = tile * kBlock + threadIdx.x;
    if (r >= nr) return;
    const int64_t b = rowptr[r], e = rowptr[r + 1];
    for (int f0 = 0; f0 < nfields; f0 += NF) {
        FmaSum<T, SM> acc[NF];
        for (int64_t j = b; j < e; ++j) {
            const int64_t c = col[j];
            const S wj = S(w[j]);
#pragma unroll
            for (int k = 0; k < NF; ++k)
                if (f0 + k < nfields) acc[k].add(wj, S(src[(int64_t)(f0 + k) * ns + c]));
        }
#pragma unroll
        for (int k = 0; k < NF; ++k)
            if (f0 + k < nfields) dst[(int64_t)(f0 + k) * nr + r] = acc[k].value();
    }
}

}  // namespace cpl

using namespace cpl;

struct couple_boxmap {
    int64_t ns = 0, nr = 0, nnz = 0, max_row = 0;
    int32_t precision = 0;
    int64_t *rowptr = nullptr;   // [nr + 1]
    int32_t *col = nullptr;      // [nnz]
    void *w = nullptr;           // [nnz], field precision
    std::string err;
};

static thread_local std::string g_boxmap_err;

static int bfail(couple_boxmap *m, int code, const std::string &msg) {
    if (m) m->err = msg;
    else g_boxmap_err = msg;
    return code;
}

static double ov1(double a0, double a1, double b0, double b1) {
    const double lo = a0 > b0 ? a0 : b0, hi = a1 < b1 ? a1 : b1;
    return hi > lo ? hi - lo : 0.0;
}

static const char *check_boxes(int64_t n, const double *b) {
    for (int64_t c = 0; c < n; ++c)
        for (int a = 0; a < 3; ++a) {
            const double lo = b[6 * c + 2 * a], hi = b[6 * c + 2 * a + 1];
            if (!(std::isfinite(lo) && std::isfinite(hi) && lo < hi)) return "boxes need finite bounds with lower < upper";
        }
    return nullptr;
}

// Candidate senders of every receiver from a uniform bucket grid over the
// sender cells (about one sender per bucket), then the exact FP64 overlaps;
// rows are built in parallel over receiver chunks and concatenated in order.
static bool build_csr(int64_t ns, const double *sb, int64_t nr, const double *rb, std::vector<int64_t> &rowptr,
                      std::vector<int32_t> &col, std::vector<double> &val, std::string &why) {
    double lo[3], hi[3];
    for (int a = 0; a < 3; ++a) {
        lo[a] = sb[2 * a];
        hi[a] = sb[2 * a + 1];
    }
    double vol = 0.0;
    for (int64_t c = 0; c < ns; ++c)
        for (int a = 0; a < 3; ++a) {
            lo[a] = std::min(lo[a], sb[6 * c + 2 * a]);
            hi[a] = std::max(hi[a], sb[6 * c + 2 * a + 1]);
        }
    for (int64_t c = 0; c < ns; ++c)
        vol += (sb[6 * c + 1] - sb[6 * c]) * (sb[6 * c + 3] - sb[6 * c + 2]) * (sb[6 * c + 5] - sb[6 * c + 4]);
    const double h = std::cbrt(vol / (double)ns);
    int64_t nb[3];
    for (int a = 0; a < 3; ++a) {
        const double m = std::ceil((hi[a] - lo[a]) / h);
        nb[a] = (int64_t)std::min(std::max(m, 1.0), 4096.0);
    }
    while (nb[0] * nb[1] * nb[2] > 4 * ns + 64)
        for (int a = 0; a < 3; ++a) nb[a] = std::max<int64_t>(1, nb[a] / 2);
    double bh[3];
    for (int a = 0; a < 3; ++a) bh[a] = (hi[a] - lo[a]) / (double)nb[a];
    auto range = [&](const double *box, int a, int64_t &i0, int64_t &i1) {
        i0 = (int64_t)std::floor((box[2 * a] - lo[a]) / bh[a]);
        i1 = (int64_t)std::floor((box[2 * a + 1] - lo[a]) / bh[a]);
        i0 = std::min(std::max<int64_t>(i0, 0), nb[a] - 1);
        i1 = std::min(std::max<int64_t>(i1, 0), nb[a] - 1);
    };
    const int64_t nbk = nb[0] * nb[1] * nb[2];
    std::vector<int64_t> bstart(nbk + 1, 0);
    std::vector<int32_t> bitems;   // sender ids per bucket (CSR over buckets)
    for (int pass = 0; pass < 2; ++pass) {
        std::vector<int64_t> fill;
        if (pass == 1) {
            for (int64_t k = 0; k < nbk; ++k) bstart[k + 1] += bstart[k];
            bitems.assign(bstart[nbk], 0);
            fill.assign(bstart.begin(), bstart.end() - 1);
        }
        for (int64_t c = 0; c < ns; ++c) {
            int64_t r0[3], r1[3];
            for (int a = 0; a < 3; ++a) range(sb + 6 * c, a, r0[a], r1[a]);
            for (int64_t k = r0[2]; k <= r1[2]; ++k)
                for (int64_t j = r0[1]; j <= r1[1]; ++j)
                    for (int64_t i = r0[0]; i <= r1[0]; ++i) {
                        const int64_t bk = i + nb[0] * (j + nb[1] * k);
                        if (pass == 0) bstart[bk + 1] += 1;
                        else bitems[fill[bk]++] = (int32_t)c;
                    }
        }
        if (pass == 1) {
            // rows, in parallel over receiver chunks
            int nth = (int)std::min<unsigned>(16, std::max(1u, std::thread::hardware_concurrency()));
            if (nr < 4096) nth = 1;
            struct Part {
                std::vector<int64_t> len;
                std::vector<int32_t> col;
                std::vector<double> val;
            };
            std::vector<Part> parts(nth);
            auto work = [&](int t) {
                const int64_t r_begin = nr * t / nth, r_end = nr * (t + 1) / nth;
                Part &P = parts[t];
                std::vector<int32_t> cand;
                for (int64_t r = r_begin; r < r_end; ++r) {
                    const double *R = rb + 6 * r;
                    int64_t r0[3], r1[3];
                    for (int a = 0; a < 3; ++a) range(R, a, r0[a], r1[a]);
                    cand.clear();
                    for (int64_t k = r0[2]; k <= r1[2]; ++k)
                        for (int64_t j = r0[1]; j <= r1[1]; ++j)
                            for (int64_t i = r0[0]; i <= r1[0]; ++i) {
                                const int64_t bk = i + nb[0] * (j + nb[1] * k);
                                for (int64_t q = bstart[bk]; q < bstart[bk + 1]; ++q) cand.push_back(bitems[q]);
                            }
                    std::sort(cand.begin(), cand.end());
                    cand.erase(std::unique(cand.begin(), cand.end()), cand.end());
                    const double vr = (R[1] - R[0]) * (R[3] - R[2]) * (R[5] - R[4]);
                    int64_t len = 0;
                    for (int32_t c : cand) {
                        const double *S = sb + 6 * (int64_t)c;
                        const double ox = ov1(R[0], R[1], S[0], S[1]);
                        if (ox == 0.0) continue;
                        const double oy = ov1(R[2], R[3], S[2], S[3]);
                        if (oy == 0.0) continue;
                        const double oz = ov1(R[4], R[5], S[4], S[5]);
                        if (oz == 0.0) continue;
                        P.col.push_back(c);
                        P.val.push_back(ox * oy * oz / vr);
                        ++len;
                    }
                    P.len.push_back(len);
                }
            };
            std::vector<std::thread> th;
            for (int t = 1; t < nth; ++t) th.emplace_back(work, t);
            work(0);
            for (auto &x : th) x.join();
            int64_t total = 0;
            for (auto &P : parts) total += (int64_t)P.col.size();
            if (total >= (int64_t(1) << 31) - 1) {
                why = "the map would hold 2^31 or more nonzeros";
                return false;
            }
            rowptr.assign(nr + 1, 0);
            col.reserve(total);
            val.reserve(total);
            int64_t r = 0;
            for (auto &P : parts) {
                for (int64_t l : P.len) {
                    rowptr[r + 1] = rowptr[r] + l;
                    ++r;
                }
                col.insert(col.end(), P.col.begin(), P.col.end());
                val.insert(val.end(), P.val.begin(), P.val.end());
            }
        }
    }
    return true;
}

extern "C" int couple_boxmap_init(int64_t ns, const double *sender_boxes, int64_t nr, const double *receiver_boxes,
                                  int32_t precision, couple_boxmap **out) {
    if (!out || !sender_boxes || !receiver_boxes) return bfail(nullptr, COUPLE_EINVAL, "couple_boxmap_init: NULL argument");
    *out = nullptr;
    const int64_t lim = (int64_t(1) << 31) - 1;
    if (ns < 1 || nr < 1 || ns >= lim || nr >= lim)
        return bfail(nullptr, COUPLE_EINVAL, "couple_boxmap_init: cell counts must be in [1, 2^31 - 1)");
    if (!(precision == COUPLE_FP64 || precision == COUPLE_FP32_WIDE || precision == COUPLE_FP32_NAIVE ||
          precision == COUPLE_FP32_KAHAN))
        return bfail(nullptr, COUPLE_EINVAL, "couple_boxmap_init: unknown precision");
    if (const char *w = check_boxes(ns, sender_boxes))
        return bfail(nullptr, COUPLE_EINVAL, std::string("couple_boxmap_init: sender ") + w);
    if (const char *w = check_boxes(nr, receiver_boxes))
        return bfail(nullptr, COUPLE_EINVAL, std::string("couple_boxmap_init: receiver ") + w);
    std::vector<int64_t> rowptr;
    std::vector<int32_t> col;
    std::vector<double> val;
    std::string why;
    if (!build_csr(ns, sender_boxes, nr, receiver_boxes, rowptr, col, val, why))
        return bfail(nullptr, COUPLE_EINVAL, "couple_boxmap_init: " + why);
    couple_boxmap *m = new (std::nothrow) couple_boxmap();
    if (!m) return bfail(nullptr, COUPLE_ENOMEM, "couple_boxmap_init: host allocation failed");
    m->ns = ns;
    m->nr = nr;
    m->nnz = (int64_t)col.size();
    m->precision = precision;
    for (int64_t r = 0; r < nr; ++r) m->max_row = std::max(m->max_row, rowptr[r + 1] - rowptr[r]);
    const size_t wsz = precision == COUPLE_FP64 ? sizeof(double) : sizeof(float);
    const size_t nz = (size_t)std::max<int64_t>(m->nnz, 1);
    bool ok = hipMalloc(&m->rowptr, sizeof(int64_t) * (nr + 1)) == hipSuccess &&
              hipMalloc(&m->col, sizeof(int32_t) * nz) == hipSuccess && hipMalloc(&m->w, wsz * nz) == hipSuccess;
    if (ok) {
        std::vector<float> wf;
        const void *wsrc = val.data();
        if (wsz == sizeof(float)) {
            wf.assign(val.begin(), val.end());
            wsrc = wf.data();
        }
        ok = hipMemcpy(m->rowptr, rowptr.data(), sizeof(int64_t) * (nr + 1), hipMemcpyHostToDevice) == hipSuccess &&
             (m->nnz == 0 ||
              (hipMemcpy(m->col, col.data(), sizeof(int32_t) * m->nnz, hipMemcpyHostToDevice) == hipSuccess &&
               hipMemcpy(m->w, wsrc, wsz * m->nnz, hipMemcpyHostToDevice) == hipSuccess));
    }
    if (!ok) {
        (void)hipGetLastError();
        if (m->rowptr) (void)hipFree(m->rowptr);
        if (m->col) (void)hipFree(m->col);
        if (m->w) (void)hipFree(m->w);
        delete m;
        return bfail(nullptr, COUPLE_ENOMEM, "couple_boxmap_init: device allocation or upload failed");
    }
    *out = m;
    return COUPLE_OK;
}

template <typename T, int SM>
static void launch_boxmap(const couple_boxmap *m, const void *src, void *dst, int nf, hipStream_t st) {
    const int64_t blocks = (m->nr + kBlock - 1) / kBlock;
    hipLaunchKernelGGL((k_boxmap<T, SM, 4>), dim3((unsigned)blocks), dim3(kBlock), 0, st, m->rowptr, m->col,
                       (const T *)m->w, m->nr, m->ns, (const T *)src, (T *)dst, nf);
}

extern "C" int couple_boxmap_apply(couple_boxmap *m, const void *src, void *dst, int32_t nfields, void *stream) {
    if (!m) return bfail(nullptr, COUPLE_EINVAL, "couple_boxmap_apply: NULL map");
    if (!src || !dst) return bfail(m, COUPLE_EINVAL, "couple_boxmap_apply: NULL field");
    if (nfields < 1 || nfields > 64) return bfail(m, COUPLE_EINVAL, "couple_boxmap_apply: nfields must be in [1, 64]");
    hipStream_t st = static_cast<hipStream_t>(stream);
    (void)hipGetLastError();
    if (m->precision == COUPLE_FP64) launch_boxmap<double, kSumPlain>(m, src, dst, nfields, st);
    else if (m->precision == COUPLE_FP32_WIDE) launch_boxmap<float, kSumWide>(m, src, dst, nfields, st);
    else if (m->precision == COUPLE_FP32_KAHAN) launch_boxmap<float, kSumKahan>(m, src, dst, nfields, st);
    else launch_boxmap<float, kSumPlain>(m, src, dst, nfields, st);
    const hipError_t e = hipGetLastError();
    if (e != hipSuccess) return bfail(m, COUPLE_EHIP, std::string("couple_boxmap_apply: launch failed: ") + hipGetErrorString(e));
    return COUPLE_OK;
}

extern "C" int couple_boxmap_info(const couple_boxmap *m, int64_t *nnz, int64_t *max_row) {
    if (!m || !nnz || !max_row) return COUPLE_EINVAL;
    *nnz = m->nnz;
    *max_row = m->max_row;
    return COUPLE_OK;
}

extern "C" int couple_boxmap_free(couple_boxmap *m) {
    if (!m) return COUPLE_OK;
    if (m->rowptr) (void)hipFree(m->rowptr);
    if (m->col) (void)hipFree(m->col);
    if (m->w) (void)hipFree(m->w);
    delete m;
    return COUPLE_OK;
}

extern "C" const char *couple_boxmap_last_error(const couple_boxmap *m) {
    return m ? m->err.c_str() : g_boxmap_err.c_str();
}
