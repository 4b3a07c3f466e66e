// part.hip -- the partitioned step: co-located z-slabs, each with its particles,
// its nested fine slab and a one-layer ghost halo, exchanging halos through a
// static sparse communication matrix, distributed or through a root buffer (see
// couple_part_step in include/couple.h).
//
// Per step: owner slab of every particle (k_owner), a stable partition of the
// particles by owner (one radix pass) and their copy into the slabs' frames
// (k_distribute, the z coordinate shifted by the slab origin); the slabs' own
// fine slabs from the input; then, with each slab's coupling phases run on its
// local grid: fine halo -> deposition -> porosity halo (reverse add, forward)
// -> velocity, drag, momentum source -> source halo -> prolongation and sums;
// finally the owned parts of every slab's outputs into the caller's arrays
// (k_collect*), the sums of the slabs' FP64 diagnostics and the maximum solid
// fraction over the assembled grid.
#include <algorithm>
#include <cmath>
#include <cstdio>
#include <string>
#include <vector>

#include "common.hpp"
#include "couple.h"
#include "handle.hpp"
#include "launch.hpp"

namespace cpl {

constexpr int kMaxParts = 64;

struct ZCut {
    int z[kMaxParts + 1];   // slab k owns bulk layers [z[k], z[k + 1])
    int K;
};

template <typename T> struct SlabShift {
    T dz[kMaxParts];            // z of the slab frame's origin in the global frame
    int64_t cell_off[kMaxParts];// global index of the slab grid's first cell
    int64_t poff[kMaxParts];    // first particle of the slab in the concatenated arrays
};

template <typename T>
__global__ __launch_bounds__(kBlock) void k_owner(const T *__restrict__ pos, int64_t n, Geo<T> g, ZCut zc,
                                                  uint32_t *__restrict__ owner) {
    const int64_t i = (int64_t)blockIdx.x * kBlock + threadIdx.x;
    if (i >= n) return;
    int o = 0;
    const T z = clamp_coord(pos[3 * i + 2], g.L[2], o);
    const int cz = cell_axis(z, g.sb[2], g.nb[2]);   // the binning's containing layer
    int k = 0;
    while (k + 1 < zc.K && zc.z[k + 1] <= cz) ++k;
    owner[i] = (uint32_t)k;
}

template <typename T>
__global__ __launch_bounds__(kBlock) void k_distribute(const uint32_t *__restrict__ okey, const uint32_t *__restrict__ ids,
                                                       int64_t n, int K, const T *__restrict__ pos,
                                                       const T *__restrict__ vel, const T *__restrict__ diam,
                                                       SlabShift<T> sh, T *__restrict__ lpos, T *__restrict__ lvel,
                                                       T *__restrict__ ldiam, int32_t *__restrict__ gid) {
    const int64_t i = (int64_t)blockIdx.x * kBlock + threadIdx.x;
    if (i >= n) return;
    int64_t id = ids[i];
    if (id < 0 || id >= n) id = 0;   // ids is a permutation of [0, n)
    int k = (int)okey[i];
    if (k >= K) k = K - 1;
    lpos[3 * i + 0] = pos[3 * id + 0];
    lpos[3 * i + 1] = pos[3 * id + 1];
    lpos[3 * i + 2] = pos[3 * id + 2] - sh.dz[k];   // exact: dz is a multiple of the power-of-two spacing
    for (int c = 0; c < 3; ++c) lvel[3 * i + c] = vel[3 * id + c];
    ldiam[i] = diam[id];
    gid[i] = (int32_t)id;
}

template <typename T>
__global__ __launch_bounds__(kBlock) void k_collect(const uint32_t *__restrict__ okey, const int32_t *__restrict__ gid,
                                                    int64_t n, int K, SlabShift<T> sh, const T *__restrict__ ldrag,
                                                    const T *__restrict__ lbeta, const int32_t *__restrict__ lcell,
                                                    const int32_t *__restrict__ lperm, const T *__restrict__ luf,
                                                    const T *__restrict__ lpos, const T *__restrict__ lvel, int advect,
                                                    T *__restrict__ drag, T *__restrict__ beta, int32_t *__restrict__ cell,
                                                    int32_t *__restrict__ perm, T *__restrict__ uf, T *__restrict__ pos,
                                                    T *__restrict__ vel) {
    const int64_t i = (int64_t)blockIdx.x * kBlock + threadIdx.x;
    if (i >= n) return;
    int k = (int)okey[i];
    if (k >= K) k = K - 1;
    int64_t id = gid[i];
    if (id < 0 || id >= n) id = 0;
    for (int c = 0; c < 3; ++c) drag[3 * id + c] = ldrag[3 * i + c];
    if (beta) beta[id] = lbeta[i];
    if (uf)
        for (int c = 0; c < 3; ++c) uf[3 * id + c] = luf[3 * i + c];
    cell[id] = (int32_t)(lcell[i] + sh.cell_off[k]);
    int64_t j = sh.poff[k] + lperm[i];   // the slab's canonical order, in the global one
    if (j < 0 || j >= n) j = 0;
    perm[i] = gid[j];
    if (advect) {
        pos[3 * id + 0] = lpos[3 * i + 0];
        pos[3 * id + 1] = lpos[3 * i + 1];
        pos[3 * id + 2] = lpos[3 * i + 2] + sh.dz[k];
        for (int c = 0; c < 3; ++c) vel[3 * id + c] = lvel[3 * i + c];
    }
}

// count and start of a slab's owned cells; the last slab also writes start[ncell]
__global__ __launch_bounds__(kBlock) void k_collect_cells(const int32_t *__restrict__ lcount,
                                                          const int32_t *__restrict__ lstart, int64_t m, int32_t poff,
                                                          int last, int32_t *__restrict__ count,
                                                          int32_t *__restrict__ start) {
    const int64_t c = (int64_t)blockIdx.x * kBlock + threadIdx.x;
    if (c >= m) return;
    count[c] = lcount[c];
    start[c] = poff + lstart[c];
    if (last && c == m - 1) start[m] = poff + lstart[m];
}

template <typename T>
__global__ __launch_bounds__(kBlock) void k_add(T *__restrict__ dst, const T *__restrict__ src, int64_t m) {
    const int64_t i = (int64_t)blockIdx.x * kBlock + threadIdx.x;
    if (i < m) dst[i] += src[i];
}

// the slabs' diagnostics added in slab order (maximum solid fraction apart)
__global__ __launch_bounds__(kWave) void k_sum_diags(const double *__restrict__ ld, int K, double *__restrict__ out) {
    const int s = threadIdx.x;
    if (s >= COUPLE_DIAG_LEN || s == COUPLE_DIAG_MAX_PHI) return;
    double t = 0.0;
    for (int k = 0; k < K; ++k) t += ld[(int64_t)k * COUPLE_DIAG_LEN + s];
    out[s] = t;
}

template <typename T>
__global__ __launch_bounds__(kBlock) void k_max1(const T *__restrict__ phi, int64_t m, double *__restrict__ part) {
    __shared__ double red[kWavesPerBlock];
    double v = 0.0;
    for (int64_t i = (int64_t)blockIdx.x * kBlock + threadIdx.x; i < m; i += (int64_t)gridDim.x * kBlock)
        v = fmax(v, (double)phi[i]);
    const double t = block_max(v, red);
    if (threadIdx.x == 0) part[blockIdx.x] = t;
}
__global__ __launch_bounds__(kBlock) void k_max2(const double *__restrict__ part, int m, double *__restrict__ out) {
    __shared__ double red[kWavesPerBlock];
    double v = 0.0;
    for (int i = threadIdx.x; i < m; i += kBlock) v = fmax(v, part[i]);
    const double t = block_max(v, red);
    if (threadIdx.x == 0) out[COUPLE_DIAG_MAX_PHI] = t;
}

}  // namespace cpl

using namespace cpl;

namespace {

struct Slab {
    int z0 = 0, z1 = 0, glo = 0, ghi = 0, nzl = 0;
    int64_t ncl = 0, nfl = 0;      // local bulk and fine cells
    couple_handle *h = nullptr;
    void *fine[4] = {nullptr, nullptr, nullptr, nullptr};
    void *phi = nullptr, *F = nullptr, *U = nullptr, *P = nullptr, *G = nullptr, *K = nullptr, *KU = nullptr;
    void *feps = nullptr, *fF = nullptr, *fK = nullptr, *fKU = nullptr;
    int32_t *count = nullptr, *start = nullptr;
};

// One block of the communication matrix: cnt values from src (slab sp) to dst
// (slab dp), copied or added.
struct Xfer {
    int sp, dp;
    void *src, *dst;
    int64_t cnt;
    bool add;
    size_t roff;   // offset in the root buffer (gather-scatter)
};

}  // namespace

struct couple_part {
    couple_config cfg{};
    int K = 1;
    size_t fsz = 4;
    std::vector<Slab> s;
    SortScratch sort{};
    uint32_t *owner = nullptr, *okey = nullptr, *oid = nullptr;
    void *lpos = nullptr, *lvel = nullptr, *ldiam = nullptr, *ldrag = nullptr, *lbeta = nullptr, *luf = nullptr;
    int32_t *lcell = nullptr, *lperm = nullptr, *gid = nullptr;
    double *ldiag = nullptr, *mpart = nullptr;
    void *root = nullptr;
    uint32_t *h_totals = nullptr;   // pinned host copy of the partition sizes
    std::vector<Xfer> fine_x, phi_rev, phi_fwd, src_rev, src_fwd;
    std::vector<void *> allocs;
    std::string err;
};

static thread_local std::string g_part_err;

static int pfail(couple_part *p, int code, const std::string &m) {
    if (p) p->err = m;
    else g_part_err = m;
    return code;
}

static void part_release(couple_part *p) {
    for (auto &s : p->s)
        if (s.h) couple_free(s.h);
    for (void *q : p->allocs)
        if (q) (void)hipFree(q);
    if (p->h_totals) (void)hipHostFree(p->h_totals);
    p->allocs.clear();
    p->s.clear();
}

template <typename X> static bool palloc(couple_part *p, X **q, size_t bytes) {
    void *v = nullptr;
    if (hipMalloc(&v, bytes ? bytes : 256) != hipSuccess) {
        (void)hipGetLastError();
        *q = nullptr;
        return false;
    }
    p->allocs.push_back(v);
    *q = static_cast<X *>(v);
    return true;
}

static bool pow2(double x) {
    int e = 0;
    return x > 0.0 && std::frexp(x, &e) == 0.5;
}

extern "C" int couple_part_init(const couple_config *cfg, int32_t nparts, couple_part **out) {
    if (!cfg || !out) return pfail(nullptr, COUPLE_EINVAL, "couple_part_init: NULL argument");
    *out = nullptr;
    if (nparts < 1 || nparts > kMaxParts || nparts > cfg->nb[2])
        return pfail(nullptr, COUPLE_EINVAL, "couple_part_init: nparts must be in [1, min(64, nb[2])]");
    if (!(cfg->vel_source == COUPLE_VEL_FINE || cfg->vel_source == COUPLE_VEL_BULK))
        return pfail(nullptr, COUPLE_EINVAL, "couple_part_init: vel_source must be FINE or BULK");
    if (cfg->vof) return pfail(nullptr, COUPLE_EINVAL, "couple_part_init: the two-fluid drag is not partitioned");
    if (!(cfg->nb[2] >= 1 && std::isfinite(cfg->box[2]) && pow2(cfg->box[2] / cfg->nb[2])))
        return pfail(nullptr, COUPLE_EINVAL, "couple_part_init: the bulk spacing box[2] / nb[2] must be a power of two");
    couple_part *p = new (std::nothrow) couple_part();
    if (!p) return pfail(nullptr, COUPLE_ENOMEM, "couple_part_init: host allocation failed");
    p->cfg = *cfg;
    p->K = nparts;
    p->fsz = cfg->precision == COUPLE_FP64 ? sizeof(double) : sizeof(float);
    const int K = nparts, nz = cfg->nb[2], R = cfg->ratio;
    const double hz = cfg->box[2] / nz;
    const int64_t nxy = (int64_t)cfg->nb[0] * cfg->nb[1];
    const int64_t nfxy = nxy * R * R;
    p->s.resize(K);
    bool ok = true;
    for (int k = 0; k < K && ok; ++k) {
        Slab &s = p->s[k];
        s.z0 = (int)((int64_t)nz * k / K);
        s.z1 = (int)((int64_t)nz * (k + 1) / K);
        s.glo = k > 0 ? 1 : 0;
        s.ghi = k < K - 1 ? 1 : 0;
        s.nzl = s.z1 - s.z0 + s.glo + s.ghi;
        s.ncl = nxy * s.nzl;
        s.nfl = s.ncl * R * R * R;
        couple_config lc = *cfg;
        lc.nb[2] = s.nzl;
        lc.box[2] = hz * s.nzl;   // exact: hz is a power of two
        const int rc = couple_init(&lc, &s.h);
        if (rc != COUPLE_OK) {
            std::string m = std::string("couple_part_init: slab ") + std::to_string(k) + ": " + couple_last_error(nullptr);
            part_release(p);
            delete p;
            return pfail(nullptr, rc, m);
        }
        const size_t f = p->fsz;
        for (int q = 0; q < 4; ++q) ok = ok && palloc(p, &s.fine[q], f * s.nfl);
        ok = ok && palloc(p, &s.phi, f * s.ncl) && palloc(p, &s.F, 3 * f * s.ncl) && palloc(p, &s.U, 3 * f * s.ncl) &&
             palloc(p, &s.P, f * s.ncl) && palloc(p, &s.G, 3 * f * s.ncl) && palloc(p, &s.feps, f * s.nfl) &&
             palloc(p, &s.fF, 3 * f * s.nfl) && palloc(p, &s.count, 4 * s.ncl) && palloc(p, &s.start, 4 * (s.ncl + 1));
        if (cfg->semi_implicit)
            ok = ok && palloc(p, &s.K, f * s.ncl) && palloc(p, &s.KU, 3 * f * s.ncl) && palloc(p, &s.fK, f * s.nfl) &&
                 palloc(p, &s.fKU, 3 * f * s.nfl);
    }
    const int64_t nmax = cfg->max_particles > 0 ? cfg->max_particles : 1;
    const int ntile = sort_tiles(nmax);
    const size_t f = p->fsz;
    ok = ok && palloc(p, &p->sort.hist, 4 * 256 * (size_t)ntile) && palloc(p, &p->sort.totals, 4 * 256) &&
         palloc(p, &p->owner, 4 * nmax) && palloc(p, &p->okey, 4 * nmax) && palloc(p, &p->oid, 4 * nmax) &&
         palloc(p, &p->lpos, 3 * f * nmax) && palloc(p, &p->lvel, 3 * f * nmax) && palloc(p, &p->ldiam, f * nmax) &&
         palloc(p, &p->ldrag, 3 * f * nmax) && palloc(p, &p->lbeta, f * nmax) && palloc(p, &p->luf, 3 * f * nmax) &&
         palloc(p, &p->lcell, 4 * nmax) && palloc(p, &p->lperm, 4 * nmax) && palloc(p, &p->gid, 4 * nmax) &&
         palloc(p, &p->ldiag, sizeof(double) * COUPLE_DIAG_LEN * K) && palloc(p, &p->mpart, sizeof(double) * 1024);
    ok = ok && hipHostMalloc((void **)&p->h_totals, 4 * 256) == hipSuccess;
    if (!ok) {
        (void)hipGetLastError();
        part_release(p);
        delete p;
        return pfail(nullptr, COUPLE_ENOMEM, "couple_part_init: device allocation failed");
    }
    // the communication matrix: blocks between neighbouring slabs A = k (below)
    // and B = k + 1; A's top owned layer is its local layer nzl - 2 and its top
    // ghost nzl - 1; B's bottom ghost is local layer 0 and its bottom owned 1
    auto byte = [](void *b, int64_t off, size_t fs) { return static_cast<char *>(b) + off * (int64_t)fs; };
    for (int k = 0; k + 1 < K; ++k) {
        Slab &A = p->s[k], &B = p->s[k + 1];
        const int tA = A.nzl - 2, gA = A.nzl - 1, gB = 0, oB = 1;
        for (int q = 0; q < 4; ++q) {
            const int64_t m = R * nfxy;
            p->fine_x.push_back({k, k + 1, byte(A.fine[q], tA * m, f), byte(B.fine[q], gB * m, f), m, false, 0});
            p->fine_x.push_back({k + 1, k, byte(B.fine[q], oB * m, f), byte(A.fine[q], gA * m, f), m, false, 0});
        }
        auto halo = [&](std::vector<Xfer> &rev, std::vector<Xfer> &fwd, void *a, void *b, int64_t ca, int64_t cb) {
            // component offsets ca, cb (cells) in A's and B's arrays
            rev.push_back({k, k + 1, byte(a, ca + gA * nxy, f), byte(b, cb + oB * nxy, f), nxy, true, 0});
            rev.push_back({k + 1, k, byte(b, cb + gB * nxy, f), byte(a, ca + tA * nxy, f), nxy, true, 0});
            fwd.push_back({k, k + 1, byte(a, ca + tA * nxy, f), byte(b, cb + gB * nxy, f), nxy, false, 0});
            fwd.push_back({k + 1, k, byte(b, cb + oB * nxy, f), byte(a, ca + gA * nxy, f), nxy, false, 0});
        };
        halo(p->phi_rev, p->phi_fwd, A.phi, B.phi, 0, 0);
        for (int c = 0; c < 3; ++c) halo(p->src_rev, p->src_fwd, A.F, B.F, c * A.ncl, c * B.ncl);
        if (cfg->semi_implicit) {
            halo(p->src_rev, p->src_fwd, A.K, B.K, 0, 0);
            for (int c = 0; c < 3; ++c) halo(p->src_rev, p->src_fwd, A.KU, B.KU, c * A.ncl, c * B.ncl);
        }
    }
    // root buffer: the largest exchange set staged whole
    size_t root = 256;
    for (std::vector<Xfer> *set : {&p->fine_x, &p->phi_rev, &p->phi_fwd, &p->src_rev, &p->src_fwd}) {
        size_t off = 0;
        for (Xfer &x : *set) {
            x.roff = off;
            off += ((size_t)x.cnt * f + 255) / 256 * 256;
        }
        root = std::max(root, off);
    }
    if (!palloc(p, &p->root, root)) {
        part_release(p);
        delete p;
        return pfail(nullptr, COUPLE_ENOMEM, "couple_part_init: device allocation failed");
    }
    *out = p;
    return COUPLE_OK;
}

template <typename T>
static hipError_t run_set(couple_part *p, const std::vector<Xfer> &set, int exchange, hipStream_t st) {
    auto apply = [&](void *dst, const void *src, int64_t cnt, bool add) -> hipError_t {
        if (add) {
            hipLaunchKernelGGL(k_add<T>, dim3((unsigned)((cnt + kBlock - 1) / kBlock)), dim3(kBlock), 0, st, (T *)dst,
                               (const T *)src, cnt);
            return hipGetLastError();
        }
        return hipMemcpyAsync(dst, src, (size_t)cnt * sizeof(T), hipMemcpyDeviceToDevice, st);
    };
    hipError_t e = hipSuccess;
    if (exchange == COUPLE_EXCHANGE_DISTRIBUTED) {
        for (const Xfer &x : set)
            if ((e = apply(x.dst, x.src, x.cnt, x.add)) != hipSuccess) return e;
        return e;
    }
    // gather to the root, then scatter from it
    char *root = static_cast<char *>(p->root);
    for (const Xfer &x : set)
        if ((e = hipMemcpyAsync(root + x.roff, x.src, (size_t)x.cnt * sizeof(T), hipMemcpyDeviceToDevice, st)) != hipSuccess)
            return e;
    for (const Xfer &x : set)
        if ((e = apply(x.dst, root + x.roff, x.cnt, x.add)) != hipSuccess) return e;
    return e;
}

template <typename T>
static int part_step(couple_part *p, const couple_inputs *in, couple_outputs *out, int exchange, hipStream_t st) {
    const couple_config &c = p->cfg;
    const int K = p->K, R = c.ratio;
    const int64_t n = in->n;
    const int64_t nxy = (int64_t)c.nb[0] * c.nb[1], nfxy = nxy * R * R;
    const int64_t ncell = nxy * c.nb[2], nfine = nfxy * R * c.nb[2];
    const Geo<T> g = make_geo<T>(c);
    ZCut zc{};
    zc.K = K;
    SlabShift<T> sh{};
    const double hz = c.box[2] / c.nb[2];
    for (int k = 0; k < K; ++k) {
        const Slab &s = p->s[k];
        zc.z[k] = s.z0;
        sh.dz[k] = (T)(hz * (s.z0 - s.glo));
        sh.cell_off[k] = (int64_t)(s.z0 - s.glo) * nxy;
    }
    zc.z[K] = c.nb[2];
    (void)hipGetLastError();
    const unsigned pb = (unsigned)((n + kBlock - 1) / kBlock);
    // owners, the stable partition by owner, the slab sizes on the host
    int bits = 1;
    while ((1 << bits) < K) ++bits;
    std::vector<int64_t> cnt(K, 0), off(K + 1, 0);
    if (n > 0) {
        hipLaunchKernelGGL(k_owner<T>, dim3(pb), dim3(kBlock), 0, st, (const T *)in->pos, n, g, zc, p->owner);
        if (launch_stable_partition(p->owner, n, bits, p->sort, p->okey, p->oid, st) != hipSuccess) return COUPLE_EHIP;
        if (hipMemcpyAsync(p->h_totals, p->sort.totals, 4 * (size_t)(1 << bits), hipMemcpyDeviceToHost, st) != hipSuccess ||
            hipStreamSynchronize(st) != hipSuccess)
            return COUPLE_EHIP;
        for (int k = 0; k < K; ++k) cnt[k] = p->h_totals[k];
    }
    for (int k = 0; k < K; ++k) off[k + 1] = off[k] + cnt[k];
    if (off[K] != n) return COUPLE_EHIP;   // the partition lost particles: cannot happen for owners < K
    for (int k = 0; k < K; ++k) sh.poff[k] = off[k];
    if (n > 0)
        hipLaunchKernelGGL(k_distribute<T>, dim3(pb), dim3(kBlock), 0, st, p->okey, p->oid, n, K, (const T *)in->pos,
                           (const T *)in->vel, (const T *)in->diam, sh, (T *)p->lpos, (T *)p->lvel, (T *)p->ldiam,
                           p->gid);
    // each slab's own fine slab, then the fine halo
    const void *fin[4] = {in->fine_u, in->fine_v, in->fine_w, in->fine_p};
    for (int k = 0; k < K; ++k) {
        const Slab &s = p->s[k];
        const int64_t m = (int64_t)(s.z1 - s.z0) * R * nfxy;
        for (int q = 0; q < 4; ++q)
            if (hipMemcpyAsync(static_cast<T *>(s.fine[q]) + (int64_t)s.glo * R * nfxy,
                               static_cast<const T *>(fin[q]) + (int64_t)s.z0 * R * nfxy, m * sizeof(T),
                               hipMemcpyDeviceToDevice, st) != hipSuccess)
                return COUPLE_EHIP;
    }
    if (run_set<T>(p, p->fine_x, exchange, st) != hipSuccess) return COUPLE_EHIP;
    // the slabs' steps, phase by phase, with the halo exchanges in between
    std::vector<couple_inputs> lin(K);
    std::vector<couple_outputs> lout(K);
    for (int k = 0; k < K; ++k) {
        Slab &s = p->s[k];
        couple_inputs &i = lin[k];
        i = couple_inputs{};
        i.n = cnt[k];
        i.pos = static_cast<T *>(p->lpos) + 3 * off[k];
        i.vel = static_cast<T *>(p->lvel) + 3 * off[k];
        i.diam = static_cast<T *>(p->ldiam) + off[k];
        i.fine_u = s.fine[0];
        i.fine_v = s.fine[1];
        i.fine_w = s.fine[2];
        i.fine_p = s.fine[3];
        i.step = in->step;
        couple_outputs &o = lout[k];
        o = couple_outputs{};
        o.drag = static_cast<T *>(p->ldrag) + 3 * off[k];
        o.beta = out->beta ? static_cast<T *>(p->lbeta) + off[k] : nullptr;
        o.uf = out->uf ? static_cast<T *>(p->luf) + 3 * off[k] : nullptr;
        o.cell = p->lcell + off[k];
        o.perm = p->lperm + off[k];
        o.count = s.count;
        o.start = s.start;
        o.bulk_phi = s.phi;
        o.bulk_F = s.F;
        o.bulk_U = s.U;
        o.bulk_P = s.P;
        o.bulk_G = s.G;
        o.fine_eps = s.feps;
        o.fine_F = s.fF;
        o.diag = p->ldiag + (int64_t)k * COUPLE_DIAG_LEN;
        o.bulk_K = s.K;
        o.bulk_KU = s.KU;
        o.fine_K = s.fK;
        o.fine_KU = s.fKU;
    }
    auto phases = [&](int ph) -> int {
        for (int k = 0; k < K; ++k) {
            const Slab &s = p->s[k];
            const char *what = nullptr;
            hipError_t herr = hipSuccess;
            const int rc = step_phases(s.h, &lin[k], &lout[k], st, ph, (int64_t)s.glo * nxy,
                                       (int64_t)(s.glo + s.z1 - s.z0) * nxy, &what, &herr);
            if (rc != COUPLE_OK) return rc;
        }
        return COUPLE_OK;
    };
    int rc;
    if ((rc = phases(kPhaseDeposit)) != COUPLE_OK) return rc;
    if (run_set<T>(p, p->phi_rev, exchange, st) != hipSuccess || run_set<T>(p, p->phi_fwd, exchange, st) != hipSuccess)
        return COUPLE_EHIP;
    if ((rc = phases(kPhaseVelocity | kPhaseSource)) != COUPLE_OK) return rc;
    if (run_set<T>(p, p->src_rev, exchange, st) != hipSuccess || run_set<T>(p, p->src_fwd, exchange, st) != hipSuccess)
        return COUPLE_EHIP;
    if ((rc = phases(kPhaseProlong | kPhaseDiag)) != COUPLE_OK) return rc;
    // the owned parts into the caller's arrays
    if (n > 0)
        hipLaunchKernelGGL(k_collect<T>, dim3(pb), dim3(kBlock), 0, st, p->okey, p->gid, n, K, sh,
                           (const T *)p->ldrag, (const T *)p->lbeta, p->lcell, p->lperm, (const T *)p->luf,
                           (const T *)p->lpos, (const T *)p->lvel, c.advect, (T *)out->drag, (T *)out->beta, out->cell,
                           out->perm, (T *)out->uf, (T *)in->pos, (T *)in->vel);
    for (int k = 0; k < K; ++k) {
        const Slab &s = p->s[k];
        const int64_t m = (int64_t)(s.z1 - s.z0) * nxy, lo = (int64_t)s.glo * nxy, go = (int64_t)s.z0 * nxy;
        const int64_t mf = m * R * R * R, lof = lo * R * R * R, gof = go * R * R * R;
        hipLaunchKernelGGL(k_collect_cells, dim3((unsigned)((m + kBlock - 1) / kBlock)), dim3(kBlock), 0, st,
                           s.count + lo, s.start + lo, m, (int32_t)off[k], k == K - 1 ? 1 : 0, out->count + go,
                           out->start + go);
        struct Piece { const void *src; void *dst; int64_t len; };
        std::vector<Piece> pieces = {{static_cast<const T *>(s.phi) + lo, static_cast<T *>(out->bulk_phi) + go, m},
                                     {static_cast<const T *>(s.P) + lo, static_cast<T *>(out->bulk_P) + go, m},
                                     {static_cast<const T *>(s.feps) + lof, static_cast<T *>(out->fine_eps) + gof, mf}};
        for (int q = 0; q < 3; ++q) {
            pieces.push_back({static_cast<const T *>(s.F) + q * s.ncl + lo, static_cast<T *>(out->bulk_F) + q * ncell + go, m});
            pieces.push_back({static_cast<const T *>(s.U) + q * s.ncl + lo, static_cast<T *>(out->bulk_U) + q * ncell + go, m});
            pieces.push_back({static_cast<const T *>(s.G) + q * s.ncl + lo, static_cast<T *>(out->bulk_G) + q * ncell + go, m});
            pieces.push_back({static_cast<const T *>(s.fF) + q * s.nfl + lof, static_cast<T *>(out->fine_F) + q * nfine + gof,
                              mf});
        }
        if (c.semi_implicit) {
            pieces.push_back({static_cast<const T *>(s.K) + lo, static_cast<T *>(out->bulk_K) + go, m});
            pieces.push_back({static_cast<const T *>(s.fK) + lof, static_cast<T *>(out->fine_K) + gof, mf});
            for (int q = 0; q < 3; ++q) {
                pieces.push_back({static_cast<const T *>(s.KU) + q * s.ncl + lo, static_cast<T *>(out->bulk_KU) + q * ncell + go, m});
                pieces.push_back({static_cast<const T *>(s.fKU) + q * s.nfl + lof,
                                  static_cast<T *>(out->fine_KU) + q * nfine + gof, mf});
            }
        }
        for (const Piece &q : pieces)
            if (hipMemcpyAsync(q.dst, q.src, (size_t)q.len * sizeof(T), hipMemcpyDeviceToDevice, st) != hipSuccess)
                return COUPLE_EHIP;
    }
    hipLaunchKernelGGL(k_sum_diags, dim3(1), dim3(kWave), 0, st, p->ldiag, K, out->diag);
    const int mb = (int)std::min<int64_t>(1024, (ncell + kBlock - 1) / kBlock);
    hipLaunchKernelGGL(k_max1<T>, dim3(mb), dim3(kBlock), 0, st, (const T *)out->bulk_phi, ncell, p->mpart);
    hipLaunchKernelGGL(k_max2, dim3(1), dim3(kBlock), 0, st, p->mpart, mb, out->diag);
    return hipGetLastError() == hipSuccess ? COUPLE_OK : COUPLE_EHIP;
}

extern "C" int couple_part_step(couple_part *p, const couple_inputs *in, couple_outputs *out, int32_t exchange,
                                void *stream) {
    if (!p) return pfail(nullptr, COUPLE_EINVAL, "couple_part_step: NULL handle");
    if (!in || !out) return pfail(p, COUPLE_EINVAL, "couple_part_step: NULL inputs or outputs");
    if (!(exchange == COUPLE_EXCHANGE_DISTRIBUTED || exchange == COUPLE_EXCHANGE_GATHER_SCATTER))
        return pfail(p, COUPLE_EINVAL, "couple_part_step: unknown exchange");
    if (in->n < 0) return pfail(p, COUPLE_EINVAL, "couple_part_step: n < 0");
    if (in->n > p->cfg.max_particles) return pfail(p, COUPLE_ECAPACITY, "couple_part_step: n exceeds max_particles");
    if (!in->fine_u || !in->fine_v || !in->fine_w || !in->fine_p)
        return pfail(p, COUPLE_EINVAL, "couple_part_step: NULL fine-grid input");
    if (!out->count || !out->start || !out->bulk_phi || !out->bulk_F || !out->bulk_U || !out->bulk_P || !out->bulk_G ||
        !out->fine_eps || !out->fine_F || !out->diag)
        return pfail(p, COUPLE_EINVAL, "couple_part_step: NULL grid output");
    if (p->cfg.semi_implicit && (!out->bulk_K || !out->bulk_KU || !out->fine_K || !out->fine_KU))
        return pfail(p, COUPLE_EINVAL, "couple_part_step: semi_implicit needs bulk_K, bulk_KU, fine_K and fine_KU");
    if (in->n > 0 && (!in->pos || !in->vel || !in->diam || !out->drag || !out->cell || !out->perm))
        return pfail(p, COUPLE_EINVAL, "couple_part_step: NULL particle array");
    hipStream_t st = static_cast<hipStream_t>(stream);
    const int rc = p->cfg.precision == COUPLE_FP64 ? part_step<double>(p, in, out, exchange, st)
                                                   : part_step<float>(p, in, out, exchange, st);
    if (rc != COUPLE_OK) return pfail(p, rc, "couple_part_step: a launch or copy failed");
    return COUPLE_OK;
}

extern "C" int couple_part_comm_matrix(const couple_part *p, int64_t *bytes) {
    if (!p || !bytes) return COUPLE_EINVAL;
    const int K = p->K;
    for (int i = 0; i < K * K; ++i) bytes[i] = 0;
    for (const std::vector<Xfer> *set : {&p->fine_x, &p->phi_rev, &p->phi_fwd, &p->src_rev, &p->src_fwd})
        for (const Xfer &x : *set) bytes[(int64_t)x.dp * K + x.sp] += x.cnt * (int64_t)p->fsz;
    return COUPLE_OK;
}

extern "C" int couple_part_free(couple_part *p) {
    if (!p) return COUPLE_OK;
    part_release(p);
    delete p;
    return COUPLE_OK;
}

extern "C" const char *couple_part_last_error(const couple_part *p) {
    return p ? p->err.c_str() : g_part_err.c_str();
}
