// sort.hip -- binning of particles into bulk cells and the deterministic,
// stable LSD radix sort that yields the canonical (cell, id) order.
//
// The particle -> cell connectivity changes with every coupling step because
// the particles move (Sec. 2.2); it is rebuilt here from scratch each step:
//
//   k_bin          containing cell per particle (output `cell`), the packed
//                  input-order copy pk = (x, y, z, d) with the position clamped
//                  into the box, and the digit histogram of the first radix
//                  pass, per tile;
//   k_radix_hist   digit histogram per tile for later passes;
//   k_radix_prefix exclusive prefix over tiles of every digit, digit totals;
//   k_radix_scatter stable ranking inside a tile (wave ballots, LDS staging) and
//                  coalesced scatter to the digit's output run;
//   k_segment_starts  start[c] = first sorted position with cell >= c, set by
//                  the sorted positions where the key changes (long runs of
//                  empty cells are left to the next kernel);
//   k_segment_counts  the starts left unset (binary search of the sorted keys)
//                  and count[c] = start[c+1] - start[c].
//
// Keys are cell indices < ncell; ids are the input order, so a stable LSD sort
// starting from the identity order gives ascending (cell, id).  Integer atomics
// are used only on LDS histogram bins (exact counts); no float atomics anywhere.
#include <algorithm>

#include "common.hpp"
#include "launch.hpp"

namespace cpl {

constexpr int kItems = 16;                         // keys per thread per tile
constexpr int kTile = kBlock * kItems;             // 4096 keys per tile
constexpr int kWaveSpan = kWave * kItems;          // keys handled by one wave
constexpr int kMaxDigits = 256;                    // radix <= 8 bits per pass

// A start entry not yet known: k_bin marks every entry so, k_segment_starts sets
// all but those inside long runs of empty cells, k_segment_counts the rest.
constexpr int32_t kUnset = -1;

// Workgroups [0, ntile) bin the particles of their tile; every workgroup of the
// grid (which may be larger, to cover the cells) also marks a share of
// start[0 .. nstart) unset.
template <typename T>
__global__ __launch_bounds__(kBlock) void k_bin(const T *__restrict__ pos, const T *__restrict__ diam, int64_t n,
                                                Geo<T> g, int32_t *__restrict__ cell, vec4<T> *__restrict__ pk,
                                                uint32_t *__restrict__ hist,
                                                int ntile, int bits0, double *__restrict__ part_nout,
                                                int32_t *__restrict__ start, int64_t nstart) {
    __shared__ uint32_t h[kMaxDigits];
    __shared__ double red[kWavesPerBlock];
    for (int64_t c = (int64_t)blockIdx.x * kBlock + threadIdx.x; c < nstart; c += (int64_t)gridDim.x * kBlock)
        start[c] = kUnset;
    if ((int)blockIdx.x >= ntile) return;   // uniform over the workgroup, before any barrier
    const int ndig = 1 << bits0;
    for (int d = threadIdx.x; d < ndig; d += kBlock) h[d] = 0;
    __syncthreads();
    const int64_t base = (int64_t)blockIdx.x * kTile;
    double nout = 0.0;
    for (int it = 0; it < kItems; ++it) {
        int64_t p = base + (int64_t)it * kBlock + threadIdx.x;
        if (p < n) {
            int outside = 0;
            T x = clamp_coord(pos[3 * p + 0], g.L[0], outside);
            T y = clamp_coord(pos[3 * p + 1], g.L[1], outside);
            T z = clamp_coord(pos[3 * p + 2], g.L[2], outside);
            int ix = cell_axis(x, g.sb[0], g.nb[0]);
            int iy = cell_axis(y, g.sb[1], g.nb[1]);
            int iz = cell_axis(z, g.sb[2], g.nb[2]);
            int32_t c = ix + g.nb[0] * (iy + g.nb[1] * iz);
            cell[p] = c;
            vec4<T> q;
            q.x = x;
            q.y = y;
            q.z = z;
            q.w = diam[p];
            pk[p] = q;
            atomicAdd(&h[(uint32_t)c & (ndig - 1)], 1u);
            nout += outside;
        }
    }
    __syncthreads();
    for (int d = threadIdx.x; d < ndig; d += kBlock) hist[(int64_t)d * ntile + blockIdx.x] = h[d];
    double t = block_sum(nout, red);
    if (threadIdx.x == 0) part_nout[blockIdx.x] = t;
}

__global__ __launch_bounds__(kBlock) void k_radix_hist(const uint32_t *__restrict__ keys, int64_t n, int shift,
                                                       int bits, uint32_t *__restrict__ hist, int ntile) {
    __shared__ uint32_t h[kMaxDigits];
    const int ndig = 1 << bits;
    for (int d = threadIdx.x; d < ndig; d += kBlock) h[d] = 0;
    __syncthreads();
    const int64_t base = (int64_t)blockIdx.x * kTile;
    for (int it = 0; it < kItems; ++it) {
        int64_t p = base + (int64_t)it * kBlock + threadIdx.x;
        if (p < n) atomicAdd(&h[(keys[p] >> shift) & (ndig - 1)], 1u);
    }
    __syncthreads();
    for (int d = threadIdx.x; d < ndig; d += kBlock) hist[(int64_t)d * ntile + blockIdx.x] = h[d];
}

// One workgroup per digit: exclusive prefix over the tiles (in place) and the
// digit's total.
__global__ __launch_bounds__(kBlock) void k_radix_prefix(uint32_t *__restrict__ hist, int ntile,
                                                         uint32_t *__restrict__ totals) {
    __shared__ uint32_t wsum[kWavesPerBlock];
    __shared__ uint32_t carry;
    uint32_t *row = hist + (int64_t)blockIdx.x * ntile;
    const int lane = threadIdx.x % kWave, w = threadIdx.x / kWave;
    if (threadIdx.x == 0) carry = 0;
    __syncthreads();
    for (int base = 0; base < ntile; base += kBlock) {
        int i = base + threadIdx.x;
        uint32_t v = i < ntile ? row[i] : 0u;
        // inclusive wave scan
        uint32_t s = v;
        for (int o = 1; o < kWave; o <<= 1) {
            uint32_t u = __shfl_up(s, o, kWave);
            if (lane >= o) s += u;
        }
        if (lane == kWave - 1) wsum[w] = s;
        __syncthreads();
        uint32_t off = carry;
        for (int k = 0; k < w; ++k) off += wsum[k];
        if (i < ntile) row[i] = off + s - v;
        __syncthreads();
        if (threadIdx.x == kBlock - 1) carry = off + s;
        __syncthreads();
    }
    if (threadIdx.x == 0) totals[blockIdx.x] = carry;
}

// Stable tile ranking and scatter.  FIRST: values are the input positions (ids).
template <bool FIRST>
__global__ __launch_bounds__(kBlock) void k_radix_scatter(const uint32_t *__restrict__ keys_in,
                                                          const uint32_t *__restrict__ vals_in, int64_t n,
                                                          int shift, int bits, const uint32_t *__restrict__ hist,
                                                          const uint32_t *__restrict__ totals, int ntile,
                                                          uint32_t *__restrict__ keys_out,
                                                          uint32_t *__restrict__ vals_out) {
    __shared__ uint32_t digit_base[kMaxDigits];       // global start of each digit's run
    __shared__ uint32_t local_start[kMaxDigits];      // start of each digit inside the tile
    __shared__ uint32_t wave_cnt[kWavesPerBlock][kMaxDigits];
    __shared__ uint32_t skey[kTile];
    __shared__ uint32_t sval[kTile];
    __shared__ uint32_t scan_tmp[kWavesPerBlock];

    const int ndig = 1 << bits;
    const uint32_t dmask = ndig - 1;
    const int lane = threadIdx.x % kWave, w = threadIdx.x / kWave;
    const int64_t tile0 = (int64_t)blockIdx.x * kTile;
    const int tile_n = (int)((n - tile0) < kTile ? (n - tile0) : kTile);

    for (int d = threadIdx.x; d < kMaxDigits; d += kBlock) {
        wave_cnt[0][d] = wave_cnt[1][d] = wave_cnt[2][d] = wave_cnt[3][d] = 0;
    }
    __syncthreads();

    // ---- rank: wave w owns keys [w*kWaveSpan, (w+1)*kWaveSpan) of the tile ----
    uint32_t key[kItems], val[kItems], rank[kItems];
    const uint64_t lt_mask = (lane == 0) ? 0ull : (~0ull >> (kWave - lane));
    for (int it = 0; it < kItems; ++it) {
        int li = w * kWaveSpan + it * kWave + lane;   // position inside the tile
        bool valid = li < tile_n;
        uint32_t k = valid ? keys_in[tile0 + li] : 0u;
        uint32_t v = valid ? (FIRST ? (uint32_t)(tile0 + li) : vals_in[tile0 + li]) : 0u;
        uint32_t d = (k >> shift) & dmask;
        uint64_t peers = __ballot(valid);
        for (int b = 0; b < bits; ++b) {
            bool bit = (d >> b) & 1u;
            uint64_t m = __ballot(bit);
            peers &= bit ? m : ~m;
        }
        uint32_t before = __popcll(peers & lt_mask);
        uint32_t cnt = valid ? wave_cnt[w][d] : 0u;
        // the lowest lane of each peer group advances the running count
        bool leader = valid && ((peers & lt_mask) == 0ull);
        __builtin_amdgcn_wave_barrier();
        if (leader) wave_cnt[w][d] = cnt + (uint32_t)__popcll(peers);
        __builtin_amdgcn_wave_barrier();
        key[it] = k;
        val[it] = v;
        rank[it] = valid ? cnt + before : 0xffffffffu;
    }
    __syncthreads();

    // ---- per digit: prefix over waves; tile-local digit starts ---------------
    uint32_t tot = 0;
    if (threadIdx.x < kMaxDigits) {
        int d = threadIdx.x;
        for (int q = 0; q < kWavesPerBlock; ++q) {
            uint32_t c = wave_cnt[q][d];
            wave_cnt[q][d] = tot;
            tot += c;
        }
    }
    // exclusive scan of `tot` over the 256 digits (one per thread), and of the
    // global digit totals for the digit bases.
    {
        uint32_t v = (threadIdx.x < kMaxDigits) ? tot : 0u;
        uint32_t s = v;
        for (int o = 1; o < kWave; o <<= 1) {
            uint32_t u = __shfl_up(s, o, kWave);
            if (lane >= o) s += u;
        }
        if (lane == kWave - 1) scan_tmp[w] = s;
        __syncthreads();
        uint32_t off = 0;
        for (int q = 0; q < w; ++q) off += scan_tmp[q];
        if (threadIdx.x < kMaxDigits) local_start[threadIdx.x] = off + s - v;
        __syncthreads();
        uint32_t g = (threadIdx.x < ndig) ? totals[threadIdx.x] : 0u;
        uint32_t gs = g;
        for (int o = 1; o < kWave; o <<= 1) {
            uint32_t u = __shfl_up(gs, o, kWave);
            if (lane >= o) gs += u;
        }
        if (lane == kWave - 1) scan_tmp[w] = gs;
        __syncthreads();
        uint32_t goff = 0;
        for (int q = 0; q < w; ++q) goff += scan_tmp[q];
        if (threadIdx.x < ndig)
            digit_base[threadIdx.x] = goff + gs - g + hist[(int64_t)threadIdx.x * ntile + blockIdx.x];
        __syncthreads();
    }

    // ---- stage the tile in digit order in LDS --------------------------------
    for (int it = 0; it < kItems; ++it) {
        if (rank[it] != 0xffffffffu) {
            uint32_t d = (key[it] >> shift) & dmask;
            uint32_t lp = local_start[d] + wave_cnt[w][d] + rank[it];
            skey[lp] = key[it];
            sval[lp] = val[it];
        }
    }
    __syncthreads();

    // ---- write out: consecutive threads write consecutive positions of a run --
    for (int i = threadIdx.x; i < tile_n; i += kBlock) {
        uint32_t k = skey[i];
        uint32_t d = (k >> shift) & dmask;
        uint32_t dst = digit_base[d] + (i - local_start[d]);
        if (dst < (uint64_t)n) {   // always true for a consistent histogram; guards the store
            keys_out[dst] = k;
            vals_out[dst] = sval[i];
        }
    }
}

// start[c] = first sorted position with key >= c, for c in [0, ncell].  Every
// sorted position i whose key differs from its predecessor's (with key[-1] = -1
// and key[n] = ncell) sets start[c] = i for the cells c in (key[i-1], key[i]],
// so every entry is written at most once and the keys are read once, coalesced,
// without searches.  A gap of more than kGapLane cells (a run of empty cells)
// is filled by the whole wave together; one of more than kGapWave cells is left
// unset for k_segment_counts, which spreads it over the grid (a single wave
// filling millions of empty cells would serialise the step).
constexpr int kGapLane = 32;
constexpr int64_t kGapWave = 4096;

__global__ __launch_bounds__(kBlock) void k_segment_starts(const uint32_t *__restrict__ skeys, int64_t n,
                                                           int64_t ncell, int32_t *__restrict__ start) {
    const int64_t i = (int64_t)blockIdx.x * kBlock + threadIdx.x;   // sorted position, 0 .. n
    const int lane = threadIdx.x % kWave;
    int32_t lo = 0, hi = -1;   // the cells set to i
    if (i <= n) {
        // keys are cells < ncell; the clamp only keeps the stores in bounds
        auto key = [&](int64_t k) { const int64_t v = skeys[k]; return (int32_t)(v < ncell ? v : ncell - 1); };
        lo = (i == 0 ? -1 : key(i - 1)) + 1;
        hi = i == n ? (int32_t)ncell : key(i);
    }
    const int32_t len = hi - lo + 1;
    if (len > 0 && len <= kGapLane)
        for (int32_t c = lo; c <= hi; ++c) start[c] = (int32_t)i;
    uint64_t m = __ballot(len > kGapLane);   // wave-uniform
    while (m) {
        const int l = __ffsll((unsigned long long)m) - 1;
        m &= m - 1;
        const int32_t glo = __shfl(lo, l, kWave), ghi = __shfl(hi, l, kWave), gi = __shfl((int32_t)i, l, kWave);
        if ((int64_t)ghi - glo + 1 > kGapWave) continue;   // left unset (wave-uniform)
        for (int64_t c = (int64_t)glo + lane; c <= ghi; c += kWave) start[c] = gi;   // 64-bit: no wrap near 2^31
    }
}

// First sorted position i in [0, n] with key[i] >= c (binary search).
__device__ __forceinline__ int32_t first_at_least(const uint32_t *__restrict__ skeys, int64_t n, int64_t c) {
    int64_t lo = 0, hi = n;
    while (lo < hi) {
        const int64_t mid = (lo + hi) >> 1;
        if ((int64_t)skeys[mid] < c) lo = mid + 1;
        else hi = mid;
    }
    return (int32_t)lo;
}

// Thread c in [0, ncell]: resolves start[c] if it is unset, and count[c] =
// start[c+1] - start[c] (an unset start[c+1] is resolved here too; its own
// thread stores the same value).
__global__ __launch_bounds__(kBlock) void k_segment_counts(int32_t *start, int64_t ncell,
                                                           const uint32_t *__restrict__ skeys, int64_t n,
                                                           int32_t *__restrict__ count) {
    const int64_t c = (int64_t)blockIdx.x * kBlock + threadIdx.x;
    if (c > ncell) return;
    int32_t v = start[c];
    if (v == kUnset) {
        v = first_at_least(skeys, n, c);
        start[c] = v;
    }
    if (c < ncell) {
        int32_t w = start[c + 1];
        if (w == kUnset) w = first_at_least(skeys, n, c + 1);
        count[c] = w - v;
    }
}

// ---------------------------------------------------------------------------
// Host side
// ---------------------------------------------------------------------------

int sort_tiles(int64_t n) { return (int)((n + kTile - 1) / kTile); }

void sort_plan(int64_t ncell, int *npass, int widths[4]) {
    int bits = 1;
    while ((int64_t(1) << bits) < ncell) ++bits;
    int p = (bits + 7) / 8;
    int base = bits / p, extra = bits % p;
    for (int i = 0; i < p; ++i) widths[i] = base + (i < extra ? 1 : 0);
    *npass = p;
}

template <typename T>
hipError_t launch_bin_sort(const T *pos, const T *diam, int64_t n, const Geo<T> &g, int32_t *cell, vec4<T> *pk,
                           int32_t *perm, int32_t *start, int32_t *count, const SortScratch &s, double *part_nout,
                           const uint32_t **sorted_keys, Marker *mk, hipStream_t st) {
    int npass, widths[4];
    sort_plan(g.ncell, &npass, widths);
    const int ntile = n > 0 ? sort_tiles(n) : 0;
    // the binning grid also covers start[0 .. ncell] (marked unset)
    const int64_t nstart = g.ncell + 1;
    const int bin_blocks = std::max<int64_t>(ntile, (nstart + kTile - 1) / kTile);
    mk->mark("bin", st);
    hipLaunchKernelGGL(k_bin<T>, dim3(bin_blocks), dim3(kBlock), 0, st, pos, diam, n, g, cell, pk, s.hist, ntile,
                       widths[0], part_nout, start, nstart);
    if (n > 0) {
        int shift = 0;
        const uint32_t *kin = (const uint32_t *)cell;
        const uint32_t *vin = nullptr;
        for (int p = 0; p < npass; ++p) {
            const bool last = (p == npass - 1);
            uint32_t *kout = (p % 2 == 0) ? s.keys_a : s.keys_b;
            uint32_t *vout = last ? (uint32_t *)perm : ((p % 2 == 0) ? s.vals_a : s.vals_b);
            if (p > 0) mk->mark("radix_hist", st);
            if (p > 0)
                hipLaunchKernelGGL(k_radix_hist, dim3(ntile), dim3(kBlock), 0, st, kin, n, shift, widths[p], s.hist,
                                   ntile);
            mk->mark("radix_prefix", st);
            hipLaunchKernelGGL(k_radix_prefix, dim3(1 << widths[p]), dim3(kBlock), 0, st, s.hist, ntile, s.totals);
            mk->mark("radix_scatter", st);
            if (p == 0)
                hipLaunchKernelGGL(k_radix_scatter<true>, dim3(ntile), dim3(kBlock), 0, st, kin, vin, n, shift,
                                   widths[p], s.hist, s.totals, ntile, kout, vout);
            else
                hipLaunchKernelGGL(k_radix_scatter<false>, dim3(ntile), dim3(kBlock), 0, st, kin, vin, n, shift,
                                   widths[p], s.hist, s.totals, ntile, kout, vout);
            kin = kout;
            vin = vout;
            shift += widths[p];
        }
        *sorted_keys = kin;
    } else {
        *sorted_keys = s.keys_a;
    }
    const int sblk = (int)((n + 1 + kBlock - 1) / kBlock), cblk = (int)((g.ncell + 1 + kBlock - 1) / kBlock);
    mk->mark("segments", st);
    hipLaunchKernelGGL(k_segment_starts, dim3(sblk), dim3(kBlock), 0, st, *sorted_keys, n, g.ncell, start);
    hipLaunchKernelGGL(k_segment_counts, dim3(cblk), dim3(kBlock), 0, st, start, g.ncell, *sorted_keys, n, count);
    return hipGetLastError();
}

hipError_t launch_stable_partition(const uint32_t *keys, int64_t n, int bits, const SortScratch &s, uint32_t *keys_out,
                                   uint32_t *ids_out, hipStream_t st) {
    if (n <= 0) return hipGetLastError();
    const int ntile = sort_tiles(n);
    hipLaunchKernelGGL(k_radix_hist, dim3(ntile), dim3(kBlock), 0, st, keys, n, 0, bits, s.hist, ntile);
    hipLaunchKernelGGL(k_radix_prefix, dim3(1 << bits), dim3(kBlock), 0, st, s.hist, ntile, s.totals);
    hipLaunchKernelGGL(k_radix_scatter<true>, dim3(ntile), dim3(kBlock), 0, st, keys, (const uint32_t *)nullptr, n, 0,
                       bits, s.hist, s.totals, ntile, keys_out, ids_out);
    return hipGetLastError();
}

template hipError_t launch_bin_sort<float>(const float *, const float *, int64_t, const Geo<float> &, int32_t *,
                                           vec4<float> *, int32_t *, int32_t *, int32_t *, const SortScratch &,
                                           double *, const uint32_t **, Marker *, hipStream_t);
template hipError_t launch_bin_sort<double>(const double *, const double *, int64_t, const Geo<double> &, int32_t *,
                                            vec4<double> *, int32_t *, int32_t *, int32_t *, const SortScratch &,
                                            double *, const uint32_t **, Marker *, hipStream_t);

}  // namespace cpl
