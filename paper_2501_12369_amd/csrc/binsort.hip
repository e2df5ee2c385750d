// binsort.hip -- tile binning and per-tile depth order.
//
// Target order: instances (tile, splat) sorted by (tile, depth bits, splat
// index); ranges[t] delimit tile t.  The work is arranged so that every
// K-sized array is written once, by runs of consecutive lanes (whole cache
// lines: partial-line stores to HBM3E turn into read-modify-writes):
//
//   keys      one thread per splat: tile box on the 16x16 tile grid, per-block
//             visible counts and box areas.  K (sum of the areas) is known here,
//             so the capacity overflow is decided before any instance is written.
//   compact   visible splats -> (depth bits, index) in index order.
//   sort      stable LSD radix sort of the N_v depth keys (8-bit digits)
//             -> splats in (depth, index) order.
//   level 1   super-tiles of 8x8 tiles.  256 depth-ordered splats per workgroup;
//             per super-tile a ballot over the lanes gives each covering splat
//             its rank; a scan over (super-tile, chunk) turns counts into
//             positions -> per super-tile lists of splats, still depth-ordered.
//   level 2   256 consecutive entries of one super-tile list per workgroup
//             (small workgroups: the 64-tile store loop of each wave is uneven,
//             and several workgroups per CU keep it busy across barriers); for
//             each of its 64 tiles a ballot ranks the covering entries and a scan
//             over (tile, chunk) gives positions -> the final list, each
//             (chunk, tile) run written contiguously.
//
// Ranks come from ballots in lane order, so every step is stable and the result
// is unique.  The tile box is recomputed from (xy, extent) with the same FP32
// expression everywhere.  HBM-bound.
#include <algorithm>

#include "common.h"

namespace darb {

namespace {

constexpr int kKeyItems = 16;                              // splats per thread in keys / compact
constexpr int kKeyTile = 256 * kKeyItems;                  // splats per keys / compact block
constexpr int kScanThreads = 256;
constexpr int kScanItems = 8;
constexpr int kScanBlock = kScanThreads * kScanItems;  // 2048 elements per block
constexpr int kRadixThreads = 256;
#ifndef DARB_RADIX_ITEMS
#define DARB_RADIX_ITEMS 16
#endif
constexpr int kRadixItems = DARB_RADIX_ITEMS;  // keys per thread of a radix tile
constexpr int kRadixTile = kRadixThreads * kRadixItems;  // 4096 keys per block
constexpr int kRadixWaves = kRadixThreads / 64;
constexpr int kRadixWaveItems = kRadixTile / kRadixWaves;  // keys per wave (16 rounds of 64)
constexpr int kSuper = 8;                                 // super-tile = 8x8 tiles
constexpr int kL1Threads = 256;                           // splats per level-1 chunk
constexpr int kL2Threads = 256;                           // list entries per level-2 chunk
constexpr int kL2Waves = kL2Threads / 64;
#ifndef DARB_L2_GRID
#define DARB_L2_GRID 8192
#endif
constexpr int kL2Grid = DARB_L2_GRID;                     // persistent level-2 workgroups (a tuning constant)

struct Counters {
    uint32_t n_visible;  // N_v
    uint32_t c1;         // level-1 chunks
    uint32_t pad0;
    uint32_t total1;     // level-1 list length
    uint32_t total2;     // level-2 chunks
    uint32_t h2_count;   // flattened level-2 count entries
    uint32_t scan_total; // scratch total of the last scan
    uint32_t pad;
    unsigned long long K;
};

// Tile rectangle [x0, x1) x [y0, y1) of a box of half-extents e = (rx, ry)
// around (u, v), clamped to the grid.
__device__ __forceinline__ int4 tile_rect(float u, float v, int2 e, int gx, int gy) {
    const float rx = (float)e.x, ry = (float)e.y;
    int x0 = (int)fminf(fmaxf(floorf((u - rx) * 0.0625f), 0.0f), (float)gx);
    int x1 = (int)fminf(fmaxf(floorf((u + rx) * 0.0625f) + 1.0f, 0.0f), (float)gx);
    int y0 = (int)fminf(fmaxf(floorf((v - ry) * 0.0625f), 0.0f), (float)gy);
    int y1 = (int)fminf(fmaxf(floorf((v + ry) * 0.0625f) + 1.0f, 0.0f), (float)gy);
    return make_int4(x0, x1, y0, y1);
}

// An empty asm use of v: the compiler waits for the loads producing v here, so
// loads issued before it are in flight together and land before what follows.
__device__ __forceinline__ void pin4(const uint4 &v) { asm volatile("" ::"v"(v.x), "v"(v.y), "v"(v.z), "v"(v.w)); }
__device__ __forceinline__ void pin_u32(uint32_t a, uint32_t b) { asm volatile("" ::"v"(a), "v"(b)); }
__device__ __forceinline__ void pin_u32(uint32_t a, uint32_t b, uint32_t c, uint32_t d) {
    asm volatile("" ::"v"(a), "v"(b), "v"(c), "v"(d));
}

__device__ __forceinline__ uint64_t lanemask_lt() {
    const int lane = threadIdx.x & 63;
    return lane == 0 ? 0ull : (~0ull >> (64 - lane));
}

// ---------------------------------------------------------------------------
// Exclusive scan of u32 (reduce -> scan block sums -> down-sweep).  The live
// element count may sit on the device (count_dev), `max_count` sizes the grid;
// blocks past the live count exit.  The total goes to *total_out (nullable).
// ---------------------------------------------------------------------------

__device__ __forceinline__ uint32_t live_count(const uint32_t *count_dev, uint32_t max_count) {
    return count_dev ? min(*count_dev, max_count) : max_count;
}

template <int T>
__device__ __forceinline__ uint32_t block_excl_scan_n(uint32_t v, uint32_t *lds_w, uint32_t *total) {
    const int lane = threadIdx.x & 63, w = threadIdx.x >> 6;
    uint32_t inc = wave_incl_scan(v);
    if (lane == 63) lds_w[w] = inc;
    __syncthreads();
    uint32_t woff = 0, tot = 0;
    for (int i = 0; i < T / 64; i++) {
        uint32_t x = lds_w[i];
        if (i < w) woff += x;
        tot += x;
    }
    __syncthreads();
    *total = tot;
    return woff + inc - v;
}

__device__ __forceinline__ uint32_t block_excl_scan(uint32_t v, uint32_t *lds_w, uint32_t *total) {
    return block_excl_scan_n<kScanThreads>(v, lds_w, total);
}

__global__ __launch_bounds__(kScanThreads) void k_scan_reduce(const uint32_t *in, const uint32_t *count_dev,
                                                              uint32_t max_count, uint32_t *parts,
                                                              const int32_t *skip) {
    __shared__ uint32_t lw[kScanThreads / 64];
    if (skip && *skip) return;
    uint32_t count = live_count(count_dev, max_count);
    uint32_t base = blockIdx.x * kScanBlock;
    if (base >= count) return;
    uint32_t v[kScanItems], s = 0;
#pragma unroll
    for (int k = 0; k < kScanItems; k++) {
        uint32_t i = base + k * kScanThreads + threadIdx.x;
        v[k] = i < count ? in[i] : 0u;
    }
#pragma unroll
    for (int k = 0; k < kScanItems; k++) s += v[k];
    uint32_t tot;
    block_excl_scan(s, lw, &tot);
    if (threadIdx.x == 0) parts[blockIdx.x] = tot;
}

// The down-sweep adds the sum of the block sums before its own block, which it
// reads itself (at most a few thousand words per block, from L2): no separate
// launch scans the block sums.  The last live block writes the total.
__global__ __launch_bounds__(kScanThreads) void k_scan_down(const uint32_t *in, uint32_t *out, const uint32_t *count_dev,
                                                            uint32_t max_count, const uint32_t *parts,
                                                            uint32_t *total_out, const int32_t *skip) {
    __shared__ uint32_t lw[kScanThreads / 64];
    __shared__ uint32_t lp[kScanThreads / 64];
    if (skip && *skip) return;
    uint32_t count = live_count(count_dev, max_count);
    uint32_t base = blockIdx.x * kScanBlock;
    if (base >= count) {
        if (count == 0 && blockIdx.x == 0 && threadIdx.x == 0 && total_out) *total_out = 0;
        return;
    }
    uint32_t v[kScanItems];
    uint32_t s = 0;
    uint32_t b0 = base + threadIdx.x * kScanItems;
    for (int k = 0; k < kScanItems; k++) {
        v[k] = (b0 + k < count) ? in[b0 + k] : 0u;
        s += v[k];
    }
    uint32_t pre = 0;
    for (uint32_t i = threadIdx.x; i < blockIdx.x; i += kScanThreads) pre += parts[i];
#pragma unroll
    for (int off = 32; off >= 1; off >>= 1) pre += (uint32_t)__shfl_xor((int)pre, off, 64);
    if ((threadIdx.x & 63) == 0) lp[threadIdx.x >> 6] = pre;
    uint32_t tot;
    uint32_t off = block_excl_scan(s, lw, &tot);  // (its barriers also publish lp)
    pre = 0;
#pragma unroll
    for (int k = 0; k < kScanThreads / 64; k++) pre += lp[k];
    off += pre;
    for (int k = 0; k < kScanItems; k++) {
        if (b0 + k < count) out[b0 + k] = off;
        off += v[k];
    }
    if (total_out && threadIdx.x == 0 && base + kScanBlock >= count) *total_out = pre + tot;
}

hipError_t scan_exclusive(uint32_t *data, const uint32_t *count_dev, uint32_t max_count, uint32_t *parts,
                          uint32_t *total_out, const int32_t *skip, hipStream_t s) {
    if (max_count == 0) return hipSuccess;
    uint32_t nb = (max_count + kScanBlock - 1) / kScanBlock;
    hipLaunchKernelGGL(k_scan_reduce, dim3(nb), dim3(kScanThreads), 0, s, data, count_dev, max_count, parts, skip);
    hipLaunchKernelGGL(k_scan_down, dim3(nb), dim3(kScanThreads), 0, s, data, data, count_dev, max_count, parts,
                       total_out, skip);
    return hipGetLastError();
}

// ---------------------------------------------------------------------------
// Stable LSD radix sort of (u32 key, u32 value), 8-bit digits, device count.
// ---------------------------------------------------------------------------

__global__ __launch_bounds__(kRadixThreads) void k_radix_hist(const uint32_t *keys, const uint32_t *count_dev, int shift,
                                                              uint32_t *hist, int nblk, const int32_t *skip) {
    __shared__ uint32_t h[256];
    if (*skip) return;
    const uint32_t n = *count_dev;
    h[threadIdx.x] = 0;
    __syncthreads();
    const uint32_t base = blockIdx.x * kRadixTile;
    // every key load in flight before the first LDS atomic (a load-atomic-load
    // chain pays the memory latency once per key)
    // (unconditional loads at clamped indices keep them in one basic block; a
    // block with n == 0 reads keys[0], which exists whenever the sort runs)
    uint32_t d[kRadixItems];
    const uint32_t last = n > 0 ? n - 1 : 0;
#pragma unroll
    for (int k = 0; k < kRadixItems; k++) d[k] = keys[min(base + k * kRadixThreads + threadIdx.x, last)];
#pragma unroll
    for (int k = 0; k < kRadixItems; k++) {
        const uint32_t i = base + k * kRadixThreads + threadIdx.x;
        d[k] = i < n ? (d[k] >> shift) & 255u : 256u;
    }
#pragma unroll
    for (int k = 0; k < kRadixItems; k++)
        if (d[k] < 256u) atomicAdd(&h[d[k]], 1u);
    __syncthreads();
    hist[threadIdx.x * nblk + blockIdx.x] = h[threadIdx.x];  // digit-major
}

// Row-wise exclusive scan, in place, one workgroup of T threads per row: rows of
// `len` counts stored back to back (len from the device when len_dev is set),
// the row's total to totals[row].  Long rows (the level-1 chunk counts) take
// T = 1024, so that a row is one round of loads, one scan and one round of
// stores.  Used where a count array is row-major over a
// small number of rows (radix digits, super-tiles) and its consumer adds the
// row's start (a scan over the few totals) itself, instead of one scan over
// all entries.
template <int T>
__device__ __forceinline__ void rowscan_row(uint32_t *data, uint32_t len, uint32_t *totals, uint32_t *lw) {
    const int nblk = (int)len;
    uint32_t *row = data + (size_t)blockIdx.x * nblk;
    uint32_t carry = 0;
    for (int base = 0; base < nblk; base += T * kScanItems) {
        const int b0 = base + threadIdx.x * kScanItems;
        uint32_t v[kScanItems], sum = 0;
#pragma unroll
        for (int k = 0; k < kScanItems; k++) {
            v[k] = b0 + k < nblk ? row[b0 + k] : 0u;
            sum += v[k];
        }
        uint32_t tot;
        uint32_t off = carry + block_excl_scan_n<T>(sum, lw, &tot);
#pragma unroll
        for (int k = 0; k < kScanItems; k++) {
            if (b0 + k < nblk) row[b0 + k] = off;
            off += v[k];
        }
        carry += tot;
    }
    if (threadIdx.x == 0) totals[blockIdx.x] = carry;
}

template <int T>
__global__ __launch_bounds__(T) void k_rowscan(uint32_t *data, const uint32_t *len_dev, uint32_t len_host,
                                               uint32_t *totals, const int32_t *skip) {
    __shared__ uint32_t lw[T / 64];
    if (*skip) return;
    rowscan_row<T>(data, len_dev ? *len_dev : len_host, totals, lw);
}

// One tile of kRadixTile keys per workgroup; wave w owns the contiguous quarter
// [w * kRadixWaveItems, (w + 1) * kRadixWaveItems) of the tile, held in
// registers (all loads issued at once).  Each wave ranks its keys by digit on
// its own (8 ballots per round of 64 keys give the lanes with the same digit;
// per-wave digit counters in LDS carry the rank across rounds -- one wave's
// LDS operations complete in order, so no barrier is needed between rounds).
// One scan over (digit, wave) then places the tile in LDS in digit order,
// stable (digit, wave, round, lane), and each digit's run is written to its
// global position by consecutive lanes.  Three workgroup barriers in all.
//
#ifndef DARB_RADIX_XCD_MAP
#define DARB_RADIX_XCD_MAP 1
#endif
// Key tile of scatter workgroup b.  With the XCD map, the workgroups the
// hardware deals to one XCD (b = x, x + 8, ...) take consecutive tiles, so the
// neighbouring runs of a digit are written through one L2.
__device__ __forceinline__ uint32_t radix_tile_of(uint32_t b, uint32_t nb) {
    if (!DARB_RADIX_XCD_MAP) return b;
    const uint32_t x = b & 7u, j = b >> 3, q = nb >> 3, r = nb & 7u;
    return x * q + min(x, r) + j;
}

// REC (the last pass of the depth sort): instead of (key, value) the output is
// the splat index and tile box of each value, in sorted order.  With 32-bit
// values (compact indices) they are gathered from the compact records while the
// tile is written out; with 64-bit values (splat index | box with 8-bit tile
// coordinates, carried through every pass) they are the value itself, and the
// last pass reads nothing at random.
template <class V, bool REC>
__global__ __launch_bounds__(kRadixThreads) void k_radix_scatter(const uint32_t *kin, const V *vin, uint32_t *kout,
                                                                 V *vout, const uint32_t *count_dev, int shift,
                                                                 const uint32_t *hist_scan, int nblk,
                                                                 const int32_t *skip, const uint4 *crec,
                                                                 uint32_t *sid, uint2 *sbox) {
    __shared__ uint32_t run[256];                  // global first slot of each digit for this tile
    __shared__ uint32_t loff[256];                 // first LDS slot of each digit
    __shared__ uint32_t wcnt[kRadixWaves][256];    // per-wave digit counts, then per-wave first slots
    __shared__ uint32_t lw[kRadixWaves];
    __shared__ uint32_t sk[kRadixTile];
    __shared__ V sv[kRadixTile];
    if (*skip) return;
    const uint32_t n = *count_dev;
    const uint32_t nlive = (n + kRadixTile - 1) / kRadixTile;  // tiles holding keys
    if (blockIdx.x >= nlive) return;
    const uint32_t tile = radix_tile_of(blockIdx.x, nlive);
    const uint32_t base = tile * kRadixTile;
    const uint32_t cnt = min((uint32_t)kRadixTile, n - base);
    const int t = threadIdx.x, w = t >> 6, lane = t & 63;
    // the tile's keys and values, and this thread's digit counts, all in flight at once
    uint32_t key[kRadixItems];
    V val[kRadixItems];
    const uint32_t w0 = (uint32_t)w * kRadixWaveItems;
#pragma unroll
    for (int r = 0; r < kRadixItems; r++) {
        const uint32_t li = w0 + r * 64 + lane;
        key[r] = li < cnt ? kin[base + li] : 0u;
        val[r] = li < cnt ? vin[base + li] : V{};
    }
    const uint32_t dtotal = hist_scan[(size_t)256 * nblk + t], dprefix = hist_scan[t * nblk + tile];
    {
        // global first slot of digit t for this tile: the digit's start (scan of the
        // digit totals) plus this tile's prefix within the digit's row
        uint32_t tot;
        run[t] = block_excl_scan(dtotal, lw, &tot) + dprefix;
    }
#pragma unroll
    for (int k = 0; k < kRadixWaves; k++) wcnt[k][t] = 0;
    __syncthreads();
    const uint64_t lt = lanemask_lt();
    uint32_t rank[kRadixItems];
    uint32_t *mycnt = wcnt[w];
#pragma unroll
    for (int r = 0; r < kRadixItems; r++) {
        const bool valid = w0 + r * 64 + lane < cnt;
        const uint32_t d = (key[r] >> shift) & 255u;
        uint64_t peers = __ballot(valid);
#pragma unroll
        for (int b = 0; b < 8; b++) {
            const bool bit = (d >> b) & 1u;
            const uint64_t m = __ballot(bit);
            peers &= bit ? m : ~m;
        }
        const uint32_t below = (uint32_t)__popcll(peers & lt);
        const uint32_t before = valid ? mycnt[d] : 0u;
        rank[r] = before + below;
        if (valid && below == 0) mycnt[d] = before + (uint32_t)__popcll(peers);
    }
    __syncthreads();
    {
        // digit t: exclusive scan of the tile's digit totals, then the per-wave firsts
        uint32_t c[kRadixWaves], tot = 0;
#pragma unroll
        for (int k = 0; k < kRadixWaves; k++) {
            c[k] = wcnt[k][t];
            tot += c[k];
        }
        const uint32_t inc = wave_incl_scan(tot);
        if (lane == 63) lw[w] = inc;
        __syncthreads();
        uint32_t off = inc - tot;
        for (int k = 0; k < w; k++) off += lw[k];
        loff[t] = off;
#pragma unroll
        for (int k = 0; k < kRadixWaves; k++) {
            wcnt[k][t] = off;
            off += c[k];
        }
    }
    __syncthreads();
#pragma unroll
    for (int r = 0; r < kRadixItems; r++) {
        if (w0 + r * 64 + lane < cnt) {
            const uint32_t o = mycnt[(key[r] >> shift) & 255u] + rank[r];
            sk[o] = key[r];
            sv[o] = val[r];
        }
    }
    __syncthreads();
    // the tile in digit order: slot i of digit d goes to run[d] + (i - loff[d])
    if constexpr (REC && sizeof(V) == 8) {
        for (uint32_t i = t; i < cnt; i += kRadixThreads) {
            const uint32_t d = (sk[i] >> shift) & 255u;
            const uint32_t g = run[d] + (i - loff[d]);
            const uint2 v = reinterpret_cast<const uint2 &>(sv[i]);
            sid[g] = v.x;
            sbox[g] = make_uint2((v.y & 0xFFu) | ((v.y >> 8) & 0xFFu) << 16,
                                 ((v.y >> 16) & 0xFFu) | (v.y >> 24) << 16);
        }
    } else if constexpr (REC) {
        // gathers and destinations first; the stores follow once every gather
        // has landed (a store between two uses of gathered data would make the
        // second use wait for it: vmcnt counts stores too)
        uint4 rec[kRadixItems];
        uint32_t g[kRadixItems];
#pragma unroll
        for (int r = 0; r < kRadixItems; r++) {
            const uint32_t i = r * kRadixThreads + t;
            g[r] = kNone;
            if (i < cnt) {
                rec[r] = crec[sv[i]];
                const uint32_t d = (sk[i] >> shift) & 255u;
                g[r] = run[d] + (i - loff[d]);
            }
        }
#pragma unroll
        for (int r = 0; r < kRadixItems; r++) pin4(rec[r]);  // every gather lands before the first store
#pragma unroll
        for (int r = 0; r < kRadixItems; r++) {
            if (g[r] != kNone) {
                sid[g[r]] = rec[r].z;
                sbox[g[r]] = make_uint2(rec[r].x, rec[r].y);
            }
        }
    } else {
        for (uint32_t i = t; i < cnt; i += kRadixThreads) {
            const uint32_t k = sk[i];
            const uint32_t d = (k >> shift) & 255u;
            const uint32_t g = run[d] + (i - loff[d]);
            kout[g] = k;
            vout[g] = sv[i];
        }
    }
}

// ---------------------------------------------------------------------------
// Keys, sizes, compaction.
// ---------------------------------------------------------------------------

// Per block of kKeyTile splats (kKeyItems per thread, all loads issued
// together): number of visible splats and the sum of their box areas.
__global__ __launch_bounds__(256) void k_bin_keys(const float *xy, const int2 *extent, int n, int gx, int gy,
                                                  uint32_t *block_vis, uint32_t *block_area) {
    __shared__ uint32_t wv[4], wa[4];
    const int base = blockIdx.x * kKeyTile + threadIdx.x;
    int2 R[kKeyItems];
    float2 p[kKeyItems];
#pragma unroll
    for (int k = 0; k < kKeyItems; k++) {
        const int i = base + k * 256;
        R[k] = i < n ? extent[i] : make_int2(0, 0);
        p[k] = i < n ? reinterpret_cast<const float2 *>(xy)[i] : make_float2(0.0f, 0.0f);
    }
    uint32_t vis = 0, area = 0;
#pragma unroll
    for (int k = 0; k < kKeyItems; k++) {
        if ((R[k].x <= 0) | (R[k].y <= 0)) continue;
        const int4 r = tile_rect(p[k].x, p[k].y, R[k], gx, gy);
        if ((r.y > r.x) & (r.w > r.z)) {
            vis++;
            area += (uint32_t)((r.y - r.x) * (r.w - r.z));
        }
    }
#pragma unroll
    for (int off = 32; off >= 1; off >>= 1) {
        area += (uint32_t)__shfl_xor((int)area, off, 64);
        vis += (uint32_t)__shfl_xor((int)vis, off, 64);
    }
    if ((threadIdx.x & 63) == 0) {
        wv[threadIdx.x >> 6] = vis;
        wa[threadIdx.x >> 6] = area;
    }
    __syncthreads();
    if (threadIdx.x == 0) {
        block_vis[blockIdx.x] = wv[0] + wv[1] + wv[2] + wv[3];
        block_area[blockIdx.x] = wa[0] + wa[1] + wa[2] + wa[3];
    }
}

// single workgroup: exclusive scan of the block visible counts (compaction
// offsets), N_v, K = sum of the areas, capacity decision, level-1 sizes
__global__ __launch_bounds__(1024) void k_bin_sizes(uint32_t *block_vis, const uint32_t *block_area, int nkb,
                                                    Counters *cnt, int64_t k_capacity, int64_t *k_dev,
                                                    int32_t *overflow_dev) {
    __shared__ uint32_t lw[16];
    __shared__ unsigned long long la[16];
    __shared__ uint32_t carry;
    const int lane = threadIdx.x & 63, w = threadIdx.x >> 6;
    if (threadIdx.x == 0) carry = 0;
    unsigned long long asum = 0;
    __syncthreads();
    for (int base = 0; base < nkb; base += 1024) {
        int i = base + threadIdx.x;
        uint32_t v = i < nkb ? block_vis[i] : 0u;
        if (i < nkb) asum += block_area[i];
        uint32_t inc = wave_incl_scan(v);
        if (lane == 63) lw[w] = inc;
        __syncthreads();
        uint32_t woff = 0, tot = 0;
        for (int k = 0; k < 16; k++) {
            if (k < w) woff += lw[k];
            tot += lw[k];
        }
        uint32_t c = carry;
        if (i < nkb) block_vis[i] = c + woff + inc - v;
        __syncthreads();
        if (threadIdx.x == 0) carry = c + tot;
        __syncthreads();
    }
#pragma unroll
    for (int off = 32; off >= 1; off >>= 1) asum += __shfl_xor(asum, off, 64);
    if (lane == 0) la[w] = asum;
    __syncthreads();
    if (threadIdx.x == 0) {
        unsigned long long K = 0;
        for (int k = 0; k < 16; k++) K += la[k];
        uint32_t nv = carry;
        *cnt = Counters{};  // every counter of this call starts here (none is read before this kernel)
        cnt->n_visible = nv;
        cnt->c1 = (nv + kL1Threads - 1) / kL1Threads;
        cnt->K = K;
        k_dev[0] = (int64_t)K;
        k_dev[1] = (int64_t)nv;
        *overflow_dev = (K > (unsigned long long)k_capacity || K >= 0xFFFFFFFFull) ? 1 : 0;
    }
}

// Visible splats in index order: depth key, value = compact index, and the
// compact record (tile box packed in 16-bit halves, splat index) that level 1
// reads after the sort instead of gathering the projected splat again.  Same
// blocking as k_bin_keys; a splat's slot is the block's offset plus the
// visible splats before it in (round, wave, lane) = index order.

// V64 (tile grids of at most 255 x 255): the value is (splat index, box with
// 8-bit tile coordinates) and no record is written; the sort carries it.
template <bool V64>
__global__ __launch_bounds__(256) void k_bin_compact(const float *xy, const int2 *extent, const float *depth, int n,
                                                     int gx, int gy, const uint32_t *block_off, uint32_t *keys,
                                                     uint32_t *vals, uint4 *crec, uint2 *vals64,
                                                     const int32_t *overflow_dev) {
    __shared__ uint32_t wv[kKeyItems * 4];  // visible count of each (round, wave), then its first slot
    if (*overflow_dev) return;
    const int w = threadIdx.x >> 6, lane = threadIdx.x & 63;
    const int base = blockIdx.x * kKeyTile + threadIdx.x;
    int2 R[kKeyItems];
    float2 p[kKeyItems];
    uint32_t db[kKeyItems];
    // every load issued up front: in the store loop below a load would wait for
    // the stores before it (vmcnt counts both)
#pragma unroll
    for (int k = 0; k < kKeyItems; k++) {
        const int i = base + k * 256;
        R[k] = i < n ? extent[i] : make_int2(0, 0);
        p[k] = i < n ? reinterpret_cast<const float2 *>(xy)[i] : make_float2(0.0f, 0.0f);
        db[k] = i < n ? __float_as_uint(depth[i]) : 0u;
    }
    uint32_t visbits = 0;
    int4 rect[kKeyItems];
#pragma unroll
    for (int k = 0; k < kKeyItems; k++) {
        rect[k] = make_int4(0, 0, 0, 0);
        bool vis = false;
        if ((R[k].x > 0) & (R[k].y > 0)) {
            rect[k] = tile_rect(p[k].x, p[k].y, R[k], gx, gy);
            vis = (rect[k].y > rect[k].x) & (rect[k].w > rect[k].z);
        }
        const uint64_t m = __ballot(vis);
        if (lane == 0) wv[k * 4 + w] = (uint32_t)__popcll(m);
        if (vis) visbits |= 1u << k;
    }
    __syncthreads();
    if (threadIdx.x < 64) {  // exclusive scan over the kKeyItems * 4 (round, wave) counts, in order
        const uint32_t c = threadIdx.x < kKeyItems * 4 ? wv[threadIdx.x] : 0u;
        const uint32_t inc = wave_incl_scan(c);
        if (threadIdx.x < kKeyItems * 4) wv[threadIdx.x] = block_off[blockIdx.x] + inc - c;
    }
    __syncthreads();
    const uint64_t lt = lanemask_lt();
#pragma unroll
    for (int k = 0; k < kKeyItems; k++) {
        const bool vis = (visbits >> k) & 1u;
        const uint64_t m = __ballot(vis);
        if (vis) {
            const int i = base + k * 256;
            const uint32_t pos = wv[k * 4 + w] + (uint32_t)__popcll(m & lt);
            keys[pos] = db[k];
            if constexpr (V64) {
                vals64[pos] = make_uint2((uint32_t)i, (uint32_t)rect[k].x | ((uint32_t)rect[k].y << 8) |
                                                          ((uint32_t)rect[k].z << 16) | ((uint32_t)rect[k].w << 24));
            } else {
                vals[pos] = pos;
                crec[pos] = make_uint4((uint32_t)rect[k].x | ((uint32_t)rect[k].y << 16),
                                       (uint32_t)rect[k].z | ((uint32_t)rect[k].w << 16), (uint32_t)i, 0u);
            }
        }
    }
}

__device__ __forceinline__ int4 unpack_box(uint2 b) {
    return make_int4((int)(b.x & 0xFFFFu), (int)(b.x >> 16), (int)(b.y & 0xFFFFu), (int)(b.y >> 16));
}

// ---------------------------------------------------------------------------
// Level 1: depth-ordered splats -> per-super-tile lists.
// ---------------------------------------------------------------------------

struct SuperBox {
    int sx0, sx1, sy0, sy1;  // inclusive super-tile range
};

__device__ __forceinline__ SuperBox super_box(int4 r) {
    return SuperBox{r.x / kSuper, (r.y - 1) / kSuper, r.z / kSuper, (r.w - 1) / kSuper};
}

// The part of box r inside super-tile (gxs, gys), in the super-tile's local
// tile coordinates, packed as c0 | c1 << 4 | r0 << 8 | r1 << 12 (each 0..8).
// Level 2 reads it with the entry instead of gathering the splat's record.
__device__ __forceinline__ uint32_t pack_local_rect(int4 r, int gxs, int gys) {
    const int tx0 = gxs * kSuper, ty0 = gys * kSuper;
    const int c0 = max(r.x - tx0, 0), c1 = min(r.y - tx0, kSuper);
    const int r0 = max(r.z - ty0, 0), r1 = min(r.w - ty0, kSuper);
    return (uint32_t)c0 | ((uint32_t)c1 << 4) | ((uint32_t)r0 << 8) | ((uint32_t)r1 << 12);
}

// Level-1 chunks hold 256 depth-ordered splats, one per thread; a splat covers
// few super-tiles, so each thread walks its own super-tile box.

__global__ __launch_bounds__(kL1Threads) void k_l1_count(const uint2 *sbox, int sxn, int nsuper, const Counters *cnt,
                                                         uint32_t *h1, const int32_t *overflow_dev) {
    extern __shared__ uint32_t cg[];  // [nsuper] splats of this chunk per super-tile
    if (*overflow_dev) return;
    const uint32_t c = blockIdx.x, c1 = cnt->c1, nv = cnt->n_visible;
    if (c >= c1) return;
    for (int g = threadIdx.x; g < nsuper; g += kL1Threads) cg[g] = 0;
    __syncthreads();
    uint32_t j = c * kL1Threads + threadIdx.x;
    if (j < nv) {
        SuperBox sb = super_box(unpack_box(sbox[j]));
        for (int gys = sb.sy0; gys <= sb.sy1; gys++)
            for (int gxs = sb.sx0; gxs <= sb.sx1; gxs++) atomicAdd(&cg[gys * sxn + gxs], 1u);
    }
    __syncthreads();
    for (int g = threadIdx.x; g < nsuper; g += kL1Threads) h1[(size_t)g * c1 + c] = cg[g];  // super-tile-major
}

// base1: per super-tile row, the exclusive prefix of its chunk counts; gtot:
// the rows' totals (the list lengths), whose exclusive scan gives each list's
// start.
__global__ __launch_bounds__(kL1Threads) void k_l1_scatter(const uint32_t *sid, const uint2 *sbox, int sxn, int nsuper,
                                                           const Counters *cnt, const uint32_t *base1,
                                                           const uint32_t *gtot, uint32_t *list1, uint32_t *list1r,
                                                           int64_t list1_cap, const int32_t *overflow_dev) {
    static_assert(kL1Threads == kScanThreads && 4 * kL1Threads >= kMaxSuperTiles, "four super-tiles per thread");
    // per super-tile: a 256-bit set of the chunk's covering threads, and the chunk's first slot
    extern __shared__ uint32_t lds1[];
    __shared__ uint32_t lw[kScanThreads / 64];
    uint32_t *bits = lds1;                   // [8][nsuper]: word-major (lanes of a wave hit distinct banks)
    uint32_t *first = lds1 + nsuper * 8;     // [nsuper]
    uint16_t *pre = reinterpret_cast<uint16_t *>(lds1 + nsuper * 9);  // [8][nsuper]: covering threads of the words before
    if (*overflow_dev) return;
    const uint32_t c = blockIdx.x, c1 = cnt->c1, nv = cnt->n_visible;
    if (c >= c1) return;
    // this thread's splat, list lengths and chunk prefixes: every load in flight at once
    const uint32_t j = c * kL1Threads + threadIdx.x;
    const uint32_t jc = min(j, nv - 1);  // nv >= 1 here (c < c1)
    const uint32_t id_in = sid[jc];
    const uint2 box_in = sbox[jc];
    const int g0 = 4 * threadIdx.x;
    uint32_t v[4], b1[4];
#pragma unroll
    for (int k = 0; k < 4; k++) {
        const int g = min(g0 + k, nsuper - 1);
        v[k] = gtot[g];
        b1[k] = base1[(size_t)g * c1 + c];
    }
    for (int k = threadIdx.x; k < nsuper * 8; k += kL1Threads) bits[k] = 0;
    {
        // first slot of this chunk in super-tile g: list start + the chunk's prefix in the row
        uint32_t sum = 0;
#pragma unroll
        for (int k = 0; k < 4; k++) {
            v[k] = g0 + k < nsuper ? v[k] : 0u;
            sum += v[k];
        }
        uint32_t tot;
        uint32_t off = block_excl_scan(sum, lw, &tot);
#pragma unroll
        for (int k = 0; k < 4; k++) {
            if (g0 + k < nsuper) first[g0 + k] = off + b1[k];
            off += v[k];
        }
    }
    __syncthreads();
    const int word = threadIdx.x >> 5;
    const uint32_t bit = 1u << (threadIdx.x & 31);
    uint32_t id = 0;
    int4 r = make_int4(0, 0, 0, 0);
    SuperBox sb{0, -1, 0, -1};
    if (j < nv) {
        id = id_in;
        r = unpack_box(box_in);
        sb = super_box(r);
    }
    for (int gys = sb.sy0; gys <= sb.sy1; gys++)
        for (int gxs = sb.sx0; gxs <= sb.sx1; gxs++) atomicOr(&bits[word * nsuper + gys * sxn + gxs], bit);
    __syncthreads();
    for (int g = threadIdx.x; g < nsuper; g += kL1Threads) {
        uint32_t c = 0;
#pragma unroll
        for (int k = 0; k < 8; k++) {
            pre[k * nsuper + g] = (uint16_t)c;
            c += (uint32_t)__popc(bits[k * nsuper + g]);
        }
    }
    __syncthreads();
    // rank = covering threads of lower index (depth order) -> stable
    for (int gys = sb.sy0; gys <= sb.sy1; gys++)
        for (int gxs = sb.sx0; gxs <= sb.sx1; gxs++) {
            const int g = gys * sxn + gxs;
            const uint32_t rank = pre[word * nsuper + g] + (uint32_t)__popc(bits[word * nsuper + g] & (bit - 1u));
            uint32_t pos = first[g] + rank;
            if ((int64_t)pos < list1_cap) {
                list1[pos] = id;
                list1r[pos] = pack_local_rect(r, gxs, gys);
            }
        }
}

// ---------------------------------------------------------------------------
// Level-2 plan: super-tile list spans, level-2 chunks, per-tile offsets of the
// (tile, chunk) count array in row-major tile order.
// ---------------------------------------------------------------------------

// (one workgroup of 1024 threads; nsuper <= 1024)
__device__ __forceinline__ void l2_plan(const uint32_t *gtot, Counters *cnt, int nsuper, int sxn, int gx, int gy,
                                        uint32_t *l1_start, uint32_t *l1_len, uint32_t *chunk2_start, uint32_t *toff) {
    __shared__ uint32_t lw[16];
    __shared__ uint32_t carry;
    __shared__ uint32_t n2s[1024];
    const int lane = threadIdx.x & 63, w = threadIdx.x >> 6;
    // spans (list lengths and their exclusive scan) and chunk counts (nsuper <= 1024)
    int g = threadIdx.x;
    const uint32_t len = g < nsuper ? gtot[g] : 0u;
    {
        const uint32_t inc1 = wave_incl_scan(len);
        if (lane == 63) lw[w] = inc1;
        __syncthreads();
        uint32_t woff = 0, tot = 0;
        for (int k = 0; k < 16; k++) {
            if (k < w) woff += lw[k];
            tot += lw[k];
        }
        if (g < nsuper) {
            l1_start[g] = woff + inc1 - len;
            l1_len[g] = len;
        }
        if (g == 0) cnt->total1 = tot;
        __syncthreads();
    }
    uint32_t n2 = 0;
    if (g < nsuper) {
        n2 = (len + kL2Threads - 1) / kL2Threads;
        n2s[g] = n2;
    }
    uint32_t inc = wave_incl_scan(n2);
    if (lane == 63) lw[w] = inc;
    __syncthreads();
    uint32_t woff = 0, tot = 0;
    for (int k = 0; k < 16; k++) {
        if (k < w) woff += lw[k];
        tot += lw[k];
    }
    if (g < nsuper) chunk2_start[g] = woff + inc - n2;
    if (g == 0) {
        chunk2_start[nsuper] = tot;
        cnt->total2 = tot;
        carry = 0;
    }
    __syncthreads();
    // toff[t] = exclusive scan over row-major tiles of the chunk count of t's super-tile
    const int ntile = gx * gy;
    for (int base = 0; base < ntile; base += 1024) {
        int t = base + threadIdx.x;
        uint32_t v = 0;
        if (t < ntile) {
            int tx = t % gx, ty = t / gx;
            v = n2s[(ty / kSuper) * sxn + tx / kSuper];
        }
        uint32_t inc2 = wave_incl_scan(v);
        __syncthreads();
        if (lane == 63) lw[w] = inc2;
        __syncthreads();
        uint32_t wo = 0, tt = 0;
        for (int k = 0; k < 16; k++) {
            if (k < w) wo += lw[k];
            tt += lw[k];
        }
        uint32_t cc = carry;
        if (t < ntile) toff[t] = cc + wo + inc2 - v;
        __syncthreads();
        if (threadIdx.x == 0) carry = cc + tt;
    }
    __syncthreads();
    if (threadIdx.x == 0) {
        toff[ntile] = carry;
        cnt->h2_count = carry;
    }
}

__global__ __launch_bounds__(1024) void k_l2_plan(const uint32_t *gtot, Counters *cnt, int nsuper, int sxn, int gx,
                                                  int gy, uint32_t *l1_start, uint32_t *l1_len, uint32_t *chunk2_start,
                                                  uint32_t *toff, const int32_t *overflow_dev) {
    if (*overflow_dev) return;
    l2_plan(gtot, cnt, nsuper, sxn, gx, gy, l1_start, l1_len, chunk2_start, toff);
}

// ---------------------------------------------------------------------------
// Level 2: one super-tile list chunk per workgroup iteration.
// ---------------------------------------------------------------------------

struct L2Chunk {
    int g;         // super-tile
    uint32_t c2;   // chunk index within the super-tile
    uint32_t len;  // entries in this chunk
    uint32_t first;  // index into list1 of the chunk's first entry
};

// chunk2_start is the workgroup's LDS copy
__device__ __forceinline__ L2Chunk l2_locate(uint32_t wi, const uint32_t *chunk2_start, int nsuper,
                                             const uint32_t *l1_start, const uint32_t *l1_len) {
    int lo = 0, hi = nsuper - 1;  // largest g with chunk2_start[g] <= wi
    while (lo < hi) {
        int mid = (lo + hi + 1) >> 1;
        if (chunk2_start[mid] <= wi) lo = mid; else hi = mid - 1;
    }
    L2Chunk C;
    C.g = lo;
    C.c2 = wi - chunk2_start[lo];
    uint32_t off = C.c2 * kL2Threads;
    C.len = min((uint32_t)kL2Threads, l1_len[lo] - off);
    C.first = l1_start[lo] + off;
    return C;
}

// Columns [c0, c1) and rows [r0, r1) of super-tile g covered by box r, in the
// super-tile's local coordinates (empty when invalid).
struct LRect {
    int c0, c1, r0, r1;
};

__device__ __forceinline__ LRect l2_local_rect(bool valid, uint32_t packed) {
    LRect L{0, 0, 0, 0};
    if (!valid) return L;
    const int c0 = packed & 15u, c1 = (packed >> 4) & 15u, r0 = (packed >> 8) & 15u, r1 = (packed >> 12) & 15u;
    if (c1 <= c0 || r1 <= r0) return L;
    return LRect{c0, c1, r0, r1};
}

// number of lanes below this one whose bit is set in m
__device__ __forceinline__ uint32_t rank_below(uint64_t m) {
    return __builtin_amdgcn_mbcnt_hi((uint32_t)(m >> 32), __builtin_amdgcn_mbcnt_lo((uint32_t)m, 0u));
}

static_assert(kSuper * kSuper == 64, "a super-tile has one tile per lane");
static_assert(kSuper == 8, "column and row masks are 8 ballots each");

// A lane covers tile (c, r) iff it covers column c and row r, so the wave's
// lanes covering the tile are colB[c] & rowB[r]: sixteen ballots give all 64
// tile masks.  Lane 0 also stores them to the wave's LDS slots (the ballots
// are used again after the branch, so they stay in wave-uniform code).
__device__ __forceinline__ void l2_colrow(const LRect &L, uint64_t (&colB)[kSuper], uint64_t (&rowB)[kSuper],
                                          uint64_t *lds_masks) {
#pragma unroll
    for (int c = 0; c < kSuper; c++) colB[c] = __ballot((c >= L.c0) & (c < L.c1));
#pragma unroll
    for (int r = 0; r < kSuper; r++) rowB[r] = __ballot((r >= L.r0) & (r < L.r1));
    if ((threadIdx.x & 63) == 0) {
#pragma unroll
        for (int k = 0; k < kSuper; k++) {
            lds_masks[k] = colB[k];
            lds_masks[kSuper + k] = rowB[k];
        }
    }
}

// The lanes of one wavefront see each other's LDS writes: a wavefront's LDS
// operations complete in order, so only the compiler has to keep them in place.
__device__ __forceinline__ void wave_lds_sync() {
    __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
    __builtin_amdgcn_wave_barrier();
    __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
}

// wc[w * 64 + tl] = lanes of wave w covering tile tl (lane tl computes it from
// the wave's masks in LDS; wave-major, so the lanes write distinct banks).
// The masks are the wave's own: a wave_lds_sync between l2_colrow and this.
__device__ __forceinline__ void l2_counts(const uint64_t *lds_masks, uint32_t *wc) {
    const int lane = threadIdx.x & 63, w = threadIdx.x >> 6;
    const uint64_t m = lds_masks[lane & (kSuper - 1)] & lds_masks[kSuper + lane / kSuper];
    wc[w * 64 + lane] = (uint32_t)__popcll(m);
}

// The tables the chunk lookup reads (chunk starts, list starts and lengths per
// super-tile), copied to LDS once per workgroup.
struct L2Tables {
    uint32_t c2s[kMaxSuperTiles + 1], l1s[kMaxSuperTiles], l1l[kMaxSuperTiles];
};

__device__ __forceinline__ void l2_load_tables(L2Tables &T, const uint32_t *chunk2_start, const uint32_t *l1_start,
                                               const uint32_t *l1_len, int nsuper) {
    for (int g = threadIdx.x; g <= nsuper; g += kL2Threads) {
        T.c2s[g] = chunk2_start[g];
        if (g < nsuper) {
            T.l1s[g] = l1_start[g];
            T.l1l[g] = l1_len[g];
        }
    }
}

// Tile (tx, ty) of lane tl of super-tile g, clamped to the image: the clamped
// tile lies in the same super-tile (every super-tile holds a tile of the
// image), so indices derived from it stay inside g's part of the count arrays.
__device__ __forceinline__ int l2_tile_clamped(int g, int tl, int sxn, int gx, int gy, bool &inside) {
    const int tx = (g % sxn) * kSuper + (tl & (kSuper - 1)), ty = (g / sxn) * kSuper + tl / kSuper;
    inside = (tx < gx) & (ty < gy);
    return min(ty, gy - 1) * gx + min(tx, gx - 1);
}

// Each workgroup walks its chunks one at a time and issues the next chunk's
// global loads (list entries, count offsets) before it works on the current
// one; they are waited for just before the current chunk's stores, so a
// chunk's round trips overlap the previous chunk's work and no load waits
// behind a store (vmcnt counts both).  One chunk in flight keeps the register
// count (and the number of resident workgroups) of the plain loop.
struct L2Next {
    L2Chunk C;
    uint32_t packed, hoff;
    bool tin;
};

__device__ __forceinline__ void l2_fetch_count(L2Next &x, uint32_t wi, const L2Tables &T, int nsuper,
                                               const uint32_t *list1r, const uint32_t *toff, int sxn, int gx, int gy) {
    x.C = l2_locate(wi, T.c2s, nsuper, T.l1s, T.l1l);
    x.packed = list1r[x.C.first + min((uint32_t)threadIdx.x, x.C.len - 1)];
    x.hoff = toff[l2_tile_clamped(x.C.g, threadIdx.x & 63, sxn, gx, gy, x.tin)];
}

__global__ __launch_bounds__(kL2Threads) void k_l2_count(const uint32_t *list1r, const uint32_t *l1_start,
                                                         const uint32_t *l1_len, const uint32_t *chunk2_start,
                                                         const uint32_t *toff, int gx, int gy, int sxn, int nsuper,
                                                         const Counters *cnt, uint32_t *h2,
                                                         const int32_t *overflow_dev) {
    // wc is double-buffered by chunk parity: a wave may start the next chunk while
    // wave 0 still sums this one's counts (one barrier per chunk)
    __shared__ uint32_t wc[2][kSuper * kSuper * kL2Waves];
    __shared__ L2Tables T;
    __shared__ uint64_t masks[kL2Waves][2 * kSuper];
    if (*overflow_dev) return;
    const uint32_t total2 = cnt->total2;
    const int w = threadIdx.x >> 6, tl = threadIdx.x & 63;
    int par = 0;
    const uint32_t G = gridDim.x;
    if (blockIdx.x >= total2) return;
    l2_load_tables(T, chunk2_start, l1_start, l1_len, nsuper);
    __syncthreads();
    L2Next cur, nxt;
    l2_fetch_count(cur, blockIdx.x, T, nsuper, list1r, toff, sxn, gx, gy);
    for (uint32_t wi = blockIdx.x; wi < total2; wi += G) {
        const bool more = wi + G < total2;  // uniform over the workgroup
        if (more) l2_fetch_count(nxt, wi + G, T, nsuper, list1r, toff, sxn, gx, gy);
        const bool valid = threadIdx.x < cur.C.len;
        uint64_t colB[kSuper], rowB[kSuper];
        l2_colrow(l2_local_rect(valid, cur.packed), colB, rowB, masks[w]);
        wave_lds_sync();
        l2_counts(masks[w], wc[par]);
        __syncthreads();
        uint32_t sum = 0;
        if (threadIdx.x < kSuper * kSuper && cur.tin)
            for (int k = 0; k < kL2Waves; k++) sum += wc[par][k * 64 + tl];
        // the next chunk's loads land before this store (pinned on every path: a pin
        // under the same condition as the loads leaves the wait analysis a path with a
        // load in flight, and every later store would wait for it)
        pin_u32(nxt.packed, nxt.hoff);
        if (threadIdx.x < kSuper * kSuper && cur.tin) h2[cur.hoff + cur.C.c2] = sum;
        cur = nxt;
        par ^= 1;
    }
}

// [start, end) of tile t in the final list: the first slot of its first
// level-2 chunk (or K when the tile has none after it).
__device__ __forceinline__ void tile_range(const uint32_t *base2, const uint32_t *toff, int t, const Counters *cnt,
                                           uint32_t *ranges) {
    const uint32_t h2 = cnt->h2_count;
    const uint32_t K = (uint32_t)cnt->K;
    uint32_t a = toff[t], b = toff[t + 1];
    ranges[2 * t] = a < h2 ? base2[a] : K;
    ranges[2 * t + 1] = b < h2 ? base2[b] : K;
}

// (only when there are no splats: otherwise the level-2 scatter writes the ranges)
__global__ __launch_bounds__(256) void k_bin_ranges(const uint32_t *base2, const uint32_t *toff, int ntile,
                                                    const Counters *cnt, uint32_t *ranges,
                                                    const int32_t *overflow_dev) {
    if (*overflow_dev) return;
    int t = blockIdx.x * blockDim.x + threadIdx.x;
    if (t >= ntile) return;
    tile_range(base2, toff, t, cnt, ranges);
}

// The ranked stores of one wave for all 64 tiles of its super-tile: for tile
// (r, c) the covering lanes are colB[c] & rowB[r]; exec is set to that mask
// directly (an empty mask skips the tile), the lane's rank is an mbcnt on exec,
// and the run's first byte offset is lane tl of slot4 (this wave's first slot
// in tile tl, times 4).  One scalar instruction and one branch per tile, four
// vector instructions and a store per covered tile; exec is restored once at
// the end (the compiled loop spent five scalar instructions per covered tile
// and three per empty one).  The offsets are 32-bit: callers keep positions
// below 2^30.
#define L2_TILE(R, C, T)                                                 \
    "s_and_b64 exec, %[c" C "], %[r" R "]\n\t"                           \
    "s_cbranch_execz 1f\n\t"                                             \
    "v_readlane_b32 %[s0], %[slot4], " T "\n\t"                          \
    "v_mbcnt_lo_u32_b32 %[off], exec_lo, 0\n\t"                          \
    "v_mbcnt_hi_u32_b32 %[off], exec_hi, %[off]\n\t"                     \
    "v_lshl_add_u32 %[off], %[off], 2, %[s0]\n\t"                        \
    "global_store_dword %[off], %[id], %[base]\n\t"                      \
    "1:\n\t"

__device__ __forceinline__ void store_all_tiles(uint32_t *base, const uint64_t (&colB)[kSuper],
                                                const uint64_t (&rowB)[kSuper], uint32_t slot4, uint32_t id) {
    uint64_t saved;
    uint32_t off, s0;
    asm volatile(
        "s_mov_b64 %[saved], exec\n\t"
    L2_TILE("0", "0", "0")
    L2_TILE("0", "1", "1")
    L2_TILE("0", "2", "2")
    L2_TILE("0", "3", "3")
    L2_TILE("0", "4", "4")
    L2_TILE("0", "5", "5")
    L2_TILE("0", "6", "6")
    L2_TILE("0", "7", "7")
    L2_TILE("1", "0", "8")
    L2_TILE("1", "1", "9")
    L2_TILE("1", "2", "10")
    L2_TILE("1", "3", "11")
    L2_TILE("1", "4", "12")
    L2_TILE("1", "5", "13")
    L2_TILE("1", "6", "14")
    L2_TILE("1", "7", "15")
    L2_TILE("2", "0", "16")
    L2_TILE("2", "1", "17")
    L2_TILE("2", "2", "18")
    L2_TILE("2", "3", "19")
    L2_TILE("2", "4", "20")
    L2_TILE("2", "5", "21")
    L2_TILE("2", "6", "22")
    L2_TILE("2", "7", "23")
    L2_TILE("3", "0", "24")
    L2_TILE("3", "1", "25")
    L2_TILE("3", "2", "26")
    L2_TILE("3", "3", "27")
    L2_TILE("3", "4", "28")
    L2_TILE("3", "5", "29")
    L2_TILE("3", "6", "30")
    L2_TILE("3", "7", "31")
    L2_TILE("4", "0", "32")
    L2_TILE("4", "1", "33")
    L2_TILE("4", "2", "34")
    L2_TILE("4", "3", "35")
    L2_TILE("4", "4", "36")
    L2_TILE("4", "5", "37")
    L2_TILE("4", "6", "38")
    L2_TILE("4", "7", "39")
    L2_TILE("5", "0", "40")
    L2_TILE("5", "1", "41")
    L2_TILE("5", "2", "42")
    L2_TILE("5", "3", "43")
    L2_TILE("5", "4", "44")
    L2_TILE("5", "5", "45")
    L2_TILE("5", "6", "46")
    L2_TILE("5", "7", "47")
    L2_TILE("6", "0", "48")
    L2_TILE("6", "1", "49")
    L2_TILE("6", "2", "50")
    L2_TILE("6", "3", "51")
    L2_TILE("6", "4", "52")
    L2_TILE("6", "5", "53")
    L2_TILE("6", "6", "54")
    L2_TILE("6", "7", "55")
    L2_TILE("7", "0", "56")
    L2_TILE("7", "1", "57")
    L2_TILE("7", "2", "58")
    L2_TILE("7", "3", "59")
    L2_TILE("7", "4", "60")
    L2_TILE("7", "5", "61")
    L2_TILE("7", "6", "62")
    L2_TILE("7", "7", "63")
        "s_mov_b64 exec, %[saved]\n\t"
        : [saved] "=&s"(saved), [off] "=&v"(off), [s0] "=&s"(s0)
        : [c0] "s"(colB[0]), [c1] "s"(colB[1]), [c2] "s"(colB[2]), [c3] "s"(colB[3]), [c4] "s"(colB[4]),
          [c5] "s"(colB[5]), [c6] "s"(colB[6]), [c7] "s"(colB[7]), [r0] "s"(rowB[0]), [r1] "s"(rowB[1]),
          [r2] "s"(rowB[2]), [r3] "s"(rowB[3]), [r4] "s"(rowB[4]), [r5] "s"(rowB[5]), [r6] "s"(rowB[6]),
          [r7] "s"(rowB[7]), [slot4] "v"(slot4), [id] "v"(id), [base] "s"(base)
        : "memory");
}
#undef L2_TILE

// The next chunk of the level-2 scatter: entries (splat index, local
// rectangle) and this thread's (wave, tile) slot base.  The slot base is two
// dependent loads (the tile's count offset, then the scanned count): the
// offset is fetched with the entries, the base one step later.
struct L2NextS {
    L2Chunk C;
    uint32_t id, packed, sbase;
    bool tin;
};

__device__ __forceinline__ void l2_fetch_scatter(L2NextS &x, uint32_t wi, const L2Tables &T, int nsuper,
                                                 const uint32_t *list1, const uint32_t *list1r, const uint32_t *toff,
                                                 int sxn, int gx, int gy) {
    x.C = l2_locate(wi, T.c2s, nsuper, T.l1s, T.l1l);
    const uint32_t e = x.C.first + min((uint32_t)threadIdx.x, x.C.len - 1);
    x.id = list1[e];
    x.packed = list1r[e];
    x.sbase = toff[l2_tile_clamped(x.C.g, threadIdx.x & 63, sxn, gx, gy, x.tin)];
}

// FAST: values only, capacity below 2^30 (32-bit byte offsets); otherwise the
// generic loop, which also writes the optional (tile, depth) keys.
template <bool FAST>
__global__ __launch_bounds__(kL2Threads) void k_l2_scatter(const uint32_t *list1, const uint32_t *list1r,
                                                           const uint32_t *l1_start, const uint32_t *l1_len,
                                                           const uint32_t *chunk2_start, const uint32_t *toff,
                                                           const uint32_t *base2, const float *depth, int gx, int gy,
                                                           int sxn, int nsuper, const Counters *cnt, int64_t k_capacity,
                                                           uint64_t *keys, uint32_t *vals, uint32_t *ranges,
                                                           const int32_t *overflow_dev) {
    // wc is double-buffered by chunk parity: one barrier per chunk (a wave may
    // start the next chunk while others still read this one's counts)
    __shared__ uint32_t wc[2][kSuper * kSuper * kL2Waves];
    __shared__ L2Tables T;
    __shared__ uint64_t masks[kL2Waves][2 * kSuper];
    if (*overflow_dev) return;
    const uint32_t total2 = cnt->total2;
    const int lane = threadIdx.x & 63, w = threadIdx.x >> 6;
    int par = 0;
    for (int t = blockIdx.x * kL2Threads + threadIdx.x; t < gx * gy; t += gridDim.x * kL2Threads)
        tile_range(base2, toff, t, cnt, ranges);
    const uint32_t G = gridDim.x;
    if (blockIdx.x >= total2) return;
    l2_load_tables(T, chunk2_start, l1_start, l1_len, nsuper);
    __syncthreads();
    const uint32_t cap32 = (uint32_t)min(k_capacity, (int64_t)0xFFFFFFFFll);
    L2NextS cur, nxt;
    l2_fetch_scatter(cur, blockIdx.x, T, nsuper, list1, list1r, toff, sxn, gx, gy);
    cur.sbase = base2[cur.sbase + cur.C.c2];
    uint32_t db = (!FAST && keys) ? __float_as_uint(depth[cur.id]) : 0u;  // depth only for the optional keys
    for (uint32_t wi = blockIdx.x; wi < total2; wi += G) {
        const bool more = wi + G < total2;  // uniform over the workgroup
        if (more) l2_fetch_scatter(nxt, wi + G, T, nsuper, list1, list1r, toff, sxn, gx, gy);
        const bool valid = threadIdx.x < cur.C.len;
        uint64_t colB[kSuper], rowB[kSuper];
        l2_colrow(l2_local_rect(valid, cur.packed), colB, rowB, masks[w]);
        wave_lds_sync();
        l2_counts(masks[w], wc[par]);
        __syncthreads();
        const int tx0 = (cur.C.g % sxn) * kSuper, ty0 = (cur.C.g / sxn) * kSuper;
        // lane tl: this wave's first slot in tile tl (broadcast per tile with v_readlane)
        uint32_t myslot = cur.sbase;
        for (int k = 0; k < w; k++) myslot += wc[par][k * 64 + lane];
        // the next chunk's slot base (its count offset has landed by now) and depth
        uint32_t dbn = 0;
        if (more) {
            nxt.sbase = base2[nxt.sbase + nxt.C.c2];
            if (!FAST && keys) dbn = __float_as_uint(depth[nxt.id]);
        }
        bool inside = true;
        if constexpr (FAST) {
            // every run of this wave lies inside the capacity (K <= capacity is decided
            // before any instance is written; this test only guards the stores)
            const uint32_t myc = wc[par][w * 64 + lane];
            inside = __ballot(myc != 0u && myslot + myc > cap32) == 0ull;
        }
        pin_u32(nxt.id, nxt.packed, nxt.sbase, dbn);  // the next chunk's loads land before the stores (every path)
        if constexpr (FAST) {
            if (inside) store_all_tiles(vals, colB, rowB, myslot << 2, cur.id);
        } else
        for (int rr = 0; rr < kSuper; rr++) {
            if (rowB[rr] == 0ull || !inside) continue;  // no lane of this wave covers the row (uniform)
            for (int cc = 0; cc < kSuper; cc++) {
                const uint64_t m = colB[cc] & rowB[rr];
                if (m == 0ull) continue;
                const int tl = rr * kSuper + cc;
                const uint32_t s0 = (uint32_t)__builtin_amdgcn_readlane((int)myslot, tl);
                if ((m >> lane) & 1ull) {
                    const uint32_t pos = s0 + rank_below(m);
                    if (pos < cap32) {
                        vals[pos] = cur.id;
                        if (keys) keys[pos] = ((uint64_t)(uint32_t)((ty0 + rr) * gx + tx0 + cc) << 32) | db;
                    }
                }
            }
        }
        cur = nxt;
        db = dbn;
        par ^= 1;
    }
}



inline size_t align_up(size_t x) { return (x + 255) & ~(size_t)255; }

struct WsLayout {
    size_t counters, blockvis, blockarea, keysA, valsA, keysB, valsB, crec, sid, sbox, hist, h1, list1, list1r, l1start,
        l1len, c2start, toff, h2, parts, gtot, total;
    uint32_t hist_n, h1_n, h2_n;
};

inline int super_count(int gx, int gy) {
    return ((gx + kSuper - 1) / kSuper) * ((gy + kSuper - 1) / kSuper);
}

WsLayout layout(int n, int gx, int gy, int64_t k_capacity) {
    WsLayout L;
    const int ntile = gx * gy, nsuper = super_count(gx, gy);
    size_t off = 0;
    const size_t nkb = ((size_t)n + kKeyTile - 1) / kKeyTile;
    const size_t nblk = ((size_t)n + kRadixTile - 1) / kRadixTile;
    const size_t c1max = ((size_t)n + kL1Threads - 1) / kL1Threads;
    const size_t cap = (size_t)std::max<int64_t>(k_capacity, 1);
    const size_t total2max = cap / kL2Threads + nsuper + 1;
    L.hist_n = (uint32_t)(256 * nblk + 256);  // per-block digit counts + the digit totals
    L.h1_n = (uint32_t)(nsuper * c1max);
    L.h2_n = (uint32_t)std::min<size_t>((size_t)kSuper * kSuper * total2max, 0xFFFFFFFFull);
    size_t parts_n = (std::max<size_t>({L.hist_n, L.h1_n, L.h2_n}) + kScanBlock - 1) / kScanBlock + 1;
    L.counters = off; off += align_up(sizeof(Counters));
    L.blockvis = off; off += align_up(nkb * 4);
    L.blockarea = off; off += align_up(nkb * 4);
    L.keysA = off; off += align_up((size_t)n * 4);
    L.valsA = off; off += align_up((size_t)n * 4);
    L.keysB = off; off += align_up((size_t)n * 4);
    L.valsB = off; off += align_up((size_t)n * 4);
    L.crec = off; off += align_up((size_t)n * 16);
    L.sid = off; off += align_up((size_t)n * 4);
    L.sbox = off; off += align_up((size_t)n * 8);
    L.hist = off; off += align_up((size_t)L.hist_n * 4);
    L.h1 = off; off += align_up((size_t)L.h1_n * 4);
    L.list1 = off; off += align_up(cap * 4);
    L.list1r = off; off += align_up(cap * 4);
    L.l1start = off; off += align_up((size_t)(nsuper + 1) * 4);
    L.l1len = off; off += align_up((size_t)(nsuper + 1) * 4);
    L.c2start = off; off += align_up((size_t)(nsuper + 1) * 4);
    L.toff = off; off += align_up((size_t)(ntile + 1) * 4);
    L.h2 = off; off += align_up((size_t)L.h2_n * 4);
    L.parts = off; off += align_up(parts_n * 4);
    L.gtot = off; off += align_up((size_t)(nsuper + 1) * 4);
    L.total = off;
    return L;
}

}  // namespace

size_t scan_parts_words(uint32_t max_count) { return (size_t)(max_count + kScanBlock - 1) / kScanBlock + 1; }

size_t radix_hist_words(uint32_t max_count) {
    return 256 * ((size_t)(max_count + kRadixTile - 1) / kRadixTile) + 256;  // + the digit totals
}

hipError_t scan_u32(uint32_t *data, const uint32_t *count_dev, uint32_t max_count, uint32_t *parts,
                    uint32_t *total_out, const int32_t *skip, hipStream_t s) {
    return scan_exclusive(data, count_dev, max_count, parts, total_out, skip, s);
}

hipError_t radix_sort_pairs(uint32_t *kA, uint32_t *vA, uint32_t *kB, uint32_t *vB, const uint32_t *count_dev,
                            uint32_t max_count, int bits, uint32_t *hist, const int32_t *skip, hipStream_t s) {
    if (max_count == 0) return hipSuccess;
    const int nblk = (int)((max_count + kRadixTile - 1) / kRadixTile);
    uint32_t *ki = kA, *vi = vA, *ko = kB, *vo = vB;
    for (int shift = 0; shift < bits; shift += 8) {
        hipLaunchKernelGGL(k_radix_hist, dim3(nblk), dim3(kRadixThreads), 0, s, ki, count_dev, shift, hist, nblk, skip);
        hipLaunchKernelGGL(k_rowscan<kScanThreads>, dim3(256), dim3(kScanThreads), 0, s, hist, nullptr, (uint32_t)nblk,
                           hist + (size_t)256 * nblk, skip);
        hipLaunchKernelGGL((k_radix_scatter<uint32_t, false>), dim3(nblk), dim3(kRadixThreads), 0, s, ki, vi, ko, vo,
                           count_dev, shift, hist, nblk, skip, nullptr, nullptr, nullptr);
        std::swap(ki, ko);
        std::swap(vi, vo);
    }
    return hipGetLastError();
}

int binsort_super_tiles(int width, int height) {
    return super_count((width + kTile - 1) / kTile, (height + kTile - 1) / kTile);
}

size_t binsort_workspace(int n, int width, int height, int64_t k_capacity) {
    const int gx = (width + kTile - 1) / kTile, gy = (height + kTile - 1) / kTile;
    return layout(n, gx, gy, k_capacity).total;
}

hipError_t launch_bin_sort(const darb_projected &p, int n, int width, int height, int64_t k_capacity, void *ws,
                           uint64_t *keys, uint32_t *vals, uint32_t *ranges, int64_t *k_dev, int32_t *overflow_dev,
                           hipStream_t s) {
    const int gx = (width + kTile - 1) / kTile, gy = (height + kTile - 1) / kTile, ntile = gx * gy;
    const int sxn = (gx + kSuper - 1) / kSuper, nsuper = super_count(gx, gy);
    WsLayout L = layout(n, gx, gy, k_capacity);
    char *base = static_cast<char *>(ws);
    auto U = [&](size_t o) { return reinterpret_cast<uint32_t *>(base + o); };
    Counters *cnt = reinterpret_cast<Counters *>(base + L.counters);
    uint32_t *kA = U(L.keysA), *vA = U(L.valsA), *kB = U(L.keysB), *vB = U(L.valsB);
    uint32_t *hist = U(L.hist), *parts = U(L.parts), *h1 = U(L.h1), *list1 = U(L.list1), *list1r = U(L.list1r), *h2 = U(L.h2);
    uint32_t *blockvis = U(L.blockvis), *blockarea = U(L.blockarea);
    uint32_t *l1start = U(L.l1start), *l1len = U(L.l1len), *c2start = U(L.c2start), *toff = U(L.toff);
    uint32_t *gtot = U(L.gtot);
    const uint32_t *nvis = &cnt->n_visible;
    hipError_t e;

    const int nkb = (n + kKeyTile - 1) / kKeyTile;
    const int2 *ext = reinterpret_cast<const int2 *>(p.extent);
    if (n > 0) hipLaunchKernelGGL(k_bin_keys, dim3(nkb), dim3(256), 0, s, p.xy, ext, n, gx, gy, blockvis, blockarea);
    hipLaunchKernelGGL(k_bin_sizes, dim3(1), dim3(1024), 0, s, blockvis, blockarea, nkb, cnt, k_capacity, k_dev,
                       overflow_dev);
    uint32_t *sid = U(L.sid);
    uint2 *sbox = reinterpret_cast<uint2 *>(base + L.sbox);
    if (n > 0) {
        uint4 *crec = reinterpret_cast<uint4 *>(base + L.crec);
        // grids of at most 255 x 255 tiles carry (splat index, box) through the sort
        // as a 64-bit value (in the record area); larger grids gather the record in
        // the last pass
        const bool v64 = gx <= 255 && gy <= 255;
        uint2 *v64A = reinterpret_cast<uint2 *>(base + L.crec), *v64B = v64A + n;
        if (v64)
            hipLaunchKernelGGL(k_bin_compact<true>, dim3(nkb), dim3(256), 0, s, p.xy, ext, p.depth, n, gx, gy,
                               blockvis, kA, nullptr, nullptr, v64A, overflow_dev);
        else
            hipLaunchKernelGGL(k_bin_compact<false>, dim3(nkb), dim3(256), 0, s, p.xy, ext, p.depth, n, gx, gy,
                               blockvis, kA, vA, crec, nullptr, overflow_dev);
        // depth sort of the N_v visible keys: 4 passes of 8 bits
        const int nblk = (n + kRadixTile - 1) / kRadixTile;
        uint32_t *ki = kA, *vi = vA, *ko = kB, *vo = vB;
        uint2 *wi = v64A, *wo = v64B;
        // (the last pass writes the splat index and tile box of each value, in
        // (depth, index) order, instead of the sorted pairs)
        for (int shift = 0; shift < 32; shift += 8) {
            hipLaunchKernelGGL(k_radix_hist, dim3(nblk), dim3(kRadixThreads), 0, s, ki, nvis, shift, hist, nblk,
                               overflow_dev);
            hipLaunchKernelGGL(k_rowscan<kScanThreads>, dim3(256), dim3(kScanThreads), 0, s, hist, nullptr, (uint32_t)nblk,
                               hist + (size_t)256 * nblk, overflow_dev);
            const bool last = shift == 24;
            if (v64 && !last)
                hipLaunchKernelGGL((k_radix_scatter<uint2, false>), dim3(nblk), dim3(kRadixThreads), 0, s, ki, wi, ko,
                                   wo, nvis, shift, hist, nblk, overflow_dev, nullptr, nullptr, nullptr);
            else if (v64)
                hipLaunchKernelGGL((k_radix_scatter<uint2, true>), dim3(nblk), dim3(kRadixThreads), 0, s, ki, wi, ko,
                                   wo, nvis, shift, hist, nblk, overflow_dev, nullptr, sid, sbox);
            else if (!last)
                hipLaunchKernelGGL((k_radix_scatter<uint32_t, false>), dim3(nblk), dim3(kRadixThreads), 0, s, ki, vi,
                                   ko, vo, nvis, shift, hist, nblk, overflow_dev, nullptr, nullptr, nullptr);
            else
                hipLaunchKernelGGL((k_radix_scatter<uint32_t, true>), dim3(nblk), dim3(kRadixThreads), 0, s, ki, vi, ko,
                                   vo, nvis, shift, hist, nblk, overflow_dev, crec, sid, sbox);
            std::swap(ki, ko);
            std::swap(vi, vo);
            std::swap(wi, wo);
        }
        const int c1max = (n + kL1Threads - 1) / kL1Threads;
        const size_t lds1 = (size_t)nsuper * 4;
        hipLaunchKernelGGL(k_l1_count, dim3(c1max), dim3(kL1Threads), lds1, s, sbox, sxn, nsuper, cnt, h1,
                           overflow_dev);
    }
    // the level-1 lists' lengths (zeros when nothing is visible: rows of length c1 = 0)
    hipLaunchKernelGGL(k_rowscan<1024>, dim3(nsuper), dim3(1024), 0, s, h1, &cnt->c1, 0u, gtot, overflow_dev);
    if (n > 0) {
        const int c1max = (n + kL1Threads - 1) / kL1Threads;
        const size_t lds1 = (size_t)nsuper * 4;
        hipLaunchKernelGGL(k_l1_scatter, dim3(c1max), dim3(kL1Threads), 13 * lds1, s, sid, sbox, sxn, nsuper, cnt, h1,
                           gtot, list1, list1r, std::max<int64_t>(k_capacity, 1), overflow_dev);
    }
    hipLaunchKernelGGL(k_l2_plan, dim3(1), dim3(1024), 0, s, gtot, cnt, nsuper, sxn, gx, gy, l1start, l1len, c2start,
                       toff, overflow_dev);
    if (n > 0) {
        hipLaunchKernelGGL(k_l2_count, dim3(kL2Grid), dim3(kL2Threads), 0, s, list1r, l1start, l1len, c2start, toff, gx,
                           gy, sxn, nsuper, cnt, h2, overflow_dev);
        if ((e = scan_exclusive(h2, &cnt->h2_count, L.h2_n, parts, &cnt->scan_total, overflow_dev, s)) != hipSuccess)
            return e;
        if (!keys && k_capacity < (int64_t)1 << 30)
            hipLaunchKernelGGL(k_l2_scatter<true>, dim3(kL2Grid), dim3(kL2Threads), 0, s, list1, list1r, l1start, l1len,
                               c2start, toff, h2, p.depth, gx, gy, sxn, nsuper, cnt, k_capacity, keys, vals, ranges,
                               overflow_dev);
        else
            hipLaunchKernelGGL(k_l2_scatter<false>, dim3(kL2Grid), dim3(kL2Threads), 0, s, list1, list1r, l1start, l1len,
                               c2start, toff, h2, p.depth, gx, gy, sxn, nsuper, cnt, k_capacity, keys, vals, ranges,
                               overflow_dev);
    } else {
        hipLaunchKernelGGL(k_bin_ranges, dim3((ntile + 255) / 256), dim3(256), 0, s, h2, toff, ntile, cnt, ranges,
                           overflow_dev);
    }
    return hipGetLastError();
}

}  // namespace darb
