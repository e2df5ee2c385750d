// binsort.hip -- tile binning and per-tile depth order.
//
// Target order: instances (tile, splat) sorted by (tile, depth bits, splat
// index).  Instead of a 45-bit radix sort over all K instances, the sort is
// split so that K-sized data is written exactly once:
//   1. keys     one thread per splat: depth bits for visible splats, a key
//               above every finite depth for the rest; splat index as value.
//   2. sort     stable LSD radix sort (8-bit digits) of the n (key, index)
//               pairs -> splats in (depth, index) order.
//   3. count    the depth-ordered splats are cut into chunks of kChunk; one
//               wavefront per chunk builds the chunk's per-tile histogram in
//               LDS and stores it tile-major: H[t * chunks + c].
//   4. scan     one exclusive scan over H gives, for every (tile, chunk), the
//               first output slot: slots of tile t come after all tiles < t,
//               and within a tile after all earlier chunks.
//   5. scatter  one wavefront per chunk loads its row of slots into LDS and
//               walks its splats in depth order; per splat the lanes cover the
//               splat's tile rectangle and claim slots with LDS fetch-adds,
//               whose in-order execution within a wavefront keeps the order
//               stable.
// The radius box of every splat is recomputed from (xy, radius) with the same
// FP32 expression everywhere.  HBM-bound.
#include "common.h"

namespace darb {

namespace {

constexpr int kScanThreads = 256;
constexpr int kScanItems = 8;
constexpr int kScanBlock = kScanThreads * kScanItems;  // 2048 elements per block
constexpr int kRadixThreads = 256;
constexpr int kRadixItems = 16;
constexpr int kRadixTile = kRadixThreads * kRadixItems;  // 4096 keys per block
constexpr int kChunk = 1024;                              // splats per binning chunk
constexpr uint32_t kKeyInvalid = 0x7FFFFFFFu;            // above every finite positive float's bits

struct Counters {
    uint32_t n_visible;
    uint32_t pad;
    unsigned long long k_total;
};

__device__ __forceinline__ int4 tile_rect(float u, float v, int radius, int gx, int gy) {
    float r = (float)radius;
    int x0 = (int)fminf(fmaxf(floorf((u - r) * 0.0625f), 0.0f), (float)gx);
    int x1 = (int)fminf(fmaxf(floorf((u + r) * 0.0625f) + 1.0f, 0.0f), (float)gx);
    int y0 = (int)fminf(fmaxf(floorf((v - r) * 0.0625f), 0.0f), (float)gy);
    int y1 = (int)fminf(fmaxf(floorf((v + r) * 0.0625f) + 1.0f, 0.0f), (float)gy);
    return make_int4(x0, x1, y0, y1);
}

// ---------------------------------------------------------------------------
// Generic exclusive scan of u32 (reduce -> scan block sums -> down-sweep).
// The element count may live on the device (count_dev), with `max_count`
// sizing the grid; blocks past the live count exit.
// ---------------------------------------------------------------------------

__device__ __forceinline__ uint32_t live_count(const uint32_t *count_dev, uint32_t max_count) {
    return count_dev ? min(*count_dev, max_count) : max_count;
}

__device__ __forceinline__ uint32_t block_excl_scan(uint32_t v, uint32_t *lds_w, uint32_t *total) {
    const int lane = threadIdx.x & 63, w = threadIdx.x >> 6;
    uint32_t inc = wave_incl_scan(v);
    if (lane == 63) lds_w[w] = inc;
    __syncthreads();
    uint32_t woff = 0, tot = 0;
    for (int i = 0; i < kScanThreads / 64; i++) {
        uint32_t x = lds_w[i];
        if (i < w) woff += x;
        tot += x;
    }
    __syncthreads();
    *total = tot;
    return woff + inc - v;
}

__global__ __launch_bounds__(kScanThreads) void k_scan_reduce(const uint32_t *in, const uint32_t *count_dev,
                                                              uint32_t max_count, uint32_t *parts) {
    __shared__ uint32_t lw[kScanThreads / 64];
    uint32_t count = live_count(count_dev, max_count);
    uint32_t base = blockIdx.x * kScanBlock;
    if (base >= count) return;
    uint32_t s = 0;
    for (int k = 0; k < kScanItems; k++) {
        uint32_t i = base + k * kScanThreads + threadIdx.x;
        if (i < count) s += in[i];
    }
    uint32_t tot;
    block_excl_scan(s, lw, &tot);
    if (threadIdx.x == 0) parts[blockIdx.x] = tot;
}

// single block: exclusive scan of the block sums; total -> parts[nblocks]
__global__ __launch_bounds__(1024) void k_scan_parts(uint32_t *parts, const uint32_t *count_dev, uint32_t max_count) {
    __shared__ uint32_t lw[16];
    __shared__ uint32_t carry;
    uint32_t count = live_count(count_dev, max_count);
    uint32_t nb = (count + kScanBlock - 1) / kScanBlock;
    if (threadIdx.x == 0) carry = 0;
    __syncthreads();
    const int lane = threadIdx.x & 63, w = threadIdx.x >> 6;
    for (uint32_t base = 0; base < nb; base += 1024) {
        uint32_t i = base + threadIdx.x;
        uint32_t v = i < nb ? parts[i] : 0u;
        uint32_t inc = wave_incl_scan(v);
        if (lane == 63) lw[w] = inc;
        __syncthreads();
        uint32_t woff = 0, tot = 0;
        for (int k = 0; k < 16; k++) {
            if (k < w) woff += lw[k];
            tot += lw[k];
        }
        uint32_t c = carry;
        if (i < nb) parts[i] = c + woff + inc - v;
        __syncthreads();
        if (threadIdx.x == 0) carry = c + tot;
        __syncthreads();
    }
    if (threadIdx.x == 0) parts[nb] = carry;
}

__global__ __launch_bounds__(kScanThreads) void k_scan_down(const uint32_t *in, uint32_t *out, const uint32_t *count_dev,
                                                            uint32_t max_count, const uint32_t *parts) {
    __shared__ uint32_t lw[kScanThreads / 64];
    uint32_t count = live_count(count_dev, max_count);
    uint32_t base = blockIdx.x * kScanBlock;
    if (base >= count) return;
    // blocked arrangement: thread t owns elements [base + t*kScanItems, +kScanItems)
    uint32_t v[kScanItems];
    uint32_t s = 0;
    uint32_t b0 = base + threadIdx.x * kScanItems;
    for (int k = 0; k < kScanItems; k++) {
        v[k] = (b0 + k < count) ? in[b0 + k] : 0u;
        s += v[k];
    }
    uint32_t tot;
    uint32_t off = block_excl_scan(s, lw, &tot) + parts[blockIdx.x];
    for (int k = 0; k < kScanItems; k++) {
        if (b0 + k < count) out[b0 + k] = off;
        off += v[k];
    }
}

hipError_t scan_exclusive(const uint32_t *in, uint32_t *out, const uint32_t *count_dev, uint32_t max_count,
                          uint32_t *parts, hipStream_t s) {
    if (max_count == 0) return hipSuccess;
    uint32_t nb = (max_count + kScanBlock - 1) / kScanBlock;
    hipLaunchKernelGGL(k_scan_reduce, dim3(nb), dim3(kScanThreads), 0, s, in, count_dev, max_count, parts);
    hipLaunchKernelGGL(k_scan_parts, dim3(1), dim3(1024), 0, s, parts, count_dev, max_count);
    hipLaunchKernelGGL(k_scan_down, dim3(nb), dim3(kScanThreads), 0, s, in, out, count_dev, max_count, parts);
    return hipGetLastError();
}

// ---------------------------------------------------------------------------
// Stable LSD radix sort of (u32 key, u32 value), 8-bit digits.
// ---------------------------------------------------------------------------

__global__ __launch_bounds__(kRadixThreads) void k_radix_hist(const uint32_t *keys, int n, int shift, uint32_t *hist,
                                                              int nblk) {
    __shared__ uint32_t h[256];
    h[threadIdx.x] = 0;
    __syncthreads();
    int base = blockIdx.x * kRadixTile;
    for (int k = 0; k < kRadixItems; k++) {
        int i = base + k * kRadixThreads + threadIdx.x;
        if (i < n) atomicAdd(&h[(keys[i] >> shift) & 255u], 1u);
    }
    __syncthreads();
    hist[threadIdx.x * nblk + blockIdx.x] = h[threadIdx.x];  // digit-major
}

__global__ __launch_bounds__(kRadixThreads) void k_radix_scatter(const uint32_t *kin, const uint32_t *vin,
                                                                 uint32_t *kout, uint32_t *vout, int n, int shift,
                                                                 const uint32_t *hist_scan, int nblk) {
    __shared__ uint32_t run[256];
    __shared__ uint32_t wc[kRadixThreads / 64][256];
    const int t = threadIdx.x, lane = t & 63, w = t >> 6;
    run[t] = hist_scan[t * nblk + blockIdx.x];
    for (int k = 0; k < kRadixThreads / 64; k++) wc[k][t] = 0;
    __syncthreads();
    const uint64_t lt = (lane == 0) ? 0ull : (~0ull >> (64 - lane));
    int base = blockIdx.x * kRadixTile;
    for (int r = 0; r < kRadixItems; r++) {
        int i = base + r * kRadixThreads + t;
        bool valid = i < n;
        uint32_t key = valid ? kin[i] : 0u;
        uint32_t val = valid ? vin[i] : 0u;
        uint32_t d = (key >> shift) & 255u;
        uint64_t peers = __ballot(valid);
#pragma unroll
        for (int b = 0; b < 8; b++) {
            bool bit = (d >> b) & 1u;
            uint64_t m = __ballot(bit);
            peers &= bit ? m : ~m;
        }
        uint32_t rank = __popcll(peers & lt);
        if (valid && rank == 0) wc[w][d] = (uint32_t)__popcll(peers);
        __syncthreads();
        if (valid) {
            uint32_t off = run[d] + rank;
            for (int k = 0; k < w; k++) off += wc[k][d];
            kout[off] = key;
            vout[off] = val;
        }
        __syncthreads();
        uint32_t add = 0;
        for (int k = 0; k < kRadixThreads / 64; k++) {
            add += wc[k][t];
            wc[k][t] = 0;
        }
        run[t] += add;
        __syncthreads();
    }
}

// ---------------------------------------------------------------------------
// Binning kernels.
// ---------------------------------------------------------------------------

__global__ void k_bin_init(Counters *cnt, int64_t *k_dev, int32_t *overflow_dev) {
    if (threadIdx.x == 0) {
        cnt->n_visible = 0;
        cnt->k_total = 0;
        *k_dev = 0;
        *overflow_dev = 0;
    }
}

// depth keys + per-block visible counts (summed by k_bin_sizes; no contended atomics)
__global__ __launch_bounds__(256) void k_bin_keys(const float *xy, const int32_t *radius, const float *depth, int n,
                                                  int gx, int gy, uint32_t *keys, uint32_t *vals,
                                                  uint32_t *block_vis) {
    __shared__ uint32_t wsum[4];
    int i = blockIdx.x * blockDim.x + threadIdx.x;
    bool vis = false;
    uint32_t key = kKeyInvalid;
    if (i < n) {
        int R = radius[i];
        if (R > 0) {
            float2 p = reinterpret_cast<const float2 *>(xy)[i];
            int4 r = tile_rect(p.x, p.y, R, gx, gy);
            if (r.y > r.x && r.w > r.z) {
                vis = true;
                key = __float_as_uint(depth[i]);
            }
        }
        keys[i] = key;
        vals[i] = (uint32_t)i;
    }
    uint64_t m = __ballot(vis);
    if ((threadIdx.x & 63) == 0) wsum[threadIdx.x >> 6] = (uint32_t)__popcll(m);
    __syncthreads();
    if (threadIdx.x == 0) block_vis[blockIdx.x] = wsum[0] + wsum[1] + wsum[2] + wsum[3];
}

// n_visible = sum of the block counts; chunks = ceil(n_visible / kChunk); element count of H = tiles * chunks
__global__ __launch_bounds__(1024) void k_bin_sizes(const uint32_t *block_vis, int nblocks, Counters *cnt, int ntile,
                                                    uint32_t *h_count) {
    __shared__ uint32_t part[16];
    uint32_t s = 0;
    for (int b = threadIdx.x; b < nblocks; b += 1024) s += block_vis[b];
#pragma unroll
    for (int off = 32; off >= 1; off >>= 1) s += (uint32_t)__shfl_xor((int)s, off, 64);
    if ((threadIdx.x & 63) == 0) part[threadIdx.x >> 6] = s;
    __syncthreads();
    if (threadIdx.x == 0) {
        uint32_t nv = 0;
        for (int k = 0; k < 16; k++) nv += part[k];
        cnt->n_visible = nv;
        uint32_t chunks = (nv + kChunk - 1) / kChunk;
        *h_count = chunks * (uint32_t)ntile;
    }
}

// Rectangles of the 64 splats a wave handles next (lane l holds splat base + l).
struct RectBatch {
    int x0, w, y0, area;
    uint32_t id, dbits;
};

__device__ __forceinline__ RectBatch load_rect(const uint32_t *sorted_ids, int j, int jend, const float *xy,
                                               const int32_t *radius, const float *depth, int gx, int gy) {
    RectBatch b;
    b.x0 = b.w = b.y0 = b.area = 0;
    b.id = 0;
    b.dbits = 0;
    if (j < jend) {
        uint32_t id = sorted_ids[j];
        float2 p = reinterpret_cast<const float2 *>(xy)[id];
        int4 r = tile_rect(p.x, p.y, radius[id], gx, gy);
        b.x0 = r.x;
        b.w = r.y - r.x;
        b.y0 = r.z;
        b.area = b.w * (r.w - r.z);
        b.id = id;
        b.dbits = __float_as_uint(depth[id]);
    }
    return b;
}

__global__ __launch_bounds__(64) void k_bin_count(const uint32_t *sorted_ids, const float *xy, const int32_t *radius,
                                                  const float *depth, int gx, int gy, const Counters *cnt,
                                                  uint32_t *H, Counters *cnt_w) {
    extern __shared__ uint32_t hist[];
    const int ntile = gx * gy;
    const uint32_t nv = cnt->n_visible;
    const uint32_t chunks = (nv + kChunk - 1) / kChunk;
    const uint32_t c = blockIdx.x;
    if (c >= chunks) return;
    const int lane = threadIdx.x;
    for (int t = lane; t < ntile; t += 64) hist[t] = 0;
    __syncthreads();
    int jbeg = c * kChunk, jend = min((int)nv, jbeg + kChunk);
    uint32_t total = 0;
    for (int jb = jbeg; jb < jend; jb += 64) {
        RectBatch rb = load_rect(sorted_ids, jb + lane, jend, xy, radius, depth, gx, gy);
        int nb = min(64, jend - jb);
        for (int s = 0; s < nb; s++) {
            int x0 = readlane_i(rb.x0, s), w = readlane_i(rb.w, s), y0 = readlane_i(rb.y0, s);
            int area = readlane_i(rb.area, s);
            float rw = 1.0f / (float)w;
            total += area;
            for (int e = lane; e < area; e += 64) {
                int q = (int)(((float)e + 0.5f) * rw);
                int tx = x0 + (e - q * w), ty = y0 + q;
                atomicAdd(&hist[ty * gx + tx], 1u);
            }
        }
    }
    __syncthreads();
    for (int t = lane; t < ntile; t += 64) H[(size_t)t * chunks + c] = hist[t];
    if (lane == 0) atomicAdd(&cnt_w->k_total, (unsigned long long)total);
}

__global__ __launch_bounds__(256) void k_bin_ranges(const uint32_t *Hs, const uint32_t *h_parts_total, int ntile,
                                                    const Counters *cnt, uint32_t *ranges, int64_t k_capacity,
                                                    int64_t *k_dev, int32_t *overflow_dev) {
    int t = blockIdx.x * blockDim.x + threadIdx.x;
    uint32_t chunks = (cnt->n_visible + kChunk - 1) / kChunk;
    unsigned long long K = cnt->k_total;
    if (t < ntile) {
        uint32_t b = chunks ? Hs[(size_t)t * chunks] : 0u;
        uint32_t e = (t + 1 < ntile) ? (chunks ? Hs[(size_t)(t + 1) * chunks] : 0u) : (uint32_t)K;
        ranges[2 * t] = b;
        ranges[2 * t + 1] = e;
    }
    if (t == 0) {
        *k_dev = (int64_t)K;
        *overflow_dev = (K > (unsigned long long)k_capacity || K >= 0xFFFFFFFFull) ? 1 : 0;
    }
}

__global__ __launch_bounds__(64) void k_bin_scatter(const uint32_t *sorted_ids, const float *xy, const int32_t *radius,
                                                    const float *depth, int gx, int gy, const Counters *cnt,
                                                    const uint32_t *Hs, const int32_t *overflow_dev, int64_t k_capacity,
                                                    uint64_t *keys, uint32_t *vals) {
    extern __shared__ uint32_t slot[];
    if (*overflow_dev) return;
    const int ntile = gx * gy;
    const uint32_t nv = cnt->n_visible;
    const uint32_t chunks = (nv + kChunk - 1) / kChunk;
    const uint32_t c = blockIdx.x;
    if (c >= chunks) return;
    const int lane = threadIdx.x;
    for (int t = lane; t < ntile; t += 64) slot[t] = Hs[(size_t)t * chunks + c];
    __syncthreads();
    int jbeg = c * kChunk, jend = min((int)nv, jbeg + kChunk);
    for (int jb = jbeg; jb < jend; jb += 64) {
        RectBatch rb = load_rect(sorted_ids, jb + lane, jend, xy, radius, depth, gx, gy);
        int nb = min(64, jend - jb);
        for (int s = 0; s < nb; s++) {
            int x0 = readlane_i(rb.x0, s), w = readlane_i(rb.w, s), y0 = readlane_i(rb.y0, s);
            int area = readlane_i(rb.area, s);
            uint32_t id = (uint32_t)readlane_i((int)rb.id, s);
            uint32_t db = (uint32_t)readlane_i((int)rb.dbits, s);
            float rw = 1.0f / (float)w;
            for (int e = lane; e < area; e += 64) {
                int q = (int)(((float)e + 0.5f) * rw);
                int tx = x0 + (e - q * w), ty = y0 + q;
                int t = ty * gx + tx;
                uint32_t pos = atomicAdd(&slot[t], 1u);
                if ((int64_t)pos < k_capacity) {  // always true when the flag is clear; guards the buffer
                    vals[pos] = id;
                    if (keys) keys[pos] = ((uint64_t)(uint32_t)t << 32) | db;
                }
            }
        }
    }
}

inline size_t align_up(size_t x) { return (x + 255) & ~(size_t)255; }

struct WsLayout {
    size_t counters, keysA, valsA, keysB, valsB, hist, parts, H, hcount, blockvis, total;
};

WsLayout layout(int n, int ntile) {
    WsLayout L;
    size_t off = 0;
    int nblk = (n + kRadixTile - 1) / kRadixTile;
    size_t chunks = ((size_t)n + kChunk - 1) / kChunk;
    size_t hist_n = (size_t)256 * nblk;
    size_t H_n = chunks * (size_t)ntile;
    size_t parts_n = (std::max(hist_n, H_n) + kScanBlock - 1) / kScanBlock + 1;
    L.counters = off; off += align_up(sizeof(Counters));
    L.keysA = off; off += align_up((size_t)n * 4);
    L.valsA = off; off += align_up((size_t)n * 4);
    L.keysB = off; off += align_up((size_t)n * 4);
    L.valsB = off; off += align_up((size_t)n * 4);
    L.hist = off; off += align_up(hist_n * 4);
    L.parts = off; off += align_up(parts_n * 4);
    L.H = off; off += align_up(H_n * 4);
    L.hcount = off; off += align_up(4);
    L.blockvis = off; off += align_up(((size_t)n + 255) / 256 * 4);
    L.total = off;
    return L;
}

}  // namespace

size_t binsort_workspace(int n, int width, int height) {
    int gx = (width + kTile - 1) / kTile, gy = (height + kTile - 1) / kTile;
    return layout(n, gx * gy).total;
}

hipError_t launch_bin_sort(const darb_projected &p, int n, int width, int height, int64_t k_capacity, void *ws,
                           uint64_t *keys, uint32_t *vals, uint32_t *ranges, int64_t *k_dev, int32_t *overflow_dev,
                           hipStream_t s) {
    const int gx = (width + kTile - 1) / kTile, gy = (height + kTile - 1) / kTile, ntile = gx * gy;
    WsLayout L = layout(n, ntile);
    char *base = static_cast<char *>(ws);
    Counters *cnt = reinterpret_cast<Counters *>(base + L.counters);
    uint32_t *kA = reinterpret_cast<uint32_t *>(base + L.keysA);
    uint32_t *vA = reinterpret_cast<uint32_t *>(base + L.valsA);
    uint32_t *kB = reinterpret_cast<uint32_t *>(base + L.keysB);
    uint32_t *vB = reinterpret_cast<uint32_t *>(base + L.valsB);
    uint32_t *hist = reinterpret_cast<uint32_t *>(base + L.hist);
    uint32_t *parts = reinterpret_cast<uint32_t *>(base + L.parts);
    uint32_t *H = reinterpret_cast<uint32_t *>(base + L.H);
    uint32_t *hcount = reinterpret_cast<uint32_t *>(base + L.hcount);
    uint32_t *blockvis = reinterpret_cast<uint32_t *>(base + L.blockvis);

    hipLaunchKernelGGL(k_bin_init, dim3(1), dim3(64), 0, s, cnt, k_dev, overflow_dev);
    if (n > 0) {
        int nkb = (n + 255) / 256;
        hipLaunchKernelGGL(k_bin_keys, dim3(nkb), dim3(256), 0, s, p.xy, p.radius, p.depth, n, gx, gy, kA, vA, blockvis);
        hipLaunchKernelGGL(k_bin_sizes, dim3(1), dim3(1024), 0, s, blockvis, nkb, cnt, ntile, hcount);
        // depth sort: 4 passes of 8 bits (keys fit in 31 bits)
        int nblk = (n + kRadixTile - 1) / kRadixTile;
        uint32_t *ki = kA, *vi = vA, *ko = kB, *vo = vB;
        for (int shift = 0; shift < 32; shift += 8) {
            hipLaunchKernelGGL(k_radix_hist, dim3(nblk), dim3(kRadixThreads), 0, s, ki, n, shift, hist, nblk);
            hipError_t e = scan_exclusive(hist, hist, nullptr, (uint32_t)(256 * nblk), parts, s);
            if (e != hipSuccess) return e;
            hipLaunchKernelGGL(k_radix_scatter, dim3(nblk), dim3(kRadixThreads), 0, s, ki, vi, ko, vo, n, shift, hist,
                               nblk);
            std::swap(ki, ko);
            std::swap(vi, vo);
        }
        // after an even number of passes the sorted ids are in vi (== vA)
        const uint32_t *sorted = vi;
        int maxchunks = (n + kChunk - 1) / kChunk;
        size_t lds = (size_t)ntile * 4;
        hipLaunchKernelGGL(k_bin_count, dim3(maxchunks), dim3(64), lds, s, sorted, p.xy, p.radius, p.depth, gx, gy,
                           cnt, H, cnt);
        hipError_t e = scan_exclusive(H, H, hcount, (uint32_t)((size_t)maxchunks * ntile), parts, s);
        if (e != hipSuccess) return e;
        hipLaunchKernelGGL(k_bin_ranges, dim3((ntile + 255) / 256), dim3(256), 0, s, H, parts, ntile, cnt, ranges,
                           k_capacity, k_dev, overflow_dev);
        hipLaunchKernelGGL(k_bin_scatter, dim3(maxchunks), dim3(64), lds, s, sorted, p.xy, p.radius, p.depth, gx, gy,
                           cnt, H, overflow_dev, k_capacity, keys, vals);
    } else {
        hipLaunchKernelGGL(k_bin_ranges, dim3((ntile + 255) / 256), dim3(256), 0, s, H, parts, ntile, cnt, ranges,
                           k_capacity, k_dev, overflow_dev);
    }
    return hipGetLastError();
}

}  // namespace darb
