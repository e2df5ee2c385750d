// raster.hip -- per-tile DARBF compositing, forward and backward.
//
// One workgroup per 16x16 tile, split into S wavefronts of 16 x (16/S) pixels
// each; lane l of wave h owns column l % 16 in rows h*16/S + l/16 + 4k,
// k < 4/S.  The forward uses S = 2: a tile's walk is short (its pixels
// saturate after a few hundred instances) and serial, so two independent
// half-tile walks shorten the longest path through the kernel and fill more
// wave slots.  The backward keeps S = 1: its per-instance wave reductions and
// atomics would double with S = 2, which costs more than the shorter walks
// gain.  The instance
// list is consumed in batches of 64: lane l gathers the projected record of
// the batch's l-th instance, then the wave walks the batch with the record of
// instance s broadcast to scalar registers (v_readlane), so every pixel test
// reads its splat operands from SGPRs.  A ballot over the lanes' "done" bits
// ends the walk early once every pixel of the wave has saturated.
//
// Forward (DARB-Splatting section, alpha blending; per-kernel forward
// listings): E = d^T Q d with d = mu' - p, alpha = min(alpha_max, o F(E)),
// skip if E outside [0, e_max] or alpha < alpha_min, stop if T(1 - alpha) <
// t_min.  Writes the image and the checkpoint (final T, last position).
//
// Backward (per-kernel backward listings): walks each tile's list from the
// largest checkpointed position down, recomputing alpha with the same device
// function, T <- T / (1 - alpha), and accumulating the per-splat partial
// gradients of its four pixels in registers; per splat the wave sums the nine
// partials (lane-half swaps pack them four to a register, then DPP row
// reductions finish three registers) and lane s of the batch keeps the sums of
// the batch's s-th instance.  At the end of a batch the lanes either issue
// their float atomics together (nine atomic instructions per 64 instances), or,
// in the deterministic mode, store them as one partial per (tile, splat); a
// stable sort by splat and a per-splat sum in tile order finish the reduction.
//
// Several views run in one launch over the concatenated tiles of all views
// (work item -> view by the views' first items); the fused kernel composites a
// tile, takes the per-pixel loss gradient in registers and runs the backward
// walk of the same tile at once.
#include <algorithm>

#include "common.h"

namespace darb {

namespace {

constexpr int kPix = 4;    // pixels per lane with one wavefront per tile
// Row coordinate given to the forward's pixels that are outside the image or
// have saturated: there E >= (l11 dy)^2 > 1e22 exceeds any e_max (l11 =
// 1/sqrt(c11) > 5e-20 for every finite conic), or overflows to +inf, so no
// splat passes their test and the walk needs no separate per-pixel state.
constexpr float kFar = 3.0e30f;
constexpr int kSplit = 2;  // wavefronts per tile in the forward kernel
// The forward also tests for saturation inside a batch, after every this many
// footprints that meet the wave's pixels (0: once per batch of 64 instances).
#ifndef DARB_FWD_SAT_CHECK
#define DARB_FWD_SAT_CHECK 4
#endif
constexpr int kFwdSatCheck = DARB_FWD_SAT_CHECK;

// Pixels of this lane: column ix, rows iy0 + 4k for k < kPix / S.
template <int S>
struct LanePix {
    static constexpr int NP = kPix / S;
    int ix, iy0;
    float ylo;  // first row of this wave's pixel block
    // part h of the tile (h = the wavefront's index in its workgroup by default)
    __device__ __forceinline__ LanePix(int tile, int gx, int h = (int)(threadIdx.x >> 6)) {
        const int tx = tile % gx, ty = tile / gx;
        const int lane = threadIdx.x & 63;
        ix = tx * kTile + (lane & 15);
        ylo = (float)(ty * kTile + h * (kTile / S));
        iy0 = ty * kTile + h * (kTile / S) + (lane >> 4);
    }
};

struct Rec {
    float x, y, a, b, c, o, r, g, bl;  // a, b, c: the conic factor (l00, l01, l11)
    uint32_t id;
    int hit;  // the footprint's bounding box meets this tile's pixels
};

// Record of instance j (zeros when `in` is false or the stored index is out of
// range; a zero-opacity record never passes the alpha test).  `hit` is false
// when the ellipse E <= e_max, grown by one pixel, misses the wave's pixel
// block (columns xlo .. xlo + 15, rows ylo .. ylo + yext): for |dx| > sqrt(e_max Sigma'_xx) every E exceeds e_max by a relative
// margin far above FP32 rounding, so skipping such a splat changes nothing.
// With Q = L^T L: Sigma' = Q^-1 has Sigma'_xx = (1 + (l01/l11)^2) / l00^2 and
// Sigma'_yy = 1 / l11^2.
__device__ __forceinline__ Rec load_rec(const darb_projected &p, const uint32_t *vals, uint32_t j, bool in, int n,
                                        float e_max, float xlo, float ylo, float yext) {
    Rec R;
    R.x = R.y = R.a = R.b = R.c = R.o = R.r = R.g = R.bl = 0.0f;
    R.id = kNone;
    R.hit = 0;
    uint32_t id = in ? vals[j] : kNone;
    if (id < (uint32_t)n) {
        float2 xy = reinterpret_cast<const float2 *>(p.xy)[id];
        float4 co = reinterpret_cast<const float4 *>(p.conic_o)[id];
        R.x = xy.x;
        R.y = xy.y;
        R.a = co.x;
        R.b = co.y;
        R.c = co.z;
        R.o = co.w;
        R.r = p.rgb[3 * id];
        R.g = p.rgb[3 * id + 1];
        R.bl = p.rgb[3 * id + 2];
        R.id = id;
        // half-extents of {E <= e_max}: sqrt(e_max * Sigma'_xx), sqrt(e_max * Sigma'_yy)
        const float r01 = co.y / co.z;
        float hx = sqrtf(e_max * fmaf(r01, r01, 1.0f)) / co.x + 1.0f;
        float hy = sqrtf(e_max) / co.z + 1.0f;
        bool ok = (co.x > 0.0f && co.z > 0.0f)
                      ? ((xy.x + hx >= xlo) & (xy.x - hx <= xlo + (kTile - 1)) & (xy.y + hy >= ylo) &
                         (xy.y - hy <= ylo + yext))
                      : true;
        R.hit = ok ? 1 : 0;
    }
    return R;
}

// A launch over one view (small kernel arguments) or over several.
struct OneView {
    RView v;
    __device__ __forceinline__ const RView &get(uint32_t item, int &tile) const {
        tile = (int)item;
        return v;
    }
    __device__ __forceinline__ darb_grads2d grads(uint32_t) const { return v.g2; }
};

struct ManyViews {
    RViews a;
    __device__ __forceinline__ const RView &get(uint32_t item, int &tile) const {
        int vi = 0;
        for (int k = 1; k < a.nv; k++) vi = (item >= a.v[k].item0) ? k : vi;
        tile = (int)(item - a.v[vi].item0);
        return a.v[vi];
    }
    // per-lane view index: select among the views (uniform loads only)
    __device__ __forceinline__ darb_grads2d grads(uint32_t vi) const {
        darb_grads2d g = a.v[0].g2;
        for (int k = 1; k < a.nv; k++)
            if ((uint32_t)k == vi) g = a.v[k].g2;
        return g;
    }
};

// Forward state of a lane's pixels.
template <int NP>
struct PixF {
    float T[NP], C0[NP], C1[NP], C2[NP];
    uint32_t lst[NP], cnt[NP];
};

// CNT: count the blended splats of each pixel (only when they are stored).
template <int KIND, int S, bool CNT>
__device__ __forceinline__ void tile_fwd(const RView &V, int tile, int n, const KParams &kp, const ROpts &o,
                                         PixF<kPix / S> &Fout) {
    constexpr int NP = kPix / S;
    PixF<NP> F;  // local state, copied out at the end (keeps the loop at 64 VGPRs)
    const LanePix<S> P(tile, V.gx);
    const int lane = threadIdx.x & 63;
    const int ix = P.ix, iy0 = P.iy0;
    const float px = (float)ix;
    float py[NP];
#pragma unroll
    for (int k = 0; k < NP; k++) {
        int iy = iy0 + 4 * k;
        py[k] = (ix < V.W && iy < V.H) ? (float)iy : kFar;
        F.T[k] = 1.0f;
        F.C0[k] = F.C1[k] = F.C2[k] = 0.0f;
        F.lst[k] = kNone;
        F.cnt[k] = 0;
    }
    const uint32_t start = V.ranges[2 * tile], end = V.ranges[2 * tile + 1];
    for (uint32_t base = start; base < end; base += 64) {
        bool alldone = true;
#pragma unroll
        for (int k = 0; k < NP; k++) alldone &= py[k] == kFar;
        if (__ballot(!alldone) == 0) break;
        uint32_t j = base + lane;
        Rec R = load_rec(V.p, V.vals, j, j < end, n, kp.e_max, (float)(ix - (lane & 15)), P.ylo,
                         (float)(kTile / S - 1));
        int since = 0;  // hit instances since the last saturation check (uniform)
        bool fin = false;
        // the batch's footprints that meet this wave's pixels, in list order: the
        // set bits of one ballot (the walk skips the others without a test each)
        for (uint64_t hm = __ballot(R.hit != 0); hm != 0; hm &= hm - 1) {
            const int s = (int)__builtin_ctzll(hm);
            float sx = readlane_f(R.x, s), sy = readlane_f(R.y, s);
            float sa = readlane_f(R.a, s), sb = readlane_f(R.b, s), sc = readlane_f(R.c, s);
            float so = readlane_f(R.o, s);
            float sr = readlane_f(R.r, s), sg = readlane_f(R.g, s), sbl = readlane_f(R.bl, s);
            uint32_t pos = base + s;
#pragma unroll
            for (int k = 0; k < NP; k++) {
                Pair q = eval_pair<KIND>(sx, sy, sa, sb, sc, so, px, py[k], kp, o.alpha_min, o.alpha_max);
                bool ok = q.ok;
                float Tn = F.T[k] * (1.0f - q.alpha);
                bool stop = ok & (Tn < o.t_min);
                ok = ok & !stop;
                py[k] = stop ? kFar : py[k];
                float aT = ok ? q.alpha * F.T[k] : 0.0f;
                F.C0[k] = fmaf(aT, sr, F.C0[k]);
                F.C1[k] = fmaf(aT, sg, F.C1[k]);
                F.C2[k] = fmaf(aT, sbl, F.C2[k]);
                F.T[k] = ok ? Tn : F.T[k];
                F.lst[k] = ok ? pos : F.lst[k];
                if constexpr (CNT) F.cnt[k] += ok ? 1u : 0u;
            }
            // every kFwdSatCheck footprints, leave once all the wave's pixels
            // saturated (no later instance changes them)
            if constexpr (kFwdSatCheck > 0) {
                if (++since == kFwdSatCheck) {
                    since = 0;
                    bool ad = true;
#pragma unroll
                    for (int k = 0; k < NP; k++) ad &= py[k] == kFar;
                    if (__ballot(!ad) == 0) {
                        fin = true;
                        break;
                    }
                }
            }
        }
        if (fin) break;
    }
    Fout = F;
}

template <int S>
__device__ __forceinline__ void store_fwd(const RView &V, int tile, const PixF<kPix / S> &F, const ROpts &o) {
    const LanePix<S> P(tile, V.gx);
    const int ix = P.ix, iy0 = P.iy0;
    const size_t plane = (size_t)V.W * V.H;
#pragma unroll
    for (int k = 0; k < kPix / S; k++) {
        int iy = iy0 + 4 * k;
        if (ix < V.W && iy < V.H) {
            size_t pidx = (size_t)iy * V.W + ix;
            V.image[pidx] = fmaf(F.T[k], o.bg0, F.C0[k]);
            V.image[plane + pidx] = fmaf(F.T[k], o.bg1, F.C1[k]);
            V.image[2 * plane + pidx] = fmaf(F.T[k], o.bg2, F.C2[k]);
            if (V.final_T) V.final_T[pidx] = F.T[k];
            if (V.last) V.last[pidx] = F.lst[k];
            if (V.n_contrib) V.n_contrib[pidx] = F.cnt[k];
        }
    }
}

// Storage of the deterministic mode: partial c of 9 planes (stride cap), its
// key (view * n + splat) and its own index; trav_off[item] = first partial of
// the work item.
struct DetOut {
    float *parts;
    uint32_t *ekey, *eval;
    const uint32_t *trav_off;
    uint32_t cap;
};

// End (last position + 1) of the tile's walk: the largest checkpointed
// position of its pixels, clamped to the tile's range.
__device__ __forceinline__ uint32_t wave_max_u32(uint32_t v) {
#pragma unroll
    for (int off = 32; off >= 1; off >>= 1) v = max(v, (uint32_t)__shfl_xor((int)v, off, 64));
    return v;
}

// Writes nine wave-uniform values into lane `lane` of nine per-lane
// accumulators (v_writelane_b32, independent of EXEC).  Written as one asm block
// so that the reductions producing the values stay in wave-uniform code: a
// select on (lane == s) may be turned into a one-lane branch, and cross-lane
// operations sunk into it would see a single active lane.
__device__ __forceinline__ void writelane9(float (&m)[9], const float (&u)[9], int lane) {
    // the lane select goes through M0: one VALU instruction reads one SGPR
    asm volatile(
        "s_mov_b32 m0, %18\n\t"
        "s_nop 4\n\t"
        "v_writelane_b32 %0, %9, m0\n\t"
        "v_writelane_b32 %1, %10, m0\n\t"
        "v_writelane_b32 %2, %11, m0\n\t"
        "v_writelane_b32 %3, %12, m0\n\t"
        "v_writelane_b32 %4, %13, m0\n\t"
        "v_writelane_b32 %5, %14, m0\n\t"
        "v_writelane_b32 %6, %15, m0\n\t"
        "v_writelane_b32 %7, %16, m0\n\t"
        "v_writelane_b32 %8, %17, m0"
        : "+v"(m[0]), "+v"(m[1]), "+v"(m[2]), "+v"(m[3]), "+v"(m[4]), "+v"(m[5]), "+v"(m[6]), "+v"(m[7]),
          "+v"(m[8])
        : "s"(u[0]), "s"(u[1]), "s"(u[2]), "s"(u[3]), "s"(u[4]), "s"(u[5]), "s"(u[6]), "s"(u[7]), "s"(u[8]),
          "s"(lane)
        : "m0");
}

// Sum of a and b over lanes l and l ^ 32: lanes 0-31 receive a's, lanes 32-63
// b's (v_permlane32_swap exchanges a's upper half with b's lower half).
__device__ __forceinline__ float fold32(float a, float b) {
    const auto r = __builtin_amdgcn_permlane32_swap(__float_as_uint(a), __float_as_uint(b), false, false);
    return __uint_as_float(r[0]) + __uint_as_float(r[1]);
}

// Sum over lanes l and l ^ 16: rows 0 and 2 (lanes 0-15, 32-47) receive a's,
// rows 1 and 3 b's (v_permlane16_swap exchanges a's odd rows with b's even rows).
__device__ __forceinline__ float fold16(float a, float b) {
    const auto r = __builtin_amdgcn_permlane16_swap(__float_as_uint(a), __float_as_uint(b), false, false);
    return __uint_as_float(r[0]) + __uint_as_float(r[1]);
}

// Sum within each row of 16 lanes; the row total lands in the row's lane 15.
__device__ __forceinline__ float row_sum_to_lane15(float v) {
    v += __int_as_float(__builtin_amdgcn_update_dpp(0, __float_as_int(v), 0x111, 0xf, 0xf, false));  // row_shr:1
    v += __int_as_float(__builtin_amdgcn_update_dpp(0, __float_as_int(v), 0x112, 0xf, 0xf, false));  // row_shr:2
    v += __int_as_float(__builtin_amdgcn_update_dpp(0, __float_as_int(v), 0x114, 0xf, 0xf, false));  // row_shr:4
    v += __int_as_float(__builtin_amdgcn_update_dpp(0, __float_as_int(v), 0x118, 0xf, 0xf, false));  // row_shr:8
    return v;
}

// Wave sums of nine per-lane values, written into lane s of m[k].  Two
// half-swap levels pack the nine values four to a register (one value per
// row of 16 lanes, already summed over the four lanes l, l^16, l^32, l^48), so
// three row reductions finish all nine: 8 swaps and 12 DPP adds instead of
// nine separate 64-lane reductions.
__device__ __forceinline__ void wave_sum9_to_lane(float (&m)[9], const float (&g)[9], int s) {
    // rows of w0: g0, g2, g1, g3; of w1: g4, g6, g5, g7; row 0 of w2: g8
    const float w0 = row_sum_to_lane15(fold16(fold32(g[0], g[1]), fold32(g[2], g[3])));
    const float w1 = row_sum_to_lane15(fold16(fold32(g[4], g[5]), fold32(g[6], g[7])));
    const float w2 = row_sum_to_lane15(fold16(fold32(g[8], 0.0f), 0.0f));
    const float u[9] = {readlane_f(w0, 15), readlane_f(w0, 47), readlane_f(w0, 31), readlane_f(w0, 63),
                        readlane_f(w1, 15), readlane_f(w1, 47), readlane_f(w1, 31), readlane_f(w1, 63),
                        readlane_f(w2, 15)};
    writelane9(m, u, s);
}

// Backward walk of one tile.  T: final transmittance per pixel (running, so
// modified); lp: last blended position + 1 (0 = none); G: dL/dI per pixel.
template <int KIND, bool DET, int S>
__device__ __forceinline__ void tile_bwd(const RView &V, int tile, uint32_t item, int n, const KParams &kp,
                                         const ROpts &o, float (&T)[kPix / S], const uint32_t (&lp)[kPix / S],
                                         const float (&G0)[kPix / S], const float (&G1)[kPix / S],
                                         const float (&G2)[kPix / S], const DetOut &d, int h = 0) {
    static_assert(!DET || S == 1, "the deterministic backward keeps one wavefront per tile");
    constexpr int NP = kPix / S;
    const LanePix<S> P(tile, V.gx, h);
    const int lane = threadIdx.x & 63;
    const int ix = P.ix, iy0 = P.iy0;
    const float px = (float)ix;
    float py[NP], S0[NP], S1[NP], S2[NP];
    uint32_t maxl = 0;
#pragma unroll
    for (int k = 0; k < NP; k++) {
        py[k] = (float)(iy0 + 4 * k);
        S0[k] = T[k] * o.bg0;
        S1[k] = T[k] * o.bg1;
        S2[k] = T[k] * o.bg2;
        maxl = max(maxl, lp[k]);
    }
    maxl = wave_max_u32(maxl);
    const uint32_t start = V.ranges[2 * tile], end = V.ranges[2 * tile + 1];
    maxl = min(maxl, end);  // a checkpoint always points inside its tile's range
    if (maxl == 0 || maxl <= start) return;
    uint32_t c0 = 0;
    if constexpr (DET) c0 = d.trav_off[item];
    // walk positions maxl-1 down to start in batches of 64
    for (uint32_t hi = maxl; hi > start;) {
        uint32_t cntb = min(64u, hi - start);
        uint32_t j = hi - 1 - lane;
        Rec R = load_rec(V.p, V.vals, j, (uint32_t)lane < cntb, n, kp.e_max, (float)(ix - (lane & 15)), P.ylo,
                         (float)(kTile / S - 1));
        // lane s keeps the reduced partials of the batch's s-th instance
        float m[9] = {0.f, 0.f, 0.f, 0.f, 0.f, 0.f, 0.f, 0.f, 0.f};
        uint64_t touched = 0;  // lanes whose instance received a contribution (uniform)
        // the batch's footprints that meet this wave's pixels, in walk order
        for (uint64_t hm = __ballot(R.hit != 0); hm != 0; hm &= hm - 1) {
            const int s = (int)__builtin_ctzll(hm);
            float sx = readlane_f(R.x, s), sy = readlane_f(R.y, s);
            float sa = readlane_f(R.a, s), sb = readlane_f(R.b, s), sc = readlane_f(R.c, s);
            float so = readlane_f(R.o, s);
            float sr = readlane_f(R.r, s), sg = readlane_f(R.g, s), sbl = readlane_f(R.bl, s);
            uint32_t pos1 = hi - (uint32_t)s;  // position + 1
            float gxy0 = 0.f, gxy1 = 0.f, gca = 0.f, gcb = 0.f, gcc = 0.f, gop = 0.f, gr = 0.f, gg = 0.f, gbl = 0.f;
            bool any = false;
#pragma unroll
            for (int k = 0; k < NP; k++) {
                Pair q = eval_pair<KIND>(sx, sy, sa, sb, sc, so, px, py[k], kp, o.alpha_min, o.alpha_max);
                bool ok = q.ok & (pos1 <= lp[k]);
                any |= ok;
                float inv = __builtin_amdgcn_rcpf(1.0f - q.alpha);
                float Tb = T[k] * inv;
                float da = G0[k] * fmaf(sr, Tb, -S0[k] * inv);
                da = fmaf(G1[k], fmaf(sg, Tb, -S1[k] * inv), da);
                da = fmaf(G2[k], fmaf(sbl, Tb, -S2[k] * inv), da);
                // the pair's factors, zero where it does not blend (selected, never
                // multiplied by a mask: outside the support F(E) may be inf)
                const float aTm = ok ? q.alpha * Tb : 0.0f;
                const float wm = ok ? q.w : 0.0f;
                const float dEm = ok ? so * profile_deriv<KIND>(q.E, q.w, kp) * da : 0.0f;
                gr = fmaf(aTm, G0[k], gr);
                gg = fmaf(aTm, G1[k], gg);
                gbl = fmaf(aTm, G2[k], gbl);
                gop = fmaf(wm, da, gop);
                // dE/dmu' = 2 Q d and the off-diagonal conic term carry a factor 2,
                // applied once to the reduced sums (exact)
                gxy0 = fmaf(dEm, q.q0, gxy0);
                gxy1 = fmaf(dEm, q.q1, gxy1);
                const float ex = dEm * q.dx, ey = dEm * q.dy;
                gca = fmaf(ex, q.dx, gca);
                gcb = fmaf(ex, q.dy, gcb);
                gcc = fmaf(ey, q.dy, gcc);
                S0[k] = fmaf(aTm, sr, S0[k]);  // unchanged where aTm = 0
                S1[k] = fmaf(aTm, sg, S1[k]);
                S2[k] = fmaf(aTm, sbl, S2[k]);
                T[k] = ok ? Tb : T[k];
            }
            if (__ballot(any) != 0) {
                const float g[9] = {gxy0, gxy1, gca, gcb, gcc, gop, gr, gg, gbl};
                wave_sum9_to_lane(m, g, s);
                touched |= 1ull << s;
            }
        }
        // the factor 2 of the mean and off-diagonal conic terms
        m[0] *= 2.0f;
        m[1] *= 2.0f;
        m[3] *= 2.0f;
        if constexpr (DET) {
            if ((uint32_t)lane < cntb) {
                const uint32_t c = c0 + (j - start);
                const size_t C = d.cap;
#pragma unroll
                for (int k = 0; k < 9; k++) d.parts[k * C + c] = m[k];
                d.ekey[c] = R.id < (uint32_t)n ? V.key0 + R.id : kNone;
                d.eval[c] = c;
            }
        } else {
            const uint32_t id = R.id;
            if (((touched >> lane) & 1ull) && id < (uint32_t)n) {
                atomicAdd(&V.g2.xy[2 * id], m[0]);
                atomicAdd(&V.g2.xy[2 * id + 1], m[1]);
                atomicAdd(&V.g2.conic[3 * id], m[2]);
                atomicAdd(&V.g2.conic[3 * id + 1], m[3]);
                atomicAdd(&V.g2.conic[3 * id + 2], m[4]);
                atomicAdd(&V.g2.opacity[id], m[5]);
                atomicAdd(&V.g2.rgb[3 * id], m[6]);
                atomicAdd(&V.g2.rgb[3 * id + 1], m[7]);
                atomicAdd(&V.g2.rgb[3 * id + 2], m[8]);
            }
        }
        hi -= cntb;
    }
}

// Checkpoint of a lane's four pixels: final T, last + 1, dL/dI.
template <int S>
__device__ __forceinline__ void load_checkpoint(const RView &V, int tile, float (&T)[kPix / S],
                                                uint32_t (&lp)[kPix / S], float (&G0)[kPix / S],
                                                float (&G1)[kPix / S], float (&G2)[kPix / S]) {
    const LanePix<S> P(tile, V.gx);
    const int ix = P.ix, iy0 = P.iy0;
    const size_t plane = (size_t)V.W * V.H;
#pragma unroll
    for (int k = 0; k < kPix / S; k++) {
        int iy = iy0 + 4 * k;
        lp[k] = 0;
        T[k] = 0.0f;
        G0[k] = G1[k] = G2[k] = 0.0f;
        if (ix < V.W && iy < V.H) {
            size_t pidx = (size_t)iy * V.W + ix;
            uint32_t l = V.last[pidx];
            if (l != kNone) {
                lp[k] = l + 1;
                T[k] = V.final_T[pidx];
                G0[k] = V.dL[pidx];
                G1[k] = V.dL[plane + pidx];
                G2[k] = V.dL[2 * plane + pidx];
            }
        }
    }
}

// Workgroup `part` of `nparts` clears its share of the four 2D-gradient arrays
// of n splats (2n, 3n, n, 3n floats, taken as one run of 9n), in runs of
// consecutive lanes.
__device__ __forceinline__ void zero_grads_part(const darb_grads2d &g, size_t n, uint32_t part, uint32_t nparts) {
    const size_t total = 9 * n;
    const size_t per = ((total + nparts - 1) / nparts + 63) & ~(size_t)63;
    const size_t lo = (size_t)part * per, hi = min(total, lo + per);
    float *const arr[4] = {g.xy, g.conic, g.opacity, g.rgb};
    const size_t beg[5] = {0, 2 * n, 5 * n, 6 * n, 9 * n};
#pragma unroll
    for (int a = 0; a < 4; a++) {
        const size_t s = max(lo, beg[a]), e = min(hi, beg[a + 1]);
        for (size_t k = s + threadIdx.x; k < e; k += blockDim.x) arr[a][k - beg[a]] = 0.0f;
    }
}

// With V.zero_n > 0 each workgroup also clears its share of the 2D gradients
// (single view): the stores go out after the tile's own work, when the wave
// has no load left to wait for, and fill the memory pipe that the compositing
// leaves idle.  They are issued on the overflow path as well.
template <int KIND, class VS, bool CNT>
__global__ __launch_bounds__(64 * kSplit) void k_raster_fwd(VS A, int n, KParams kp, ROpts o) {
    int tile;
    const RView &V = A.get(blockIdx.x, tile);
    if (!(V.overflow && *V.overflow)) {
        PixF<kPix / kSplit> F;
        tile_fwd<KIND, kSplit, CNT>(V, tile, n, kp, o, F);
        store_fwd<kSplit>(V, tile, F, o);
    }
    if (V.zero_n > 0) zero_grads_part(V.g2, (size_t)V.zero_n, blockIdx.x, gridDim.x);
}

template <int KIND, bool DET, class VS>
__global__ __launch_bounds__(64) void k_raster_bwd(VS A, int n, KParams kp, ROpts o, DetOut d) {
    constexpr int S = 1;
    int tile;
    const RView &V = A.get(blockIdx.x, tile);
    if (V.overflow && *V.overflow) return;
    float T[kPix / S], G0[kPix / S], G1[kPix / S], G2[kPix / S];
    uint32_t lp[kPix / S];
    load_checkpoint<S>(V, tile, T, lp, G0, G1, G2);
    tile_bwd<KIND, DET, S>(V, tile, blockIdx.x, n, kp, o, T, lp, G0, G1, G2, d);
}

// Backward with the long walks split: one four-wavefront workgroup per tile.
// Wavefront h first reads the checkpointed positions of rows 4h .. 4h+3 (one
// pixel per lane); the tile's cost is its walk, the largest position past the
// tile's start.  A walk longer than split2 (split4) instances is shared by two
// (four) wavefronts, each taking 8 (4) of the tile's rows and walking only to
// its own pixels' largest position; otherwise wavefront 0 takes the whole tile
// (four pixels per lane) and the others leave after the one barrier.  So the
// heaviest tiles no longer run alone at the end of the launch, and consecutive
// workgroups (which the hardware deals to different XCDs) are different tiles.
// A one-wavefront lane's k-th pixel (row lane/16 + 4k) is lane `lane` of
// wavefront k here, and a two-wavefront part h's k-th pixel is wavefront
// 2h + k's: the positions are shared through LDS.  The sums per splat are
// those of the one-wavefront backward in another order (atomic accumulation).
//
// Heavy-first order: with nonzero thresholds h0 >= h1 the grid holds every tile
// once per class (walks above h0, above h1, the rest; a zero threshold drops
// its class); the workgroup of the tile's own class takes it and the others
// leave after reading its checkpoint.  The hardware dispatches workgroups in
// order, so the longest walks start first and overlap the rest instead of
// running alone at the end of the launch.
__device__ __forceinline__ uint32_t walk_class(uint32_t walk, uint32_t h0, uint32_t h1) {
    return (h0 && walk > h0) ? 0u : (h1 && walk > h1) ? (h0 ? 1u : 0u) : (h0 ? 1u : 0u) + (h1 ? 1u : 0u);
}

template <int KIND, class VS>
__global__ __launch_bounds__(256) void k_raster_bwd_split(VS A, int n, KParams kp, ROpts o, uint32_t split2,
                                                          uint32_t split4, uint32_t h0, uint32_t h1) {
    __shared__ uint32_t lps[4][64];
    __shared__ uint32_t wmax[4];
    int tile;
    const uint32_t ncls = 1u + (h0 ? 1u : 0u) + (h1 ? 1u : 0u);
    const uint32_t nitems = gridDim.x / ncls;
    const uint32_t cls = blockIdx.x / nitems;
    const uint32_t item = blockIdx.x - cls * nitems;
    const RView &V = A.get(item, tile);
    if (V.overflow && *V.overflow) return;
    const int h = threadIdx.x >> 6, lane = threadIdx.x & 63;
    {
        const LanePix<4> P4(tile, V.gx, h);
        const bool in = P4.ix < V.W && P4.iy0 < V.H;
        const uint32_t l = in ? V.last[(size_t)P4.iy0 * V.W + P4.ix] : kNone;
        const uint32_t lp = l == kNone ? 0u : l + 1u;
        lps[h][lane] = lp;
        const uint32_t m = wave_max_u32(lp);
        if (lane == 0) wmax[h] = m;
    }
    __syncthreads();
    const uint32_t start = V.ranges[2 * tile], end = V.ranges[2 * tile + 1];
    const uint32_t maxl = min(max(max(wmax[0], wmax[1]), max(wmax[2], wmax[3])), end);
    const uint32_t walk = maxl > start ? maxl - start : 0u;
    if (walk_class(walk, h0, h1) != cls) return;  // another class's workgroup takes this tile
    const int parts = walk > split4 ? 4 : (walk > split2 ? 2 : 1);
    if (h >= parts) return;
    const size_t plane = (size_t)V.W * V.H;
    // checkpoint of this part's pixels: T, dL/dI where the pixel blended
    auto load = [&](int ix, int iy, uint32_t lp, float &T, float &g0, float &g1, float &g2) {
        T = g0 = g1 = g2 = 0.0f;
        if (lp != 0u) {
            const size_t pidx = (size_t)iy * V.W + ix;
            T = V.final_T[pidx];
            g0 = V.dL[pidx];
            g1 = V.dL[plane + pidx];
            g2 = V.dL[2 * plane + pidx];
        }
    };
    if (parts == 1) {
        const LanePix<1> P(tile, V.gx, 0);
        float T[4], G0[4], G1[4], G2[4];
        uint32_t lp[4];
#pragma unroll
        for (int k = 0; k < 4; k++) {
            lp[k] = lps[k][lane];
            load(P.ix, P.iy0 + 4 * k, lp[k], T[k], G0[k], G1[k], G2[k]);
        }
        tile_bwd<KIND, false, 1>(V, tile, item, n, kp, o, T, lp, G0, G1, G2, DetOut{}, 0);
    } else if (parts == 2) {
        const LanePix<2> P(tile, V.gx, h);
        float T[2], G0[2], G1[2], G2[2];
        uint32_t lp[2];
#pragma unroll
        for (int k = 0; k < 2; k++) {
            lp[k] = lps[2 * h + k][lane];
            load(P.ix, P.iy0 + 4 * k, lp[k], T[k], G0[k], G1[k], G2[k]);
        }
        tile_bwd<KIND, false, 2>(V, tile, item, n, kp, o, T, lp, G0, G1, G2, DetOut{}, h);
    } else {
        const LanePix<4> P(tile, V.gx, h);
        float T[1], G0[1], G1[1], G2[1];
        uint32_t lp[1];
        lp[0] = lps[h][lane];
        load(P.ix, P.iy0, lp[0], T[0], G0[0], G1[0], G2[0]);
        tile_bwd<KIND, false, 4>(V, tile, item, n, kp, o, T, lp, G0, G1, G2, DetOut{}, h);
    }
}

// Forward, per-pixel loss gradient and backward of one tile in one wavefront.
template <int KIND, int LOSS, class VS>
__global__ __launch_bounds__(64) void k_raster_fwdbwd(VS A, int n, KParams kp, ROpts o) {
    constexpr int S = 1, NP = kPix;
    int tile;
    const RView &V = A.get(blockIdx.x, tile);
    if (V.overflow && *V.overflow) return;
    PixF<NP> F;
    tile_fwd<KIND, S, true>(V, tile, n, kp, o, F);
    store_fwd<S>(V, tile, F, o);
    const LanePix<S> P(tile, V.gx);
    const int ix = P.ix, iy0 = P.iy0;
    const size_t plane = (size_t)V.W * V.H;
    float G0[NP], G1[NP], G2[NP];
    uint32_t lp[NP];
#pragma unroll
    for (int k = 0; k < NP; k++) {
        int iy = iy0 + 4 * k;
        G0[k] = G1[k] = G2[k] = 0.0f;
        lp[k] = F.lst[k] == kNone ? 0u : F.lst[k] + 1u;
        if (ix < V.W && iy < V.H) {
            size_t pidx = (size_t)iy * V.W + ix;
            // the image values exactly as stored above
            G0[k] = loss_grad<LOSS>(fmaf(F.T[k], o.bg0, F.C0[k]), V.target[pidx], V.loss_scale);
            G1[k] = loss_grad<LOSS>(fmaf(F.T[k], o.bg1, F.C1[k]), V.target[plane + pidx], V.loss_scale);
            G2[k] = loss_grad<LOSS>(fmaf(F.T[k], o.bg2, F.C2[k]), V.target[2 * plane + pidx], V.loss_scale);
        }
    }
    tile_bwd<KIND, false, S>(V, tile, blockIdx.x, n, kp, o, F.T, lp, G0, G1, G2, DetOut{});
}

// Deterministic mode, pass 0: number of partials of each work item (the same
// walk end as the backward computes).
template <class VS>
__global__ __launch_bounds__(64) void k_trav_len(VS A, uint32_t *len) {
    int tile;
    const RView &V = A.get(blockIdx.x, tile);
    uint32_t out = 0;
    if (!(V.overflow && *V.overflow)) {
        float T[kPix], G0[kPix], G1[kPix], G2[kPix];
        uint32_t lp[kPix];
        load_checkpoint<1>(V, tile, T, lp, G0, G1, G2);
        uint32_t maxl = max(max(lp[0], lp[1]), max(lp[2], lp[3]));
        maxl = wave_max_u32(maxl);
        const uint32_t start = V.ranges[2 * tile], end = V.ranges[2 * tile + 1];
        maxl = min(maxl, end);
        out = maxl > start ? maxl - start : 0u;
    }
    if (threadIdx.x == 0) len[blockIdx.x] = out;
}

struct DetHdr {
    uint32_t total;  // number of stored partials
    int32_t zero;    // always 0 (the "skip" flag of the scan and sort kernels)
};

__global__ void k_det_init(DetHdr *h) {
    if (threadIdx.x == 0) {
        h->total = 0;
        h->zero = 0;
    }
}

// Deterministic mode, pass 2: per splat (run of equal keys in the stably
// sorted list) the sum of its partials in tile order.
template <class VS>
__global__ __launch_bounds__(256) void k_det_reduce(VS A, uint32_t n, const uint32_t *skey, const uint32_t *sval,
                                                    const float *parts, uint32_t cap, const DetHdr *hdr,
                                                    uint32_t limit) {
    const uint32_t total = hdr->total;
    for (uint32_t i = blockIdx.x * blockDim.x + threadIdx.x; i < total; i += gridDim.x * blockDim.x) {
        const uint32_t key = skey[i];
        if (key >= limit) continue;
        if (i > 0 && skey[i - 1] == key) continue;
        // FP64 sum over the splat's tiles: a large splat collects thousands of
        // per-tile partials of mixed sign
        double acc[9];
#pragma unroll
        for (int k = 0; k < 9; k++) acc[k] = 0.0;
        for (uint32_t j = i; j < total && skey[j] == key; j++) {
            const size_t c = sval[j];
#pragma unroll
            for (int k = 0; k < 9; k++) acc[k] += (double)parts[(size_t)k * cap + c];
        }
        const uint32_t vi = key / n, id = key - vi * n;
        const darb_grads2d g = A.grads(vi);
        g.xy[2 * id] = (float)acc[0];
        g.xy[2 * id + 1] = (float)acc[1];
        g.conic[3 * id] = (float)acc[2];
        g.conic[3 * id + 1] = (float)acc[3];
        g.conic[3 * id + 2] = (float)acc[4];
        g.opacity[id] = (float)acc[5];
        g.rgb[3 * id] = (float)acc[6];
        g.rgb[3 * id + 1] = (float)acc[7];
        g.rgb[3 * id + 2] = (float)acc[8];
    }
}

// The four 2D-gradient arrays of a view in one launch (n splats: 2n, 3n, n, 3n
// floats); each block clears a contiguous stretch of one array.
__global__ __launch_bounds__(256) void k_zero_grads2d(darb_grads2d g, size_t n) {
    const size_t chunk = (size_t)256 * 16;
    const size_t nb0 = (2 * n + chunk - 1) / chunk, nb1 = (3 * n + chunk - 1) / chunk, nb2 = (n + chunk - 1) / chunk;
    size_t b = blockIdx.x;
    float *a;
    size_t len;
    if (b < nb0) {
        a = g.xy, len = 2 * n;
    } else if ((b -= nb0) < nb1) {
        a = g.conic, len = 3 * n;
    } else if ((b -= nb1) < nb2) {
        a = g.opacity, len = n;
    } else {
        b -= nb2;
        a = g.rgb, len = 3 * n;
    }
    const size_t end = min(len, (b + 1) * chunk);
    for (size_t i = b * chunk + threadIdx.x; i < end; i += 256) a[i] = 0.0f;
}

inline size_t align_up(size_t x) { return (x + 255) & ~(size_t)255; }

struct DetLayout {
    size_t hdr, trav, sparts, parts, kA, vA, kB, vB, hist, total;
};

DetLayout det_layout(uint32_t items, uint64_t cap) {
    DetLayout L;
    size_t off = 0;
    const uint32_t cap32 = (uint32_t)cap;
    const size_t hist_n = radix_hist_words(cap32);
    const size_t sp = scan_parts_words(items);
    L.hdr = off; off += align_up(sizeof(DetHdr));
    L.trav = off; off += align_up(((size_t)items + 1) * 4);
    L.sparts = off; off += align_up(sp * 4);
    L.parts = off; off += align_up((size_t)9 * cap * 4);
    L.kA = off; off += align_up((size_t)cap * 4);
    L.vA = off; off += align_up((size_t)cap * 4);
    L.kB = off; off += align_up((size_t)cap * 4);
    L.vB = off; off += align_up((size_t)cap * 4);
    L.hist = off; off += align_up(hist_n * 4);
    L.total = off;
    return L;
}

int bits_for(uint64_t v) {
    int b = 0;
    while (b < 32 && (v >> b) != 0) b++;
    return b;
}

}  // namespace

size_t det_workspace(uint32_t items, uint64_t capacity) { return det_layout(items, capacity).total; }

#define DARB_KIND_SWITCH(kind, F, ...)                     \
    switch (kind) {                                        \
    case DARB_GAUSS: F<DARB_GAUSS> __VA_ARGS__; break;     \
    case DARB_HALF_COS: F<DARB_HALF_COS> __VA_ARGS__; break; \
    case DARB_RAISED_COS: F<DARB_RAISED_COS> __VA_ARGS__; break; \
    case DARB_SINC: F<DARB_SINC> __VA_ARGS__; break;       \
    case DARB_IMQ: F<DARB_IMQ> __VA_ARGS__; break;         \
    case DARB_IMQ_SQRT: F<DARB_IMQ_SQRT> __VA_ARGS__; break; \
    case DARB_PARABOLA: F<DARB_PARABOLA> __VA_ARGS__; break; \
    default: F<DARB_GAUSS_BETA> __VA_ARGS__; break;        \
    }

namespace {

template <int KIND>
void fwd_launch(const RViews &V, uint32_t items, int n, const KParams &kp, const ROpts &o, hipStream_t s) {
    bool cnt = false;
    for (int v = 0; v < V.nv; v++) cnt |= V.v[v].n_contrib != nullptr;
    if (V.nv == 1) {
        if (cnt)
            hipLaunchKernelGGL((k_raster_fwd<KIND, OneView, true>), dim3(items), dim3(64 * kSplit), 0, s,
                               OneView{V.v[0]}, n, kp, o);
        else
            hipLaunchKernelGGL((k_raster_fwd<KIND, OneView, false>), dim3(items), dim3(64 * kSplit), 0, s,
                               OneView{V.v[0]}, n, kp, o);
    } else {
        if (cnt)
            hipLaunchKernelGGL((k_raster_fwd<KIND, ManyViews, true>), dim3(items), dim3(64 * kSplit), 0, s,
                               ManyViews{V}, n, kp, o);
        else
            hipLaunchKernelGGL((k_raster_fwd<KIND, ManyViews, false>), dim3(items), dim3(64 * kSplit), 0, s,
                               ManyViews{V}, n, kp, o);
    }
}

// Walks longer than these (instances past the tile's start) are shared by two /
// four wavefronts in the atomic backward.
#ifndef DARB_BWD_SPLIT2
#define DARB_BWD_SPLIT2 512
#endif
#ifndef DARB_BWD_SPLIT4
#define DARB_BWD_SPLIT4 1024
#endif
// Walks longer than HEAVY0 go first, then those longer than HEAVY1 (0: no such
// class).  Tuning constants: on the 3M-splat scene (mean walk ~117, longest
// ~370) a single class above 96 took the backward from 187 to 166 us.
#ifndef DARB_BWD_HEAVY0
#define DARB_BWD_HEAVY0 0
#endif
#ifndef DARB_BWD_HEAVY1
#define DARB_BWD_HEAVY1 48
#endif

template <int KIND>
void bwd_launch(const RViews &V, uint32_t items, int n, const KParams &kp, const ROpts &o, bool det, const DetOut &d,
                hipStream_t s) {
    const uint32_t s2 = DARB_BWD_SPLIT2, s4 = DARB_BWD_SPLIT4;
    // heavy-first classes (the grid of one workgroup per tile and class must fit
    // the launch's 32-bit grid size)
    const bool fits = items <= 0x55555555u;
    const uint32_t h0 = fits ? DARB_BWD_HEAVY0 : 0u, h1 = fits ? DARB_BWD_HEAVY1 : 0u;
    const uint32_t ncls = 1u + (h0 ? 1u : 0u) + (h1 ? 1u : 0u);
    if (V.nv == 1) {
        if (det)
            hipLaunchKernelGGL((k_raster_bwd<KIND, true, OneView>), dim3(items), dim3(64), 0, s, OneView{V.v[0]}, n,
                               kp, o, d);
        else
            hipLaunchKernelGGL((k_raster_bwd_split<KIND, OneView>), dim3(ncls * items), dim3(256), 0, s,
                               OneView{V.v[0]}, n, kp, o, s2, s4, h0, h1);
    } else {
        if (det)
            hipLaunchKernelGGL((k_raster_bwd<KIND, true, ManyViews>), dim3(items), dim3(64), 0, s, ManyViews{V}, n, kp,
                               o, d);
        else
            hipLaunchKernelGGL((k_raster_bwd_split<KIND, ManyViews>), dim3(ncls * items), dim3(256), 0, s,
                               ManyViews{V}, n, kp, o, s2, s4, h0, h1);
    }
}

template <int KIND>
void fwdbwd_launch(int loss, const RViews &V, uint32_t items, int n, const KParams &kp, const ROpts &o,
                   hipStream_t s) {
    if (loss == DARB_LOSS_L1)
        hipLaunchKernelGGL((k_raster_fwdbwd<KIND, DARB_LOSS_L1, ManyViews>), dim3(items), dim3(64), 0, s, ManyViews{V},
                           n, kp, o);
    else
        hipLaunchKernelGGL((k_raster_fwdbwd<KIND, DARB_LOSS_L2, ManyViews>), dim3(items), dim3(64), 0, s, ManyViews{V},
                           n, kp, o);
}

hipError_t zero_grads(const RViews &V, int n, hipStream_t s) {
    if (n <= 0) return hipSuccess;
    const size_t chunk = (size_t)256 * 16, nn = (size_t)n;
    const size_t blocks = (2 * nn + chunk - 1) / chunk + (3 * nn + chunk - 1) / chunk + (nn + chunk - 1) / chunk +
                          (3 * nn + chunk - 1) / chunk;
    for (int v = 0; v < V.nv; v++)
        hipLaunchKernelGGL(k_zero_grads2d, dim3((unsigned)blocks), dim3(256), 0, s, V.v[v].g2, nn);
    return hipGetLastError();
}

}  // namespace

hipError_t launch_raster_fwd(int kind, const RViews &V, uint32_t items, int n, const KParams &kp, const ROpts &o,
                             hipStream_t s) {
    if (items == 0) return hipSuccess;
    DARB_KIND_SWITCH(kind, fwd_launch, (V, items, n, kp, o, s))
    return hipGetLastError();
}

hipError_t launch_raster_bwd(int kind, const RViews &V, uint32_t items, int n, const KParams &kp, const ROpts &o,
                             void *det_ws, uint64_t det_capacity, bool g2_zeroed, hipStream_t s) {
    hipError_t e;
    if (!g2_zeroed && (e = zero_grads(V, n, s)) != hipSuccess) return e;
    if (items == 0 || n == 0) return hipGetLastError();
    if (!det_ws) {
        DARB_KIND_SWITCH(kind, bwd_launch, (V, items, n, kp, o, false, DetOut{}, s))
        return hipGetLastError();
    }
    const DetLayout L = det_layout(items, det_capacity);
    char *base = static_cast<char *>(det_ws);
    auto U = [&](size_t off) { return reinterpret_cast<uint32_t *>(base + off); };
    DetHdr *hdr = reinterpret_cast<DetHdr *>(base + L.hdr);
    const uint32_t cap = (uint32_t)det_capacity;
    uint32_t *trav = U(L.trav), *sparts = U(L.sparts), *kA = U(L.kA), *vA = U(L.vA), *kB = U(L.kB), *vB = U(L.vB);
    float *parts = reinterpret_cast<float *>(base + L.parts);
    hipLaunchKernelGGL(k_det_init, dim3(1), dim3(64), 0, s, hdr);
    if (V.nv == 1)
        hipLaunchKernelGGL((k_trav_len<OneView>), dim3(items), dim3(64), 0, s, OneView{V.v[0]}, trav);
    else
        hipLaunchKernelGGL((k_trav_len<ManyViews>), dim3(items), dim3(64), 0, s, ManyViews{V}, trav);
    if ((e = scan_u32(trav, nullptr, items, sparts, &hdr->total, &hdr->zero, s)) != hipSuccess) return e;
    const DetOut d{parts, kA, vA, trav, cap};
    DARB_KIND_SWITCH(kind, bwd_launch, (V, items, n, kp, o, true, d, s))
    const uint64_t limit = (uint64_t)V.nv * (uint64_t)n;
    const int bits = bits_for(limit);  // 2^bits > limit: kNone keys sort after every valid key
    if ((e = radix_sort_pairs(kA, vA, kB, vB, &hdr->total, cap, bits, U(L.hist), &hdr->zero, s)) != hipSuccess)
        return e;
    const bool in_b = ((bits + 7) / 8) % 2 == 1;
    const uint32_t *sk = in_b ? kB : kA, *sv = in_b ? vB : vA;
    const unsigned blocks = (unsigned)std::min<uint64_t>((det_capacity + 255) / 256, 8192);
    if (blocks > 0) {
        if (V.nv == 1)
            hipLaunchKernelGGL((k_det_reduce<OneView>), dim3(blocks), dim3(256), 0, s, OneView{V.v[0]}, (uint32_t)n,
                               sk, sv, parts, cap, hdr, (uint32_t)limit);
        else
            hipLaunchKernelGGL((k_det_reduce<ManyViews>), dim3(blocks), dim3(256), 0, s, ManyViews{V}, (uint32_t)n, sk,
                               sv, parts, cap, hdr, (uint32_t)limit);
    }
    return hipGetLastError();
}

hipError_t launch_raster_fwdbwd(int kind, int loss, const RViews &V, uint32_t items, int n, const KParams &kp,
                                const ROpts &o, hipStream_t s) {
    hipError_t e;
    if ((e = zero_grads(V, n, s)) != hipSuccess) return e;
    if (items == 0) return hipGetLastError();
    DARB_KIND_SWITCH(kind, fwdbwd_launch, (loss, V, items, n, kp, o, s))
    return hipGetLastError();
}

}  // namespace darb
