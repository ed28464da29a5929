// Device-side tile renderer shared by the batched render kernel and the
// serving kernel (see lf_render.hip for the design).
#pragma once

#include <hip/hip_runtime.h>

#include "lf_internal.h"


struct Ray {
    int a0, a1, b0, b1, x0, x1, y0, y1;
    float fu, fv, fs, ft;
};

__device__ __forceinline__ Ray lf_ray_setup(const LfGeom& g, const float* __restrict__ cam, int i, int j)
{
    Ray r;
    float u, v, s, t;
    lf_ray(cam, i, j, u, v, s, t);
    lf_axis(u, g.na, r.a0, r.a1, r.fu);
    lf_axis(v, g.nb, r.b0, r.b1, r.fv);
    lf_axis(s, g.w, r.x0, r.x1, r.fs);
    lf_axis(t, g.h, r.y0, r.y1, r.ft);
    return r;
}

// Quadrilinear blend of 16 samples given as unscaled 8-bit values (sample
// 4 q + k: view q = (v-bit << 1 | u-bit), pixel k = (t-bit << 1 | s-bit)):
// per view the st-bilinear sum with weights (1-fs)(1-ft), fs(1-ft), (1-fs)ft,
// fs ft, then the uv-bilinear sum of the four, in that fixed order; scaled
// by 1/255 at the end.
struct BlendW {
    float st[4], uv[4];
};

__device__ __forceinline__ BlendW lf_blend_weights(const Ray& r)
{
    BlendW w;
    const float gs = 1.0f - r.fs, gt = 1.0f - r.ft, gu = 1.0f - r.fu, gv = 1.0f - r.fv;
    w.st[0] = gs * gt;
    w.st[1] = r.fs * gt;
    w.st[2] = gs * r.ft;
    w.st[3] = r.fs * r.ft;
    w.uv[0] = gu * gv;
    w.uv[1] = r.fu * gv;
    w.uv[2] = gu * r.fv;
    w.uv[3] = r.fu * r.fv;
    return w;
}

__device__ __forceinline__ float lf_blend16(const float (&sm)[16], const BlendW& w)
{
    float acc = 0.0f;
#pragma unroll
    for (int q = 0; q < 4; q++) {
        float t = sm[4 * q] * w.st[0];
        t = fmaf(sm[4 * q + 1], w.st[1], t);
        t = fmaf(sm[4 * q + 2], w.st[2], t);
        t = fmaf(sm[4 * q + 3], w.st[3], t);
        acc = q == 0 ? t * w.uv[0] : fmaf(t, w.uv[q], acc);
    }
    return acc * (1.0f / 255.0f);
}

// ---------------------------------------------------------------------------
// per-ray reference path
// ---------------------------------------------------------------------------

// SRV values of node (B, A) of level l, channel c, at the pixels (ys[k >> 1],
// xs[k & 1]), k < 4: a reference node reads its resident SRV; a predictive
// node adds its dequantised residual and its phase-signed prediction.  The
// block descriptor (table entry and motion record) is read once when the four
// pixels share a block.
template <int RES>
__device__ inline void lf_srv_quad(const LfGeom& g, const LfPtrs& p, int c, int l, int B, int A, const int ys[2],
                                   const int xs[2], int v[4])
{
    const uint32_t rp = lf_ref_index(g, c, l, B >> 1, A >> 1);
    if (!((A | B) & 1)) {
#pragma unroll
        for (int k = 0; k < 4; k++) v[k] = lf_ref_tap<RES>(g, p, rp, ys[k >> 1], xs[k & 1]);
        return;
    }
    const int node = g.node_base[l] + B * g.na_l[l] + A;
    const uint32_t rec = (uint32_t)(pred_ordinal(g.na_l[l], B, A) * g.nblk);
    const size_t tab = ((size_t)c * g.n_nodes + node) * g.nblk;
    int blk0 = -1, mode = 0, mn = 0, mx = 0, my = 0, sg = 0;
    uint32_t word = 0;
#pragma unroll 1  // unrolled, the four inlined walks of a ray exhaust the registers
    for (int k = 0; k < 4; k++) {
        const int y = ys[k >> 1], x = xs[k & 1];
        const int blk = (y >> g.bsl) * g.nbx + (x >> g.bsl);
        if (blk != blk0) {
            const uint2 e = p.table[tab + blk];
            mode = (int)((e.y >> 16) & 0xFFu);
            mn = (int)(int16_t)(e.y & 0xFFFFu);
            word = e.x;
            lf_motion(g, p, c, l, rec + (uint32_t)blk, mx, my, sg);
            blk0 = blk;
        }
        const int i = ((y & (g.bs - 1)) << g.bsl) | (x & (g.bs - 1));
        int r = mode == LF_MODE_ZERO ? 0 : (mn + (int)lf_bise_get(p.payload + word, mode, (uint32_t)i)) * g.step[l];
        if (sg) r += sg * lf_qpel<RES>(g, p, rp, y, x, mx, my);
        v[k] = r;
    }
}

// One channel of the 16 samples of a ray (4 views x 4 pixels; sample k is
// view k >> 2 = b0a0, b0a1, b1a0, b1a1 and pixel k & 3): root plus the SRVs
// of levels lod .. H-1.  Per level, views whose tree nodes coincide share one
// SRV evaluation (views (b, a) and (b', a') share the level-l node when
// b >> l == b' >> l and a >> l == a' >> l): the same sums as 16 independent
// tree walks.
template <int RES>
__device__ __forceinline__ void lf_ray_channel(const LfGeom& g, const LfPtrs& p, const Ray& r, int c, int lod,
                                               int acc[16])
{
    const int ys[2] = {r.y0, r.y1}, xs[2] = {r.x0, r.x1};
    const int H = g.H;
    {
        const bool eqA = (r.a0 >> H) == (r.a1 >> H), eqB = (r.b0 >> H) == (r.b1 >> H);
        const size_t plane = (size_t)g.w * g.h;
        int v[4][4];
#pragma unroll
        for (int q = 0; q < 4; q++) {
            const int b = (q & 2) ? r.b1 : r.b0, a = (q & 1) ? r.a1 : r.a0;
            const bool dup = (q == 1 && eqA) || (q == 2 && eqB) || (q == 3 && (eqA || eqB));
            if (!dup) {
                const int16_t* rt = p.root + ((size_t)(c * g.root_nb + (b >> H)) * g.root_na + (a >> H)) * plane;
#pragma unroll
                for (int k = 0; k < 4; k++) v[q][k] = rt[ys[k >> 1] * g.w + xs[k & 1]];
            }
        }
#pragma unroll
        for (int k = 0; k < 4; k++) {
            if (eqA) v[1][k] = v[0][k];
            if (eqB) v[2][k] = v[0][k];
            if (eqB) v[3][k] = v[1][k];
            else if (eqA) v[3][k] = v[2][k];
#pragma unroll
            for (int q = 0; q < 4; q++) acc[4 * q + k] = v[q][k];
        }
    }
    for (int l = lod; l < H; l++) {
        const bool eqA = (r.a0 >> l) == (r.a1 >> l), eqB = (r.b0 >> l) == (r.b1 >> l);
        int v[4][4];
        lf_srv_quad<RES>(g, p, c, l, r.b0 >> l, r.a0 >> l, ys, xs, v[0]);
        if (!eqA) lf_srv_quad<RES>(g, p, c, l, r.b0 >> l, r.a1 >> l, ys, xs, v[1]);
        if (!eqB) lf_srv_quad<RES>(g, p, c, l, r.b1 >> l, r.a0 >> l, ys, xs, v[2]);
        if (!eqA && !eqB) lf_srv_quad<RES>(g, p, c, l, r.b1 >> l, r.a1 >> l, ys, xs, v[3]);
#pragma unroll
        for (int k = 0; k < 4; k++) {
            if (eqA) v[1][k] = v[0][k];
            if (eqB) v[2][k] = v[0][k];
            if (eqB) v[3][k] = v[1][k];
            else if (eqA) v[3][k] = v[2][k];
#pragma unroll
            for (int q = 0; q < 4; q++) acc[4 * q + k] += v[q][k];
        }
    }
}

template <int RES = LF_RES_DENSE>
__device__ inline void lf_render_one(const LfGeom& g, const LfPtrs& p, const float* __restrict__ cam, int i, int j,
                                     float out[3], int lod = 0)
{
    const Ray r = lf_ray_setup(g, cam, i, j);
    int Y[16], Co[16], Cg[16];
    lf_ray_channel<RES>(g, p, r, 0, lod, Y);
    lf_ray_channel<RES>(g, p, r, 1, lod, Co);
    lf_ray_channel<RES>(g, p, r, 2, lod, Cg);
    uint32_t px[16];
#pragma unroll
    for (int k = 0; k < 16; k++) {
        int R, G, B;
        lf_ycocg_to_rgb(Y[k], Co[k], Cg[k], R, G, B);
        px[k] = (uint32_t)R | ((uint32_t)G << 8) | ((uint32_t)B << 16);
    }
    const BlendW w = lf_blend_weights(r);
#pragma unroll
    for (int c = 0; c < 3; c++) {
        float sm[16];
#pragma unroll
        for (int k = 0; k < 16; k++) sm[k] = (float)((px[k] >> (8 * c)) & 255u);
        out[c] = lf_blend16(sm, w);
    }
}

// One ray of a 4:2:0 stream (luma geometry g, p; chroma geometry gc, pc):
// each of the 16 samples is luma plus up-sampled Co and Cg, blended as in
// lf_render_one.
__device__ inline void lf_render_one420(const LfGeom& g, const LfPtrs& p, const LfGeom& gc, const LfPtrs& pc,
                                        const float* __restrict__ cam, int i, int j, float out[3], int lod = 0)
{
    const Ray ray = lf_ray_setup(g, cam, i, j);
    uint32_t rgb[16];
#pragma unroll 1
    for (int k = 0; k < 16; k++) {
        const int b = (k & 8) ? ray.b1 : ray.b0, a = (k & 4) ? ray.a1 : ray.a0;
        const int y = (k & 2) ? ray.y1 : ray.y0, x = (k & 1) ? ray.x1 : ray.x0;
        int R, G, B;
        lf_ycocg_to_rgb(lf_decode_channel(g, p, 0, b, a, y, x, lod), lf_chroma_up(gc, pc, 0, b, a, y, x, lod),
                        lf_chroma_up(gc, pc, 1, b, a, y, x, lod), R, G, B);
        rgb[k] = (uint32_t)R | ((uint32_t)G << 8) | ((uint32_t)B << 16);
    }
    const BlendW w = lf_blend_weights(ray);
#pragma unroll
    for (int c = 0; c < 3; c++) {
        float sm[16];
#pragma unroll
        for (int k = 0; k < 16; k++) sm[k] = (float)((rgb[k] >> (8 * c)) & 255u);
        out[c] = lf_blend16(sm, w);
    }
}

// ---------------------------------------------------------------------------
// batched tile renderer
// ---------------------------------------------------------------------------

#ifndef GROUP_FIRST
#define GROUP_FIRST(gmax) (gmax)
#endif
#define TW 32
#define TH 8
#define NT (TW * TH)
#define FMAX 64          // views per workgroup chunk (4 FMAX <= NT: phase 0 gives each view 4 lanes)
#define LMAX 64          // nodes of one level inside a group's bounding rectangle
#define SLOT_MAX 192  // staged channel planes decoded for one group (3 x CMAX)
#define CMAX 64       // cache entries per kind (leaf views, ancestor nodes)
#define CKEY_EMPTY 0xFFFFFFFFu

// LDS staging budgets (entries): descriptors (16 B), assembled samples (4 B),
// staged ancestor/root values (2 B).  About 46 KiB plus 6 KiB of tables keeps
// three 256-thread workgroups resident per CU.
#define B_DESC 384
#define B_RGBA 4096
#define B_SVAL 12288
#define LDS_DYN_BYTES (B_DESC * 16 + B_RGBA * 4 + B_SVAL * 2)
// Blocks smaller than 16x16: a tile's footprint spans four times as many
// blocks per node at 8x8, so a single view can need more descriptors and
// decoded values than the budgets above hold.  The small-block instance takes
// larger budgets and runs two workgroups per CU instead of three.
#define B_DESC_SB 1024
#define B_RGBA_SB 6144
#define B_SVAL_SB 16384
#define LDS_DYN_BYTES_SB (B_DESC_SB * 16 + B_RGBA_SB * 4 + B_SVAL_SB * 2)

// 16-bit packed min/max (both halves at once)
typedef unsigned short lf_u16x2 __attribute__((ext_vector_type(2)));

__device__ __forceinline__ uint32_t pk_min(uint32_t a, uint32_t b)
{
    lf_u16x2 x = __builtin_bit_cast(lf_u16x2, a), y = __builtin_bit_cast(lf_u16x2, b);
    return __builtin_bit_cast(uint32_t, __builtin_elementwise_min(x, y));
}

__device__ __forceinline__ uint32_t pk_max(uint32_t a, uint32_t b)
{
    lf_u16x2 x = __builtin_bit_cast(lf_u16x2, a), y = __builtin_bit_cast(lf_u16x2, b);
    return __builtin_bit_cast(uint32_t, __builtin_elementwise_max(x, y));
}

__device__ __forceinline__ uint32_t wave_pk_min(uint32_t v)
{
#pragma unroll
    for (int o = 32; o > 0; o >>= 1) v = pk_min(v, (uint32_t)__shfl_xor((int)v, o, 64));
    return v;
}

__device__ __forceinline__ uint32_t wave_pk_max(uint32_t v)
{
#pragma unroll
    for (int o = 32; o > 0; o >>= 1) v = pk_max(v, (uint32_t)__shfl_xor((int)v, o, 64));
    return v;
}

// Bounded-integer value i of a block, one code path for the three families
// (no divergence between neighbouring blocks of different families): a value
// is (high digit << b) | b-bit low part, where the group of G values (G = 1,
// 5 or 3) starts with an hb-bit header (hb = 0, 8 or 7).  Table entries
// tab[t] hold the base-3 digits of t and tab[256 + q] the base-5 digits of q,
// one per 4-bit nibble (tab[0] = 0, so the empty header of plain bits reads
// digit 0); tab[LF_TAB_QUAD + 5 fam + r] describes a quad (below).
#define LF_TAB_QUAD 384
#define LF_TAB_SIZE (LF_TAB_QUAD + 15)

__device__ __forceinline__ uint32_t lf_bise_any(const uint32_t* __restrict__ w, uint32_t mode, uint32_t i,
                                                const uint32_t* __restrict__ tab)
{
    const uint32_t fam = mode >> 5, b = mode & 31u;
    const uint32_t hb = fam == 0u ? 0u : (fam == 1u ? 8u : 7u);
    const uint32_t gs = fam == 0u ? 1u : (fam == 1u ? 5u : 3u);
    const uint32_t mg = fam == 1u ? 858993460u : 1431655766u;  // ceil(2^32 / 5), ceil(2^32 / 3)
    const uint32_t grp = fam == 0u ? i : __umulhi(i, mg);
    const uint32_t k = i - __umul24(grp, gs);
    const uint32_t base = __umul24(grp, hb + gs * b);
    const uint32_t head = lf_field(w, base, (int)hb);
    const uint32_t lo = lf_field(w, base + hb + __umul24(k, b), (int)b);
    const uint32_t dig = tab[(fam == 2u ? 256u : 0u) + head];
    return (((dig >> (4u * k)) & 15u) << b) | lo;
}

// Fill the shared decode table (every thread of the workgroup calls it).
__device__ __forceinline__ void lf_fill_tab(uint32_t* tab)
{
    for (uint32_t t = threadIdx.x; t < LF_TAB_SIZE; t += blockDim.x) {
        uint32_t d = 0;
        if (t < 256u) {
            uint32_t v = t;
            for (int k = 0; k < 5; k++, v /= 3u) d |= (v % 3u) << (4 * k);
        } else if (t < LF_TAB_QUAD) {
            uint32_t v = t - 256u;
            for (int k = 0; k < 3; k++, v /= 5u) d |= (v % 5u) << (4 * k);
        } else {
            // quad starting at position r of its group, family fam: for value
            // k, 5 bits = group step from the quad's first group (2) | digit
            // index inside the group (3) << 2
            const uint32_t fam = (t - LF_TAB_QUAD) / 5u, r = (t - LF_TAB_QUAD) % 5u;
            const uint32_t gs = fam == 0u ? 1u : (fam == 1u ? 5u : 3u);
            for (uint32_t k = 0; k < 4; k++) {
                const uint32_t q = (fam == 0u ? 0u : r) + k;
                d |= ((q / gs) | ((q % gs) << 2)) << (5 * k);
            }
        }
        tab[t] = d;
    }
}

// Packed 16-bit lanes.  Decoded values of a valid stream stay far inside
// int16 (reference SRVs are checked to |v| <= 2047 at load, so even the
// 16x-weighted prediction sums fit), so pairs of pixels are carried in one
// register and added, scaled and shifted two at a time.
typedef short lf_i16x2 __attribute__((ext_vector_type(2)));

__device__ __forceinline__ lf_i16x2 lf_as_i16x2(uint32_t v) { return __builtin_bit_cast(lf_i16x2, v); }
__device__ __forceinline__ uint32_t lf_as_u32(lf_i16x2 v) { return __builtin_bit_cast(uint32_t, v); }
__device__ __forceinline__ lf_i16x2 lf_splat(int v) { return (lf_i16x2)(short)v; }
// low halves of a and b as one pair (a in the low half)
__device__ __forceinline__ uint32_t lf_pack_lo(uint32_t a, uint32_t b)
{
    return __builtin_amdgcn_perm(b, a, 0x05040100u);
}

// Bit position of the first group of values i0 .. i0 + 3 (i0 a multiple of
// 4) of a block with the given mode.
__device__ __forceinline__ uint32_t lf_bise_first(uint32_t mode, uint32_t i0)
{
    const uint32_t fam = mode >> 5, b = mode & 31u;
    const uint32_t hb = fam == 0u ? 0u : (fam == 1u ? 8u : 7u);
    const uint32_t gs = fam == 0u ? 1u : (fam == 1u ? 5u : 3u);
    const uint32_t mg = fam == 1u ? 858993460u : 1431655766u;  // ceil(2^32 / 5), ceil(2^32 / 3)
    const uint32_t g0 = fam == 0u ? i0 : __umulhi(i0, mg);
    return __umul24(g0, hb + gs * b);
}

// Values i0 .. i0 + 3 of a block (i0 a multiple of 4).  They lie in at most
// two groups (plain bits: four one-value groups).  w0, w1, w2 are the three
// payload words from word lf_bise_first(...) >> 5 on.  When the groups span
// at most 64 bits (always for b <= 4 bits per value, and for plain bits up
// to 16), the words are shifted so that the first group starts at bit 0 of
// one 64-bit word and every field is cut from it with one shift and mask;
// otherwise each value is read on its own from the block payload w.
__device__ __forceinline__ void lf_bise_quad(const uint32_t* __restrict__ w, uint32_t mode, uint32_t i0,
                                             const uint32_t* __restrict__ tab, uint32_t w0, uint32_t w1,
                                             uint32_t w2, uint32_t (&v)[4])
{
    const uint32_t fam = mode >> 5, b = mode & 31u;
    const uint32_t hb = fam == 0u ? 0u : (fam == 1u ? 8u : 7u);
    const uint32_t gs = fam == 0u ? 1u : (fam == 1u ? 5u : 3u);
    const uint32_t mg = fam == 1u ? 858993460u : 1431655766u;
    const uint32_t gl = hb + gs * b;  // bits per group
    const uint32_t g0 = fam == 0u ? i0 : __umulhi(i0, mg);
    const uint32_t pat = tab[LF_TAB_QUAD + 5u * fam + (i0 - __umul24(g0, gs))];
    const uint32_t o0 = __umul24(g0, gl) & 31u;
    const uint64_t X = ((uint64_t)__builtin_amdgcn_alignbit(w2, w1, o0) << 32) | __builtin_amdgcn_alignbit(w1, w0, o0);
    if (__umul24(((pat >> 15) & 3u) + 1u, gl) <= 64u) {  // end of the last value's group
        const uint32_t tb = fam == 2u ? 256u : 0u;
        const uint32_t hm = (1u << hb) - 1u, bm = (1u << b) - 1u;
        const uint32_t d0 = tab[tb + ((uint32_t)X & hm)];
        const uint32_t d1 = tab[tb + ((uint32_t)(X >> (gl & 63u)) & hm)];
#pragma unroll
        for (int k = 0; k < 4; k++) {
            const uint32_t dk = (pat >> (5 * k)) & 3u, kk = (pat >> (5 * k + 2)) & 7u;
            const uint32_t lo = (uint32_t)(X >> ((hb + __umul24(dk, gl) + __umul24(kk, b)) & 63u)) & bm;
            const uint32_t dig = dk != 0u ? d1 : d0;
            v[k] = (((dig >> (4u * kk)) & 15u) << b) | lo;
        }
    } else {
#pragma unroll
        for (int k = 0; k < 4; k++) v[k] = lf_bise_any(w, mode, i0 + (uint32_t)k, tab);
    }
}

// SRV values at (y, x0 .. x0 + 3) of the node a descriptor belongs to (x0 a
// multiple of 4, so the quad lies in one block: one descriptor, one motion
// vector, shared prediction taps and weights), as two int16 pairs
// (x = pixels 0, 1; y = pixels 2, 3).  The decode is split in two so that the
// loads of several quads are in flight together: lf_quad_fetch issues every
// load (payload window, two rows of prediction taps) unconditionally, and
// lf_quad_finish computes.  A reference node's descriptor (MODE_PLANE) reads
// its own plane, from `base` (resident reference planes, or the root planes
// for a root slot): the first tap row is then the quad itself.
struct QuadIn {
    uint32_t w0, w1, w2;              // payload words from the quad's first group
    uint32_t a0, a1, a2, b0, b1, b2;  // aligned words of tap rows y0, y0 + 1
};

__device__ __forceinline__ QuadIn lf_quad_fetch(const LfGeom& g, const LfPtrs& p, const int16_t* __restrict__ base,
                                                const uint4& d, int y, int x0)
{
    QuadIn in;
    const uint32_t mode = d.z >> 24;
    const bool plane = mode == MODE_PLANE;
    const uint32_t i0 = ((uint32_t)(y & (g.bs - 1)) << g.bsl) | (uint32_t)(x0 & (g.bs - 1));
    const uint32_t* q = p.payload + d.x + (plane ? 0u : lf_bise_first(mode, i0) >> 5);
    in.w0 = q[0];
    in.w1 = q[1];
    in.w2 = q[2];
    const int mx = ((int)(d.z << 20)) >> 20, my = ((int)(d.z << 8)) >> 20;
    const int xb = x0 + (mx >> 2), y0 = (4 * y + my) >> 2;
    // five taps from xb: the aligned words holding columns xs .. xs + 4, xs =
    // xb clamped into the row (a reference node: its own quad at x0)
    const int xs = plane ? x0 : max(min(xb, g.w - 5), 0);
    const uint32_t ea = d.w + (uint32_t)__mul24(lf_clampi(y0, 0, g.h - 1), g.w) + (uint32_t)xs;
    const uint32_t eb = d.w + (uint32_t)__mul24(lf_clampi(y0 + 1, 0, g.h - 1), g.w) + (uint32_t)xs;
    const uint32_t* ra = reinterpret_cast<const uint32_t*>(base) + (ea >> 1);
    const uint32_t* rb = reinterpret_cast<const uint32_t*>(base) + (eb >> 1);
    in.a0 = ra[0];
    in.a1 = ra[1];
    in.a2 = ra[2];
    in.b0 = rb[0];
    in.b1 = rb[1];
    in.b2 = rb[2];
    return in;
}

__device__ __forceinline__ uint2 lf_quad_finish(const LfGeom& g, const LfPtrs& p, const QuadIn& in, const uint4& d,
                                                int y, int x0, const uint32_t* __restrict__ digits)
{
    const uint32_t mode = d.z >> 24;
    if (mode == MODE_PLANE) return make_uint2(in.a0, in.a1);  // x0 is even: the words hold the quad
    const uint32_t i0 = ((uint32_t)(y & (g.bs - 1)) << g.bsl) | (uint32_t)(x0 & (g.bs - 1));
    uint32_t v[4];
    lf_bise_quad(p.payload + d.x, mode, i0, digits, in.w0, in.w1, in.w2, v);
    const lf_i16x2 mn = lf_splat((int)(int16_t)(d.y & 0xFFFFu));
    const lf_i16x2 step = lf_splat((int)((d.y >> 16) & 0x1FFFu));
    const lf_i16x2 r01 = (lf_as_i16x2(lf_pack_lo(v[0], v[1])) + mn) * step;
    const lf_i16x2 r23 = (lf_as_i16x2(lf_pack_lo(v[2], v[3])) + mn) * step;
    const uint32_t code = d.y >> 29;
    const int mx = ((int)(d.z << 20)) >> 20, my = ((int)(d.z << 8)) >> 20;
    const int xb = x0 + (mx >> 2), fx = mx & 3;
    const int Y = 4 * y + my, fy = Y & 3;
    const int xs = max(min(xb, g.w - 5), 0);
    const uint32_t sh = (uint32_t)(xs & 1) << 4;  // plane offsets and rows are even: the parity is xs's
    // pairs (t0,t1) (t1,t2) (t2,t3) (t3,t4) of each row
    uint32_t A[4], B[4];
    A[0] = __builtin_amdgcn_alignbit(in.a1, in.a0, sh);
    A[2] = __builtin_amdgcn_alignbit(in.a2, in.a1, sh);
    A[1] = __builtin_amdgcn_alignbit(A[2], A[0], 16);
    A[3] = __builtin_amdgcn_alignbit(in.a2 >> sh, A[2], 16);
    B[0] = __builtin_amdgcn_alignbit(in.b1, in.b0, sh);
    B[2] = __builtin_amdgcn_alignbit(in.b2, in.b1, sh);
    B[1] = __builtin_amdgcn_alignbit(B[2], B[0], 16);
    B[3] = __builtin_amdgcn_alignbit(in.b2 >> sh, B[2], 16);
    if (xs != xb) {
        // image border: tap c is column clamp(xb + c) = xs + k of the window
        uint32_t ta[5], tb[5];
#pragma unroll
        for (int c = 0; c < 5; c++) {
            const int k = lf_clampi(xb + c, 0, g.w - 1) - xs;  // 0 .. 4
            const uint32_t pa = k < 2 ? A[0] : A[2], pb = k < 2 ? B[0] : B[2];
            ta[c] = k == 4 ? A[3] >> 16 : (k & 1 ? pa >> 16 : pa & 0xFFFFu);
            tb[c] = k == 4 ? B[3] >> 16 : (k & 1 ? pb >> 16 : pb & 0xFFFFu);
        }
#pragma unroll
        for (int c = 0; c < 4; c++) {
            A[c] = ta[c] | (ta[c + 1] << 16);
            B[c] = tb[c] | (tb[c + 1] << 16);
        }
    }
    const lf_i16x2 wx0 = lf_splat(4 - fx), wx1 = lf_splat(fx), wy0 = lf_splat(4 - fy), wy1 = lf_splat(fy);
    const lf_i16x2 top01 = wx0 * lf_as_i16x2(A[0]) + wx1 * lf_as_i16x2(A[1]);
    const lf_i16x2 top23 = wx0 * lf_as_i16x2(A[2]) + wx1 * lf_as_i16x2(A[3]);
    const lf_i16x2 bot01 = wx0 * lf_as_i16x2(B[0]) + wx1 * lf_as_i16x2(B[1]);
    const lf_i16x2 bot23 = wx0 * lf_as_i16x2(B[2]) + wx1 * lf_as_i16x2(B[3]);
    const lf_i16x2 q01 = (wy0 * top01 + wy1 * bot01 + lf_splat(8)) >> lf_splat(4);
    const lf_i16x2 q23 = (wy0 * top23 + wy1 * bot23 + lf_splat(8)) >> lf_splat(4);
    const lf_i16x2 sg = lf_splat(code == 0u ? 1 : (code == 1u ? -1 : 0));  // phase sign; 0: no prediction
    return make_uint2(lf_as_u32(r01 + sg * q01), lf_as_u32(r23 + sg * q23));
}

// floor(n / d) for n, d < 2^16: m = ceil(2^32 / d) for d >= 2 (exact in that
// range); d = 1 would need m = 2^32, so it is encoded as m = 0 (identity)
__device__ __forceinline__ uint32_t lf_magic(uint32_t d)
{
    return d <= 1u ? 0u : 0xFFFFFFFFu / d + 1u;  // ceil(2^32 / d), also for powers of two
}
__device__ __forceinline__ int lf_qdiv(int n, uint32_t m) { return m ? (int)__umulhi((uint32_t)n, m) : n; }

// floor(n / d) for 0 <= n, 1 <= d, n * d < 2^20 (small node and block
// indices): (n + 1/2) / d is at least 1/(2d) away from an integer, and one
// rounded reciprocal and product are off by less than n * 2^-22.
__device__ __forceinline__ int lf_div_small(int n, int d)
{
    return (int)(((float)n + 0.5f) * __builtin_amdgcn_rcpf((float)d));
}

// Plan of one group of views: the footprint's pixel box, and per level l
// (0 = leaf views .. H = root) the bounding rectangle of the nodes the group
// reaches.  Decoded values stay in LDS across the groups of one call while
// the box stays the same: assembled leaf-view samples (RGBA8, one entry per
// view) and staged ancestor values (one entry per node, three channel
// planes) are kept in entries keyed by (level, node).  A group decodes only
// the leaf views some ray needs that no entry holds, and only the ancestors
// of those views that no entry holds ("new" nodes).
struct GroupPlan {
    int ok;
    int xq0, ymin, sy, nq, sxp, npix;  // quad-aligned rows: x from xq0, nq quads per row, stride sxp = 4 nq
    int bkx0, bky0, nbkx, nbk;
    int B0[LF_MAX_LEVELS + 1], A0[LF_MAX_LEVELS + 1], nA[LF_MAX_LEVELS + 1];
    int nnew[LF_MAX_LEVELS + 1];   // new nodes of each level
    int sbase[LF_MAX_LEVELS + 1];  // first new staged slot of each level (1..H); slot = sbase + 3 k + c
    int dbase[LF_MAX_LEVELS];      // first descriptor of each level (0..H-1); + (3 k + c) nbk + block
    int nslots, ndesc;
    uint32_t m_rowq, m_nq, m_nbk;  // reciprocals of sy * nq, nq and nbk
    uint32_t cbox0, cbox1;         // box the cache entries hold values of (all ones: none)
    int st_shared;                 // every view of the call has the same st homography
};

// Key of node (B, A) of level l (B, A < 2^14)
__device__ __forceinline__ uint32_t lf_node_key(int l, int B, int A)
{
    return ((uint32_t)l << 28) | ((uint32_t)B << 14) | (uint32_t)A;
}

#define FALLBACK_MARK 0x7FC0DEADu  // NaN payload: "this tile of this view needs per-ray decoding"

// LDS of one tile renderer instance.
struct TileLds {
    uint4* desc;       // [B_DESC]
    uint32_t* rgba;    // [B_RGBA]
    int16_t* sval;     // [B_SVAL]
    uint32_t (*fbox)[4];
    GroupPlan* gpp;
    int8_t (*nodemap)[LMAX];         // cache entry of each used node of the level rectangles, -1: unused
    uint16_t (*nodelist)[LMAX];      // k-th new node of a level: rectangle lane | entry << 8
    uint8_t (*ancs)[LF_MAX_LEVELS];  // per new leaf view: staged slot (channel 0) of its ancestor at level 1 + k
    uint32_t* slotinfo;              // per new staged slot: descriptor base, or root plane | 1 << 31
    uint8_t* slotdst;                // per new staged slot: destination slot (3 entry + channel)
    uint32_t (*ckey)[CMAX];          // cache keys: [0] leaf views, [1] ancestor nodes
    const uint32_t* digits;  // decode table (lf_fill_tab)
};

#define TILE_LDS_DECL                                                                            \
    extern __shared__ uint4 lds_dyn[];                                                           \
    __shared__ uint32_t fbox_s[FMAX][4];                                                         \
    __shared__ GroupPlan gp_s;                                                                   \
    __shared__ int8_t nodemap_s[LF_MAX_LEVELS + 1][LMAX];                                        \
    __shared__ uint16_t nodelist_s[LF_MAX_LEVELS + 1][LMAX];                                     \
    __shared__ __align__(8) uint8_t ancs_s[LMAX][LF_MAX_LEVELS];                                 \
    __shared__ uint32_t slotinfo_s[SLOT_MAX];                                                    \
    __shared__ uint8_t slotdst_s[SLOT_MAX];                                                      \
    __shared__ uint32_t ckey_s[2][CMAX];                                                         \
    __shared__ uint32_t digits_s[LF_TAB_SIZE];                                                   \
    const TileLds S{lds_dyn,                                                                     \
                    reinterpret_cast<uint32_t*>(lds_dyn + B_DESC),                               \
                    reinterpret_cast<int16_t*>(reinterpret_cast<uint32_t*>(lds_dyn + B_DESC) + B_RGBA), \
                    fbox_s, &gp_s, nodemap_s, nodelist_s, ancs_s, slotinfo_s, slotdst_s, ckey_s, digits_s};                 \
    lf_fill_tab(digits_s);                                                                       \
    __syncthreads();

// Render screen tile (txi, tyi) of views v0 .. v0 + nf - 1 (cameras cams[v],
// output out[v][3][ho][wo]; nf <= FMAX), in groups of at most gmax
// consecutive views.  A single view whose tile footprint exceeds the LDS
// budget is rendered ray by ray here (INLINE_FALLBACK) or left with
// FALLBACK_MARK at the tile origin for a per-ray pass; the return value says
// whether any view was left so (the same in every thread).  Every thread of
// the workgroup calls it; LDS contents do not carry over between calls.
// C420: a 4:2:0 stream (luma geometry g, p; chroma geometry gc, pc): the
// leaf samples are reconstructed one by one (luma walk, up-sampled chroma
// walks) into the same LDS sample cache, without descriptors or staged
// ancestors; the plan, the cache across groups and the blend are shared.
template <bool INLINE_FALLBACK, bool SMALL_BLOCKS = false, bool C420 = false>
__device__ bool lf_tile_views(const LfGeom& g, const LfPtrs& p, const LfGeom& gc, const LfPtrs& pc,
                              const float* __restrict__ cams, int v0, int nf, int gmax, int wo, int ho, int txi,
                              int tyi, float* __restrict__ out, const TileLds& S)
{
    // budgets of this instance (the dynamic LDS the launch reserved)
    constexpr int BD = SMALL_BLOCKS ? B_DESC_SB : B_DESC;
    constexpr int BR = SMALL_BLOCKS ? B_RGBA_SB : B_RGBA;
    constexpr int BSV = SMALL_BLOCKS ? B_SVAL_SB : B_SVAL;
    uint4* desc = S.desc;
    uint32_t* rgba = reinterpret_cast<uint32_t*>(S.desc + BD);
    int16_t* sval = reinterpret_cast<int16_t*>(rgba + BR);
    uint32_t* red = rgba;  // phase-0 reduction scratch [FMAX][4][NT/64], before any sample is staged
    uint32_t (*fbox)[4] = S.fbox;
    GroupPlan& gp = *S.gpp;
    int8_t (*nodemap)[LMAX] = S.nodemap;
    uint16_t (*nodelist)[LMAX] = S.nodelist;
    uint8_t (*ancs)[LF_MAX_LEVELS] = S.ancs;
    uint32_t* slotinfo = S.slotinfo;
    uint8_t* slotdst = S.slotdst;
    uint32_t (*ckey)[CMAX] = S.ckey;
    const uint32_t* digits = S.digits;
    // plan only: [0] leaf, [1] ancestor entries in order of their rank among
    // the free ones (the slot table's destinations are written after the plan)
    static_assert(SLOT_MAX >= 128, "the plan's rank tables alias the slot destinations");
    uint8_t (*inv)[64] = reinterpret_cast<uint8_t (*)[64]>(S.slotdst);
    const int lx = threadIdx.x % TW, ly = threadIdx.x / TW;
    const int i = txi * TW + lx, j = tyi * TH + ly;
    const bool live = i < wo && j < ho;
    const int ii = live ? i : txi * TW, jj = live ? j : tyi * TH;  // dead lanes repeat the tile origin
    const int wid = threadIdx.x >> 6, lane = threadIdx.x & 63;
    if (threadIdx.x == 0) gp.cbox0 = gp.cbox1 = CKEY_EMPTY;  // nothing cached yet
    // phase 0: footprint box of every view of the group (packed 16-bit
    // min/max of a0|b0<<16, a1|b1<<16, x0|y0<<16, x1|y1<<16).  For an affine
    // camera (third rows 0 0 1) each computed coordinate is, without
    // contraction, a product by a constant, a sum and a rounding of monotone
    // terms, so it is monotone in i for fixed j and in j for fixed i, and so
    // are the clamp and the floor: the four corner rays of the tile bound
    // every ray of it.  Four lanes per view compute them; a view whose camera
    // is not affine (or whose corner coordinates are not finite) reduces
    // over every pixel of the tile instead.
    if ((int)threadIdx.x < 4 * nf) {
        const int f = threadIdx.x >> 2, k = threadIdx.x & 3;
        const float* cam = cams + 18 * (v0 + f);
        const int ci = (k & 1) ? min(txi * TW + TW - 1, wo - 1) : txi * TW;
        const int cj = (k & 2) ? min(tyi * TH + TH - 1, ho - 1) : tyi * TH;
        float u, v, s, t;
        lf_ray(cam, ci, cj, u, v, s, t);
        Ray r;
        lf_axis(u, g.na, r.a0, r.a1, r.fu);
        lf_axis(v, g.nb, r.b0, r.b1, r.fv);
        lf_axis(s, g.w, r.x0, r.x1, r.fs);
        lf_axis(t, g.h, r.y0, r.y1, r.ft);
        const bool exact = cam[6] == 0.0f && cam[7] == 0.0f && cam[8] == 1.0f && cam[15] == 0.0f &&
                           cam[16] == 0.0f && cam[17] == 1.0f && __builtin_isfinite(u) && __builtin_isfinite(v) &&
                           __builtin_isfinite(s) && __builtin_isfinite(t);
        uint32_t m0 = (uint32_t)r.a0 | ((uint32_t)r.b0 << 16), m1 = (uint32_t)r.a1 | ((uint32_t)r.b1 << 16);
        uint32_t m2 = (uint32_t)r.x0 | ((uint32_t)r.y0 << 16), m3 = (uint32_t)r.x1 | ((uint32_t)r.y1 << 16);
        int all = exact;
#pragma unroll
        for (int o = 1; o < 4; o <<= 1) {
            m0 = pk_min(m0, (uint32_t)__shfl_xor((int)m0, o, 64));
            m1 = pk_max(m1, (uint32_t)__shfl_xor((int)m1, o, 64));
            m2 = pk_min(m2, (uint32_t)__shfl_xor((int)m2, o, 64));
            m3 = pk_max(m3, (uint32_t)__shfl_xor((int)m3, o, 64));
            all &= __shfl_xor(all, o, 64);
        }
        if (k == 0) {
            fbox[f][0] = all ? m0 : 0xFFFFFFFFu;  // all ones: not bounded by the corners
            fbox[f][1] = m1;
            fbox[f][2] = m2;
            fbox[f][3] = m3;
        }
    }
    if (wid == 0) {
        bool eq = true;
        if (lane < nf)
#pragma unroll
            for (int e = 0; e < 9; e++) eq = eq && cams[18 * (v0 + lane) + 9 + e] == cams[18 * v0 + 9 + e];
        const bool shared = __ballot(lane < nf && !eq) == 0ull;
        if (lane == 0) gp.st_shared = shared;
    }
    __syncthreads();
    for (int f = 0; f < nf; f++) {
        if (fbox[f][0] != 0xFFFFFFFFu) continue;  // uniform
        const Ray r = lf_ray_setup(g, cams + 18 * (v0 + f), ii, jj);
        const uint32_t m0 = wave_pk_min((uint32_t)r.a0 | ((uint32_t)r.b0 << 16));
        const uint32_t m1 = wave_pk_max((uint32_t)r.a1 | ((uint32_t)r.b1 << 16));
        const uint32_t m2 = wave_pk_min((uint32_t)r.x0 | ((uint32_t)r.y0 << 16));
        const uint32_t m3 = wave_pk_max((uint32_t)r.x1 | ((uint32_t)r.y1 << 16));
        if (lane == 0) {
            red[0 * (NT / 64) + wid] = m0;
            red[1 * (NT / 64) + wid] = m1;
            red[2 * (NT / 64) + wid] = m2;
            red[3 * (NT / 64) + wid] = m3;
        }
        __syncthreads();
        if (threadIdx.x < 4) {
            const int k = threadIdx.x;
            uint32_t v = red[k * (NT / 64)];
#pragma unroll
            for (int w = 1; w < NT / 64; w++) v = (k & 1) ? pk_max(v, red[k * (NT / 64) + w]) : pk_min(v, red[k * (NT / 64) + w]);
            fbox[f][k] = v;
        }
        __syncthreads();
    }

    const int64_t npix_out = (int64_t)wo * ho;
    bool left = false;
    // group sizes: after a success the next group doubles, but stays below
    // the smallest size that failed; that ceiling rises by one every four
    // successes in a row
    int f = 0, n = GROUP_FIRST(gmax), ceil_n = gmax + 1, streak = 0;
    while (f < nf) {
        n = min(n, nf - f);
        // plan the group [f, f + n) (wave 0); a plan that fails stops at the
        // first check that fails
        if (wid == 0) {
            int ok = 0;
            __builtin_amdgcn_s_setprio(3);  // the plan holds up the workgroup: issue it first
            do {
            uint32_t lo_ab = 0xFFFFFFFFu, hi_ab = 0u, lo_xy = 0xFFFFFFFFu, hi_xy = 0u;
            for (int q = f; q < f + n; q++) {
                lo_ab = pk_min(lo_ab, fbox[q][0]);
                hi_ab = pk_max(hi_ab, fbox[q][1]);
                lo_xy = pk_min(lo_xy, fbox[q][2]);
                hi_xy = pk_max(hi_xy, fbox[q][3]);
            }
            // the box is the same in every lane: scalar from here on
            lo_ab = (uint32_t)__builtin_amdgcn_readfirstlane((int)lo_ab);
            hi_ab = (uint32_t)__builtin_amdgcn_readfirstlane((int)hi_ab);
            lo_xy = (uint32_t)__builtin_amdgcn_readfirstlane((int)lo_xy);
            hi_xy = (uint32_t)__builtin_amdgcn_readfirstlane((int)hi_xy);
            const int amin = (int)(lo_ab & 0xFFFFu), bmin = (int)(lo_ab >> 16);
            const int amax = (int)(hi_ab & 0xFFFFu), bmax = (int)(hi_ab >> 16);
            const int xmin = (int)(lo_xy & 0xFFFFu), ymin = (int)(lo_xy >> 16);
            const int xmax = (int)(hi_xy & 0xFFFFu), ymax = (int)(hi_xy >> 16);
            const int xq0 = xmin & ~3, nq = (xmax >> 2) - (xmin >> 2) + 1, sxp = 4 * nq;
            const int sy = ymax - ymin + 1, npix = sxp * sy;
            const int bkx0 = xmin >> g.bsl, bky0 = ymin >> g.bsl;
            const int nbkx = (xmax >> g.bsl) - bkx0 + 1, nbk = nbkx * ((ymax >> g.bsl) - bky0 + 1);
            const uint32_t bx0 = (uint32_t)xq0 | ((uint32_t)ymin << 16), bx1 = (uint32_t)nq | ((uint32_t)sy << 16);
            const bool same = (uint32_t)__builtin_amdgcn_readfirstlane((int)gp.cbox0) == bx0 &&
                              (uint32_t)__builtin_amdgcn_readfirstlane((int)gp.cbox1) == bx1;  // cached entries hold this box
            const int cap0 = min(CMAX, BR / npix), cap1 = min(CMAX, BSV / (3 * npix));
            const int nA0 = amax - amin + 1, nB0 = bmax - bmin + 1;
            ok = nA0 * nB0 <= LMAX && npix <= BR;
            if (!ok) break;
            // node maps start empty; cache entries that a node of this group
            // keeps write their index into the node's map (entry side), and
            // each node then reads its map (node side; same wave, LDS in order)
#pragma unroll
            for (int l = 0; l <= LF_MAX_LEVELS; l++)
                if (l <= g.H) nodemap[l][lane] = -1;
            // level 0: leaf views some ray of the group reaches
            bool use0 = false;
            if (ok && lane < nA0 * nB0) {
                const int qb = lf_div_small(lane, nA0), b = bmin + qb, a = amin + lane - qb * nA0;
                for (int q = f; q < f + n && !use0; q++) {
                    const uint32_t q0 = fbox[q][0], q1 = fbox[q][1];
                    use0 = (int)(q0 >> 16) <= b && (int)(q1 >> 16) >= b && (int)(q0 & 0xFFFFu) <= a &&
                           (int)(q1 & 0xFFFFu) >= a;
                }
            }
            const uint64_t used0 = __ballot(use0);
            const uint32_t key0 = same && lane < cap0 ? ckey[0][lane] : CKEY_EMPTY;
            const uint32_t key1 = same && lane < cap1 ? ckey[1][lane] : CKEY_EMPTY;
            bool keep = false;
            if (key0 != CKEY_EMPTY) {
                const int b = (int)((key0 >> 14) & 0x3FFFu) - bmin, a = (int)(key0 & 0x3FFFu) - amin;
                keep = ok && b >= 0 && b < nB0 && a >= 0 && a < nA0 && ((used0 >> (b * nA0 + a)) & 1ull);
                if (keep) nodemap[0][b * nA0 + a] = (int8_t)lane;
            }
            const uint64_t free0 = ~__ballot(keep) & (cap0 >= 64 ? ~0ull : ((1ull << cap0) - 1ull));
            __atomic_signal_fence(__ATOMIC_SEQ_CST);
            int ent0 = nodemap[0][lane];
            const bool new0 = use0 && ent0 < 0;
            const uint64_t newm0 = __ballot(new0);
            const int nnew0 = __popcll(newm0);
            ok = ok && nnew0 <= __popcll(free0);
            if (!ok) break;
            // the k-th new leaf view takes the k-th free entry
            if ((free0 >> lane) & 1ull) inv[0][__popcll(free0 & ((1ull << lane) - 1ull))] = (uint8_t)lane;
            __atomic_signal_fence(__ATOMIC_SEQ_CST);
            if (new0) ent0 = inv[0][__popcll(newm0 & ((1ull << lane) - 1ull))];
            // levels 1..H: ancestors of the new leaf views.  A node (B, A) of
            // level l covers leaf rows [B << l, (B + 1) << l) and columns
            // [A << l, (A + 1) << l); it is needed when one of the new leaf
            // views lies there.
            const int kl = key1 != CKEY_EMPTY ? (int)(key1 >> 28) : 0;
            bool kneed = false;
            if (kl >= 1 && kl <= g.H) {
                const int B = (int)((key1 >> 14) & 0x3FFFu), A = (int)(key1 & 0x3FFFu);
                if (B >= (bmin >> kl) && B <= (bmax >> kl) && A >= (amin >> kl) && A <= (amax >> kl)) {
                    const int rb0 = max(B << kl, bmin) - bmin, rb1 = min(((B + 1) << kl) - 1, bmax) - bmin;
                    const int ra0 = max(A << kl, amin) - amin, ra1 = min(((A + 1) << kl) - 1, amax) - amin;
                    for (int r = rb0; r <= rb1 && !kneed; r++)
                        kneed = ((newm0 >> (r * nA0 + ra0)) & ((2ull << (ra1 - ra0)) - 1ull)) != 0ull;
                    const int nA = (amax >> kl) - (amin >> kl) + 1;
                    const int el = (B - (bmin >> kl)) * nA + (A - (amin >> kl));
                    kneed = kneed && el < LMAX;
                    if (kneed) nodemap[kl][el] = (int8_t)lane;
                }
            }
            const uint64_t keep1 = __ballot(kneed);
            __atomic_signal_fence(__ATOMIC_SEQ_CST);
            int nd = C420 ? 0 : 3 * nbk * nnew0;
            int cnt[LF_MAX_LEVELS + 1];
            cnt[0] = nnew0;
            const uint64_t free1 = ~keep1 & (cap1 >= 64 ? ~0ull : ((1ull << cap1) - 1ull));
            ok = ok && nd <= BD;
            if (!ok) break;
            // Levels 1..H at once: the level rectangles laid end to end (level
            // 1 first), node t of the concatenation in lane t % 64 of pass t / 64.
            // Their total stays below 128: level l holds at most
            // (nB0 / 2^l + 1)(nA0 / 2^l + 1) nodes and nA0 nB0 <= 64.
            int off[LF_MAX_LEVELS + 2];
            int total = 0;
#pragma unroll
            for (int l = 1; l <= LF_MAX_LEVELS + 1; l++) {
                off[l] = total;
                if (!C420 && l <= g.H) {  // a 4:2:0 group stages no ancestors
                    const int nBl = (bmax >> l) - (bmin >> l) + 1, nAl = (amax >> l) - (amin >> l) + 1;
                    if (nBl * nAl > LMAX) ok = 0;
                    total += nBl * nAl;
                }
            }
            ok = ok && total <= 128;
            if (!ok) break;
            bool newp[2];
            int lvp[2], idxp[2];
            uint64_t nmp[2];
#pragma unroll
            for (int pp = 0; pp < 2; pp++) {
                const int t = 64 * pp + lane;
                newp[pp] = false;
                lvp[pp] = 1;
                idxp[pp] = 0;
                if (t < total) {
                    // level of node t and its place in that level's rectangle
                    int l = 1, base = 0;
#pragma unroll
                    for (int k = 2; k <= LF_MAX_LEVELS; k++)
                        if (k <= g.H && t >= off[k]) {
                            l = k;
                            base = off[k];
                        }
                    const int B0 = bmin >> l, A0 = amin >> l, nA = (amax >> l) - A0 + 1;
                    const int e = t - base;
                    const int qb = lf_div_small(e, nA), B = B0 + qb, A = A0 + e - qb * nA;
                    // A node (B, A) of level l covers leaf rows [B << l, (B + 1) << l)
                    // and columns [A << l, (A + 1) << l); it is needed when one of the
                    // new leaf views lies there.
                    const int rb0 = max(B << l, bmin) - bmin, rb1 = min(((B + 1) << l) - 1, bmax) - bmin;
                    const int ra0 = max(A << l, amin) - amin, ra1 = min(((A + 1) << l) - 1, amax) - amin;
                    bool need = false;
                    for (int r = rb0; r <= rb1 && !need; r++)
                        need = ((newm0 >> (r * nA0 + ra0)) & ((2ull << (ra1 - ra0)) - 1ull)) != 0ull;
                    newp[pp] = need && nodemap[l][e] < 0;
                    lvp[pp] = l;
                    idxp[pp] = e;
                }
                nmp[pp] = __ballot(newp[pp]);
            }
            // new nodes per level: the set bits of each level's segment
            int nnew1 = 0;
#pragma unroll
            for (int l = 1; l <= LF_MAX_LEVELS; l++) {
                cnt[l] = 0;
                if (l > g.H) continue;
#pragma unroll
                for (int pp = 0; pp < 2; pp++) {
                    const int lo = min(max(off[l] - 64 * pp, 0), 64), hi = min(max(off[l + 1] - 64 * pp, 0), 64);
                    const uint64_t m = (hi >= 64 ? ~0ull : ((1ull << hi) - 1ull)) & ~(lo >= 64 ? ~0ull : ((1ull << lo) - 1ull));
                    cnt[l] += __popcll(nmp[pp] & m);
                }
                nnew1 += cnt[l];
                if (l < g.H) nd += 3 * nbk * cnt[l];
            }
            const int ns = 3 * nnew1;
            ok = ok && nnew1 <= __popcll(free1) && nd <= BD && ns <= SLOT_MAX;
            if (!ok) break;
            if ((free1 >> lane) & 1ull) inv[1][__popcll(free1 & ((1ull << lane) - 1ull))] = (uint8_t)lane;
            __atomic_signal_fence(__ATOMIC_SEQ_CST);
            {
                // commit: entries of the new nodes, node maps, new-node lists, keys
                if (!same && lane < CMAX) {
                    ckey[0][lane] = CKEY_EMPTY;
                    ckey[1][lane] = CKEY_EMPTY;
                }
                if (new0) {
                    nodemap[0][lane] = (int8_t)ent0;
                    const int k = __popcll(newm0 & ((1ull << lane) - 1ull));
                    nodelist[0][k] = (uint16_t)(lane | (ent0 << 8));
                    const int qb = lf_div_small(lane, nA0);
                    ckey[0][ent0] = lf_node_key(0, bmin + qb, amin + lane - qb * nA0);
                }
                // a new node's entry is the r-th free one, r its rank among the
                // new nodes of all levels (level order); its list index is r less
                // the new nodes of the levels before
#pragma unroll
                for (int pp = 0; pp < 2; pp++) {
                    if (newp[pp]) {
                        const int r = (pp ? __popcll(nmp[0]) : 0) + __popcll(nmp[pp] & ((1ull << lane) - 1ull));
                        const int e = inv[1][r];
                        int before = 0;
#pragma unroll
                        for (int k = 1; k < LF_MAX_LEVELS; k++)
                            if (k < lvp[pp]) before += cnt[k];
                        const int l = lvp[pp], nA = (amax >> l) - (amin >> l) + 1;
                        const int qb = lf_div_small(idxp[pp], nA);
                        nodelist[l][r - before] = (uint16_t)(idxp[pp] | (e << 8));
                        ckey[1][e] = lf_node_key(l, (bmin >> l) + qb, (amin >> l) + idxp[pp] - qb * nA);
                        nodemap[lvp[pp]][idxp[pp]] = (int8_t)e;
                    }
                }
            }
            if (lane <= g.H) {
                // per-level fields, lane l for level l: the level's rectangle,
                // its new nodes, and the first staged slot (levels 1..H) and
                // descriptor (levels 0..H-1) of its new nodes
                const int l = lane;
                int cl = 0, s3 = 0, d3 = 0;
#pragma unroll
                for (int k = 0; k <= LF_MAX_LEVELS; k++) {
                    if (k == l) cl = cnt[k];
                    if (k >= 1 && k < l) s3 += 3 * cnt[k];
                    if (k < l) d3 += 3 * nbk * cnt[k];
                }
                gp.B0[l] = bmin >> l;
                gp.A0[l] = amin >> l;
                gp.nA[l] = (amax >> l) - (amin >> l) + 1;
                gp.nnew[l] = cl;
                if (l >= 1) gp.sbase[l] = s3;
                if (l < g.H) gp.dbase[l] = d3;
            }
            if (lane == 0) {
                gp.ok = ok;
                if (ok) {
                    gp.xq0 = xq0;
                    gp.ymin = ymin;
                    gp.sy = sy;
                    gp.nq = nq;
                    gp.sxp = sxp;
                    gp.npix = npix;
                    gp.bkx0 = bkx0;
                    gp.bky0 = bky0;
                    gp.nbkx = nbkx;
                    gp.nbk = nbk;
                    gp.nslots = ns;
                    gp.ndesc = nd;
                    gp.m_rowq = lf_magic((uint32_t)(sy * nq));
                    gp.m_nq = lf_magic((uint32_t)nq);
                    gp.m_nbk = lf_magic((uint32_t)nbk);
                    gp.cbox0 = bx0;
                    gp.cbox1 = bx1;
                }
            }
            } while (false);
            if (!ok && lane == 0) gp.ok = 0;
            __builtin_amdgcn_s_setprio(0);
        }
        __syncthreads();
        // the plan's fields are the same in every lane: read into scalar
        // registers, so the group loop's control and the phases' uniform
        // index arithmetic stay on the scalar unit
        if (!__builtin_amdgcn_readfirstlane(gp.ok)) {
            if (n > 1) {
                if (n <= 4) ceil_n = n;  // views far apart: stop doubling into failures
                streak = 0;
                n = (n + 1) / 2;  // try half the group
                __syncthreads();
                continue;
            }
            if (INLINE_FALLBACK) {
                // one view whose footprint exceeds the budget: per-ray decoding here
                float o[3];
                lf_render_one(g, p, cams + 18 * (v0 + f), ii, jj, o);
                if (live)
#pragma unroll
                    for (int c = 0; c < 3; c++) out[((int64_t)(v0 + f) * 3 + c) * npix_out + (int64_t)j * wo + i] = o[c];
            } else {
                // one view whose footprint exceeds the budget: leave a marker for the per-ray pass
                left = true;
                if (threadIdx.x == 0)
                    out[((int64_t)(v0 + f) * 3) * npix_out + (int64_t)(tyi * TH) * wo + txi * TW] =
                        __uint_as_float(FALLBACK_MARK);
            }
            f += 1;
            n = 1;  // the next group starts small again (below)
            __syncthreads();
            continue;
        }
#define LF_UNI(x) __builtin_amdgcn_readfirstlane(x)
        const int npix = LF_UNI(gp.npix), sxp = LF_UNI(gp.sxp), nq = LF_UNI(gp.nq), nbk = LF_UNI(gp.nbk),
                  nbkx = LF_UNI(gp.nbkx);
        const int xq0 = LF_UNI(gp.xq0), ymin = LF_UNI(gp.ymin), bkx0 = LF_UNI(gp.bkx0), bky0 = LF_UNI(gp.bky0);
        const int rowq = LF_UNI(gp.sy) * nq;  // quads per staged plane
        const uint32_t m_rowq = (uint32_t)LF_UNI((int)gp.m_rowq), m_nq = (uint32_t)LF_UNI((int)gp.m_nq),
                       m_nbk = (uint32_t)LF_UNI((int)gp.m_nbk);
        const int ndesc = LF_UNI(gp.ndesc), nslots = LF_UNI(gp.nslots), nnew0 = LF_UNI(gp.nnew[0]);
        const int B00 = LF_UNI(gp.B0[0]), A00 = LF_UNI(gp.A0[0]), nA0 = LF_UNI(gp.nA[0]);
#undef LF_UNI
        // phase 1a: block descriptors of the new nodes of levels 0..H-1, the
        // slot table of the new staged values (levels 1..H), and the
        // ancestor slots of the new leaf views
        for (int d = threadIdx.x; d < ndesc; d += NT) {
            int l = 0;
            while (l + 1 < g.H && d >= gp.dbase[l + 1]) l++;
            const int row = lf_qdiv(d - gp.dbase[l], m_nbk);  // 3 k + c
            const int kb = d - gp.dbase[l] - row * nbk;
            const int k = row / 3, c = row - 3 * k;
            const int e = nodelist[l][k] & 0xFF;
            const int qb = lf_div_small(e, gp.nA[l]), B = gp.B0[l] + qb, A = gp.A0[l] + e - qb * gp.nA[l];
            const int qk = lf_div_small(kb, nbkx), blk = (bky0 + qk) * g.nbx + bkx0 + kb - qk * nbkx;
            const int node = g.node_base[l] + B * g.na_l[l] + A;
            desc[d] = p.desc[((size_t)c * g.n_nodes + node) * g.nblk + blk];
        }
        for (int sl = threadIdx.x; sl < nslots; sl += NT) {
            int l = 1;
            while (l < g.H && sl >= gp.sbase[l + 1]) l++;
            const int row = sl - gp.sbase[l];  // 3 k + c
            const int k = row / 3, c = row - 3 * k;
            const uint32_t nl = nodelist[l][k];
            uint32_t info;
            if (l == g.H) {
                const int e = nl & 0xFF;
                const int qb = lf_div_small(e, gp.nA[l]), B = gp.B0[l] + qb, A = gp.A0[l] + e - qb * gp.nA[l];
                info = 0x80000000u | (uint32_t)((c * g.root_nb + B) * g.root_na + A);
            } else {
                info = (uint32_t)(gp.dbase[l] + row * nbk);
            }
            slotinfo[sl] = info;
            slotdst[sl] = (uint8_t)(3 * (nl >> 8) + c);
        }
        for (int k = threadIdx.x; k < (C420 ? 0 : nnew0); k += NT) {
            const int e = nodelist[0][k] & 0xFF;
            const int qb = lf_div_small(e, nA0), b = B00 + qb, a = A00 + e - qb * nA0;
            for (int l = 1; l <= g.H; l++) {
                const int el = __mul24((b >> l) - gp.B0[l], gp.nA[l]) + ((a >> l) - gp.A0[l]);
                ancs[k][l - 1] = (uint8_t)(3 * nodemap[l][el]);
            }
        }
        __syncthreads();
        // phase 1b: new values shared by several views, once per node and pixel
        // quad: SRVs of levels 1..H-1 and the root RKV (level H).  Four quads
        // per thread at a time: all their loads are issued before any is used.
        {
            const int n1b = nslots * rowq;
            const uint32_t plane = (uint32_t)(g.w * g.h);
            for (int it0 = threadIdx.x; it0 < n1b; it0 += 4 * NT) {
                QuadIn in[4];
                int yy[4], xx[4], sl4[4];
#pragma unroll
                for (int u = 0; u < 4; u++) {
                    const int it = min(it0 + u * NT, n1b - 1);  // past the end: repeat the last quad, not stored
                    const int sl = lf_qdiv(it, m_rowq), rq = it - sl * rowq;
                    const int yl = lf_qdiv(rq, m_nq), qi = rq - yl * nq;
                    const int y = ymin + yl, x0 = xq0 + 4 * qi;
                    const uint32_t info = slotinfo[sl];
                    const bool root = info & 0x80000000u;
                    const int kb = __mul24((y >> g.bsl) - bky0, nbkx) + (x0 >> g.bsl) - bkx0;
                    const uint4 d = root ? make_uint4(0u, 0u, (uint32_t)MODE_PLANE << 24, (info & 0x7FFFFFFFu) * plane)
                                         : desc[info + kb];
                    in[u] = lf_quad_fetch(g, p, root ? p.root : p.refs, d, y, x0);
                    yy[u] = y;
                    xx[u] = x0;
                    sl4[u] = sl;
                }
#pragma unroll
                for (int u = 0; u < 4; u++) {
                    const int it = it0 + u * NT;
                    if (it < n1b) {
                        const int sl = sl4[u], rq = it - sl * rowq;
                        const uint32_t info = slotinfo[sl];
                        const bool root = info & 0x80000000u;
                        const int kb = __mul24((yy[u] >> g.bsl) - bky0, nbkx) + (xx[u] >> g.bsl) - bkx0;
                        const uint4 d = root ? make_uint4(0u, 0u, (uint32_t)MODE_PLANE << 24, 0u) : desc[info + kb];
                        reinterpret_cast<uint2*>(sval)[__mul24((int)slotdst[sl], rowq) + rq] =
                            lf_quad_finish(g, p, in[u], d, yy[u], xx[u], digits);
                    }
                }
            }
        }
        __syncthreads();
        // phase 2: every new (view, pixel quad) sample: level-0 SRV + staged
        // ancestors and root; two quads (six channel decodes) per thread at a time
        const int n2 = nnew0 * rowq;
        if (C420) {
            // 4:2:0: each sample of the quad from the luma walk and the
            // up-sampled chroma walks, inverse YCoCg-R, RGBA8
            for (int it = threadIdx.x; it < n2; it += NT) {
                const int k = lf_qdiv(it, m_rowq), rq = it - k * rowq;
                const int yl = lf_qdiv(rq, m_nq), qi = rq - yl * nq;
                const int y = ymin + yl, x0 = xq0 + 4 * qi;
                const uint32_t nl = nodelist[0][k];
                const int e = nl & 0xFF;
                const int qb = lf_div_small(e, nA0), b = B00 + qb, a = A00 + e - qb * nA0;
                uint32_t px[4];
#pragma unroll 1
                for (int t = 0; t < 4; t++) {
                    int R, G, B;
                    lf_ycocg_to_rgb(lf_decode_channel(g, p, 0, b, a, y, x0 + t), lf_chroma_up(gc, pc, 0, b, a, y, x0 + t),
                                    lf_chroma_up(gc, pc, 1, b, a, y, x0 + t), R, G, B);
                    px[t] = (uint32_t)R | ((uint32_t)G << 8) | ((uint32_t)B << 16);
                }
                reinterpret_cast<uint4*>(rgba)[__mul24((int)(nl >> 8), rowq) + rq] = make_uint4(px[0], px[1], px[2], px[3]);
            }
        }
        for (int it0 = threadIdx.x; it0 < (C420 ? 0 : n2); it0 += 2 * NT) {
            QuadIn in[2][3];
            int kk2[2], rq2[2], yy[2], xx[2];
#pragma unroll
            for (int u = 0; u < 2; u++) {
                const int it = min(it0 + u * NT, n2 - 1);
                const int k = lf_qdiv(it, m_rowq), rq = it - k * rowq;
                const int yl = lf_qdiv(rq, m_nq), qi = rq - yl * nq;
                const int y = ymin + yl, x0 = xq0 + 4 * qi;
                const int kb = __mul24((y >> g.bsl) - bky0, nbkx) + (x0 >> g.bsl) - bkx0;
                const uint4* dq = desc + __mul24(3 * k, nbk) + kb;
#pragma unroll
                for (int c = 0; c < 3; c++) in[u][c] = lf_quad_fetch(g, p, p.refs, dq[c * nbk], y, x0);
                kk2[u] = k;
                rq2[u] = rq;
                yy[u] = y;
                xx[u] = x0;
            }
#pragma unroll
            for (int u = 0; u < 2; u++) {
            if (it0 + u * NT >= n2) continue;
            const int k = kk2[u], rq = rq2[u], y = yy[u], x0 = xx[u];
            const int kb = __mul24((y >> g.bsl) - bky0, nbkx) + (x0 >> g.bsl) - bkx0;
            const uint4* dq = desc + __mul24(3 * k, nbk) + kb;
            lf_i16x2 ch[3][2];
#pragma unroll
            for (int c = 0; c < 3; c++) {
                const uint2 q = lf_quad_finish(g, p, in[u][c], dq[c * nbk], y, x0, digits);
                ch[c][0] = lf_as_i16x2(q.x);
                ch[c][1] = lf_as_i16x2(q.y);
            }
            const uint2 an = *reinterpret_cast<const uint2*>(ancs[k]);
            for (int l = 1; l <= g.H; l++) {
                const uint32_t sl = ((l <= 4 ? an.x : an.y) >> (8 * ((l - 1) & 3))) & 0xFFu;
                const uint2* sv = reinterpret_cast<const uint2*>(sval) + __mul24(sl, rowq) + rq;
#pragma unroll
                for (int c = 0; c < 3; c++) {
                    const uint2 s4 = sv[c * rowq];
                    ch[c][0] += lf_as_i16x2(s4.x);
                    ch[c][1] += lf_as_i16x2(s4.y);
                }
            }
            // inverse YCoCg-R on pixel pairs, clamped to [0, 255], packed as RGBA8
            uint4 px4;
#pragma unroll
            for (int h = 0; h < 2; h++) {
                const lf_i16x2 Yv = ch[0][h], Co = ch[1][h], Cg = ch[2][h];
                const lf_i16x2 t = Yv - (Cg >> lf_splat(1));
                const lf_i16x2 G = Cg + t;
                const lf_i16x2 Bv = t - (Co >> lf_splat(1));
                const lf_i16x2 R = Bv + Co;
                const lf_i16x2 z = lf_splat(0), m = lf_splat(255);
                const uint32_t r2 = lf_as_u32(__builtin_elementwise_min(__builtin_elementwise_max(R, z), m));
                const uint32_t g2 = lf_as_u32(__builtin_elementwise_min(__builtin_elementwise_max(G, z), m));
                const uint32_t b2 = lf_as_u32(__builtin_elementwise_min(__builtin_elementwise_max(Bv, z), m));
                const uint32_t rg = r2 | (g2 << 8);  // bytes R0 G0 R1 G1
                // pixel 2h: R0 G0 B0 0; pixel 2h+1: R1 G1 B1 0
                const uint32_t p0 = __builtin_amdgcn_perm(b2, rg, 0x0C040100u);
                const uint32_t p1 = __builtin_amdgcn_perm(b2, rg, 0x0C060302u);
                if (h == 0) {
                    px4.x = p0;
                    px4.y = p1;
                } else {
                    px4.z = p0;
                    px4.w = p1;
                }
            }
            reinterpret_cast<uint4*>(rgba)[__mul24((int)(nodelist[0][k] >> 8), rowq) + rq] = px4;
            }
        }
        __syncthreads();
        // phase 3: blend every ray of the group's views: with one shared (s, t)
        // axis view by view, reusing per-view (s, t) sums; otherwise two views
        // at a time (the second view's sample reads in flight during the
        // first's blend)
        {
            // all views of the call share one st homography (a camera path with
            // one st window): each ray's (s, t) axis is computed once
            const bool st_shared = __builtin_amdgcn_readfirstlane(gp.st_shared) != 0;
            const float* hst = cams + 18 * v0 + 9;
            Ray rst;
            {
                float s, t;
                lf_ray_h(hst, (float)ii + 0.5f, (float)jj + 0.5f, s, t);
                lf_axis(s, g.w, rst.x0, rst.x1, rst.fs);
                lf_axis(t, g.h, rst.y0, rst.y1, rst.ft);
            }
            if (st_shared) {
                // Every view of the call has this pixel's (s, t) axis, so a
                // neighbouring light-field view's (s, t) bilinear sum depends only
                // on the 2x2 block of views (b0, a0) the ray reaches.  Each thread
                // keeps the four sums of its last block; a view reaching the same
                // block reuses them when every lane of the wave does, otherwise
                // the wave recomputes them.  Same operations, in the same order,
                // as lf_blend16.
                const float gs = 1.0f - rst.fs, gt = 1.0f - rst.ft;
                const float wst0 = gs * gt, wst1 = rst.fs * gt, wst2 = gs * rst.ft, wst3 = rst.fs * rst.ft;
                const int pix = __mul24(rst.y0 - ymin, sxp) + (rst.x0 - xq0);
                uint32_t ckey = 0xFFFFFFFFu;
                float tc[4][3];
                for (int q = f; q < f + n; q++) {
                    float u, v;
                    lf_ray_h(cams + 18 * (v0 + q), (float)ii + 0.5f, (float)jj + 0.5f, u, v);
                    int a0, a1, b0, b1;
                    float fu, fv;
                    lf_axis(u, g.na, a0, a1, fu);
                    lf_axis(v, g.nb, b0, b1, fv);
                    const uint32_t key = ((uint32_t)b0 << 16) | (uint32_t)a0;
                    if (__ballot(key != ckey) != 0ull) {  // uniform
#pragma unroll
                        for (int k = 0; k < 4; k++) {
                            const int b = (k & 2) ? b1 : b0, a = (k & 1) ? a1 : a0;
                            const uint32_t* q0 =
                                rgba + __mul24(nodemap[0][__mul24(b - B00, nA0) + (a - A00)], npix) + pix;
                            const uint32_t* q1 = q0 + sxp;
                            const uint32_t s0 = q0[0], s1 = q0[1], s2 = q1[0], s3 = q1[1];
#pragma unroll
                            for (int c = 0; c < 3; c++) {
                                float t = (float)((s0 >> (8 * c)) & 255u) * wst0;
                                t = fmaf((float)((s1 >> (8 * c)) & 255u), wst1, t);
                                t = fmaf((float)((s2 >> (8 * c)) & 255u), wst2, t);
                                tc[k][c] = fmaf((float)((s3 >> (8 * c)) & 255u), wst3, t);
                            }
                        }
                        ckey = key;
                    }
                    if (live) {
                        const float gu = 1.0f - fu, gv = 1.0f - fv;
                        const float uv0 = gu * gv, uv1 = fu * gv, uv2 = gu * fv, uv3 = fu * fv;
#pragma unroll
                        for (int c = 0; c < 3; c++) {
                            float acc = tc[0][c] * uv0;
                            acc = fmaf(tc[1][c], uv1, acc);
                            acc = fmaf(tc[2][c], uv2, acc);
                            acc = fmaf(tc[3][c], uv3, acc);
                            // written once, never read here: streaming stores keep L2 for the stream
                            __builtin_nontemporal_store(acc * (1.0f / 255.0f),
                                                        &out[((int64_t)(v0 + q) * 3 + c) * npix_out + (int64_t)j * wo + i]);
                        }
                    }
                }
            } else
            for (int q = f; q < f + n; q += 2) {
                const bool two = q + 1 < f + n;  // uniform
                Ray r[2];
                uint32_t s16[2][16];
#pragma unroll
                for (int h = 0; h < 2; h++) {
                    const int qq = (h == 1 && two) ? q + 1 : q;  // odd tail: repeat view q, not stored
                    if (st_shared) {
                        float u, v;
                        lf_ray_h(cams + 18 * (v0 + qq), (float)ii + 0.5f, (float)jj + 0.5f, u, v);
                        lf_axis(u, g.na, r[h].a0, r[h].a1, r[h].fu);
                        lf_axis(v, g.nb, r[h].b0, r[h].b1, r[h].fv);
                        r[h].x0 = rst.x0;
                        r[h].x1 = rst.x1;
                        r[h].y0 = rst.y0;
                        r[h].y1 = rst.y1;
                        r[h].fs = rst.fs;
                        r[h].ft = rst.ft;
                    } else {
                        r[h] = lf_ray_setup(g, cams + 18 * (v0 + qq), ii, jj);
                    }
                    // x1 = x0 + 1 and y1 = y0 + 1: the captured views are at least one
                    // 4-pixel block wide and high on this path
                    const int pix = __mul24(r[h].y0 - ymin, sxp) + (r[h].x0 - xq0);
#pragma unroll
                    for (int k = 0; k < 4; k++) {
                        const int b = (k & 2) ? r[h].b1 : r[h].b0, a = (k & 1) ? r[h].a1 : r[h].a0;
                        const uint32_t* q0 = rgba + __mul24(nodemap[0][__mul24(b - B00, nA0) + (a - A00)], npix) + pix;
                        const uint32_t* q1 = q0 + sxp;
                        s16[h][4 * k + 0] = q0[0];
                        s16[h][4 * k + 1] = q0[1];
                        s16[h][4 * k + 2] = q1[0];
                        s16[h][4 * k + 3] = q1[1];
                    }
                }
                if (live) {
#pragma unroll
                    for (int h = 0; h < 2; h++) {
                        if (h == 1 && !two) break;
                        const BlendW w = lf_blend_weights(r[h]);
#pragma unroll
                        for (int c = 0; c < 3; c++) {
                            float sm[16];
#pragma unroll
                            for (int k = 0; k < 16; k++) sm[k] = (float)((s16[h][k] >> (8 * c)) & 255u);
                            __builtin_nontemporal_store(
                                lf_blend16(sm, w), &out[((int64_t)(v0 + q + h) * 3 + c) * npix_out + (int64_t)j * wo + i]);
                        }
                    }
                }
            }
        }
        __syncthreads();  // the next group's plan rewrites the node maps
        f += n;
        if (++streak == 4) {
            ceil_n = min(ceil_n + 1, gmax + 1);
            streak = 0;
        }
        n = min(min(gmax, 2 * n), ceil_n - 1);
    }
    return left;
}

