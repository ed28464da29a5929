// Relaxed (real-valued) forward model and its adjoint, for encoder-side
// refinement of the dequantised residual planes and per-block shifts.
//
// Relaxed model: parameters are a real residual for every SRV value,
// res[c][node][y][x] (BFS node order), and a real shift per motion-compensated
// block, shift[rec] = (dx, dy) in pixels (initially the quarter-pel vector / 4;
// Phase-shifted Motion Compensation).  A reference SRV equals its residual
// plane; a predictive SRV is phase * bilinear(reference, shifted) + its
// residual, without rounding; a sample is root + the sum of its path's SRVs;
// the colour inverse is the linear one (R = Y + Co/2 - Cg/2, G = Y + Cg/2,
// B = Y - Co/2 - Cg/2); nothing is clamped; rendering is the quadrilinear
// blend of the renderer.  Within a block every pixel has the same bilinear
// fraction (floor(x + dx) = x + floor(dx)), which both directions use.
//
// Adjoint, deterministic and without atomics:
//  1. every ray emits one record per light-field view it blends, keyed by
//     the sample at the top-left of its 2x2 pixel footprint in that view
//     (ray * 4 + view corner), and its four blend fractions;
//  2. a stable radix sort groups the records by key, and a table gives the
//     first record of each key;
//  3. every sample gathers the records keyed at itself and at its left, upper
//     and upper-left neighbours (the footprints that cover it), in that order
//     and in ray order within each, forms each ray's blend weight from its
//     fractions and applies the colour transpose, writing the sample
//     gradients into the level-0 node planes;
//  4. node gradients are summed up the tree level by level in fixed order;
//  5. each reference residual pulls the phase-signed bilinear transpose of
//     its predictive siblings' gradients;
//  6. each block's shift gradient is a fixed-order wave64 reduction.
#include <hip/hip_runtime.h>
#include <hipcub/hipcub.hpp>

#include <algorithm>

#include "lf_internal.h"

#define AD_MAX_PARTS 1024  // partial maxima of the shift reduction
#define AD_TILE 16         // reference tile side of the pull kernel
#define AD_PPT 1           // pixels per thread (rows AD_TILE * k / AD_PPT apart)
// LDS of the reference pull: 23.5 KB, six workgroups per CU (the budgets
// fit tiles whose reach is up to 11 pixels; beyond, the unstaged paths)
#define AD_CAND_MAX 192    // candidate blocks a tile stages in LDS
#define AD_WIN_MAX 4336    // sibling gradient values a tile stages in LDS (3 windows of up to 38 x 38)

__device__ __forceinline__ float ad_lerp(float p, float q, float f) { return fmaf(f, q - p, p); }

struct AdRay {
    int a0, a1, b0, b1, x0, x1, y0, y1;
    float fu, fv, fs, ft;
};

__device__ __forceinline__ AdRay ad_ray(const LfGeom& g, const float* __restrict__ cam, int i, int j)
{
    AdRay r;
    float u, v, s, t;
    lf_ray(cam, i, j, u, v, s, t);
    lf_axis(u, g.na, r.a0, r.a1, r.fu);
    lf_axis(v, g.nb, r.b0, r.b1, r.fv);
    lf_axis(s, g.w, r.x0, r.x1, r.fs);
    lf_axis(t, g.h, r.y0, r.y1, r.ft);
    return r;
}

// record index of predictive node (B, A) of level l, channel c, block blk
__device__ __forceinline__ int64_t ad_record(const LfGeom& g, int c, int l, int B, int A, int blk)
{
    return g.rec_base[c][l] + (int64_t)pred_ordinal(g.na_l[l], B, A) * g.nblk + blk;
}

__device__ __forceinline__ int ad_phase(const LfGeom& g, const LfPtrs& p, int c, int l, int B, int A, int blk)
{
    int mx, my, sg;
    lf_motion(g, p, c, l, (uint32_t)(pred_ordinal(g.na_l[l], B, A) * g.nblk + blk), mx, my, sg);
    return sg;
}

// ---------------------------------------------------------------------------
// parameter export: dequantised residuals and vector / 4
// ---------------------------------------------------------------------------

__global__ void k_export_residual(LfGeom g, LfPtrs p, float* __restrict__ res)
{
    const int64_t plane = (int64_t)g.w * g.h;
    const int64_t total = 3 * (int64_t)g.n_nodes * plane;
    for (int64_t t = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; t < total; t += (int64_t)gridDim.x * blockDim.x) {
        const int64_t px = t % plane;
        const int node = (int)((t / plane) % g.n_nodes);
        const int c = (int)(t / (plane * g.n_nodes));
        int l = 0;
        while (node < g.node_base[l]) l++;
        const int y = (int)(px / g.w), x = (int)(px % g.w);
        const int blk = (y / g.bs) * g.nbx + x / g.bs, i = (y % g.bs) * g.bs + x % g.bs;
        res[t] = (float)lf_residual(g, p, c, l, node, blk, i);
    }
}

__global__ void k_export_shift(LfGeom g, LfPtrs p, int64_t n_rec, float2* __restrict__ shift)
{
    const int64_t r = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (r >= n_rec) return;
    int c = 0, l = g.H - 1;
    while (c < 2 && r >= g.rec_base[c + 1][g.H - 1]) c++;
    while (l > 0 && r >= g.rec_base[c][l - 1]) l--;
    const uint32_t j = (uint32_t)(r - g.rec_base[c][l]);
    int mx, my, sg;
    lf_motion(g, p, c, l, j, mx, my, sg);
    shift[r] = make_float2((float)mx * 0.25f, (float)my * 0.25f);
}

extern "C" lf_status lf_export_params(const lf_handle* h, float* d_residual, float* d_shift, void* stream)
{
    if (!h || !d_residual || !d_shift) return lf_fail(LF_EINVAL, "null argument");
    if (lf_status cs = lf_require_full_chroma(h, "lf_export_params")) return cs;
    const LfGeom& g = h->L.g;
    hipStream_t s = (hipStream_t)stream;
    hipLaunchKernelGGL(k_export_residual, dim3(65536), dim3(256), 0, s, g, h->p, d_residual);
    if (h->L.n_rec > 0)
        hipLaunchKernelGGL(k_export_shift, dim3((unsigned)((h->L.n_rec + 255) / 256)), dim3(256), 0, s, g, h->p,
                           h->L.n_rec, (float2*)d_shift);
    return lf_check_launch("export_params");
}

// ---------------------------------------------------------------------------
// relaxed forward
// ---------------------------------------------------------------------------

// bilinear sample of a real plane at (y + dy, x + dx), taps clamped
__device__ __forceinline__ float ad_bilerp(const float* __restrict__ R, int w, int h, int y, int x, float2 d)
{
    const float fdx = floorf(d.x), fdy = floorf(d.y);
    const float fx = d.x - fdx, fy = d.y - fdy;
    const int x0 = x + (int)fdx, y0 = y + (int)fdy;
    const int xa = lf_clampi(x0, 0, w - 1), xb = lf_clampi(x0 + 1, 0, w - 1);
    const int ya = lf_clampi(y0, 0, h - 1), yb = lf_clampi(y0 + 1, 0, h - 1);
    return ad_lerp(ad_lerp(R[ya * w + xa], R[ya * w + xb], fx), ad_lerp(R[yb * w + xa], R[yb * w + xb], fx), fy);
}

// Relaxed SRV values of node (B, A) of level l, channel c, at the pixels
// (ys[k >> 1], xs[k & 1]): the residual plus the phase-signed bilinear
// prediction; the block's phase and shift are read once per block.
__device__ inline void ad_srv_quad(const LfGeom& g, const LfPtrs& p, const float* __restrict__ res,
                                   const float2* __restrict__ shift, int c, int l, int B, int A, const int ys[2],
                                   const int xs[2], float v[4])
{
    const int64_t plane = (int64_t)g.w * g.h;
    const float* S = res + ((int64_t)c * g.n_nodes + g.node_base[l] + B * g.na_l[l] + A) * plane;
    const bool pred = (A | B) & 1;
    const float* R = res + ((int64_t)c * g.n_nodes + g.node_base[l] + (B & ~1) * g.na_l[l] + (A & ~1)) * plane;
    int blk0 = -1, sg = 0;
    float2 d = make_float2(0.0f, 0.0f);
#pragma unroll 1
    for (int k = 0; k < 4; k++) {
        const int y = ys[k >> 1], x = xs[k & 1];
        float sv = S[y * g.w + x];
        if (pred) {
            const int blk = (y / g.bs) * g.nbx + x / g.bs;
            if (blk != blk0) {
                sg = ad_phase(g, p, c, l, B, A, blk);
                if (sg) d = shift[ad_record(g, c, l, B, A, blk)];
                blk0 = blk;
            }
            if (sg) {
                const float q = ad_bilerp(R, g.w, g.h, y, x, d);
                sv += sg > 0 ? q : -q;
            }
        }
        v[k] = sv;
    }
}

// One channel of the 16 samples of a ray (view k >> 2 = b0a0, b0a1, b1a0,
// b1a1, pixel k & 3): root plus the relaxed SRVs of levels 0 .. H-1, added in
// that order; views sharing a tree node share its evaluation.
__device__ __forceinline__ void ad_ray_channel(const LfGeom& g, const LfPtrs& p, const float* __restrict__ res,
                                               const float2* __restrict__ shift, const AdRay& r, int c, float acc[16])
{
    const int ys[2] = {r.y0, r.y1}, xs[2] = {r.x0, r.x1};
    const int64_t plane = (int64_t)g.w * g.h;
    const int H = g.H;
#pragma unroll
    for (int q = 0; q < 4; q++) {
        const int b = (q & 2) ? r.b1 : r.b0, a = (q & 1) ? r.a1 : r.a0;
        const int16_t* rt = p.root + ((size_t)(c * g.root_nb + (b >> H)) * g.root_na + (a >> H)) * plane;
#pragma unroll
        for (int k = 0; k < 4; k++) acc[4 * q + k] = (float)rt[ys[k >> 1] * g.w + xs[k & 1]];
    }
    for (int l = 0; l < H; l++) {
        const bool eqA = (r.a0 >> l) == (r.a1 >> l), eqB = (r.b0 >> l) == (r.b1 >> l);
        float v[4][4];
        ad_srv_quad(g, p, res, shift, c, l, r.b0 >> l, r.a0 >> l, ys, xs, v[0]);
        if (!eqA) ad_srv_quad(g, p, res, shift, c, l, r.b0 >> l, r.a1 >> l, ys, xs, v[1]);
        if (!eqB) ad_srv_quad(g, p, res, shift, c, l, r.b1 >> l, r.a0 >> l, ys, xs, v[2]);
        if (!eqA && !eqB) ad_srv_quad(g, p, res, shift, c, l, r.b1 >> l, r.a1 >> l, ys, xs, v[3]);
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

__global__ void __launch_bounds__(256) k_render_relaxed(LfGeom g, LfPtrs p, const float* __restrict__ res,
                                                        const float2* __restrict__ shift,
                                                        const float* __restrict__ cams, int nv, int wo, int ho,
                                                        float* __restrict__ out)
{
    const int64_t npix = (int64_t)wo * ho;
    const int64_t r = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (r >= npix * nv) return;
    const int v = (int)(r / npix);
    const int64_t px = r - (int64_t)v * npix;
    const int j = (int)(px / wo), i = (int)(px % wo);
    const AdRay ry = ad_ray(g, cams + 18 * v, i, j);
    float Ys[16], Cos[16], Cgs[16];
    ad_ray_channel(g, p, res, shift, ry, 0, Ys);
    ad_ray_channel(g, p, res, shift, ry, 1, Cos);
    ad_ray_channel(g, p, res, shift, ry, 2, Cgs);
    float sm[16][3];
#pragma unroll
    for (int k = 0; k < 16; k++) {
        const float Y = Ys[k], Co = Cos[k], Cg = Cgs[k];
        sm[k][0] = Y + 0.5f * Co - 0.5f * Cg;
        sm[k][1] = Y + 0.5f * Cg;
        sm[k][2] = Y - 0.5f * Co - 0.5f * Cg;
    }
#pragma unroll
    for (int c = 0; c < 3; c++) {
        float vw[4];
#pragma unroll
        for (int q = 0; q < 4; q++)
            vw[q] = ad_lerp(ad_lerp(sm[4 * q][c], sm[4 * q + 1][c], ry.fs), ad_lerp(sm[4 * q + 2][c], sm[4 * q + 3][c], ry.fs),
                            ry.ft);
        out[((int64_t)v * 3 + c) * npix + px] =
            ad_lerp(ad_lerp(vw[0], vw[1], ry.fu), ad_lerp(vw[2], vw[3], ry.fu), ry.fv) * (1.0f / 255.0f);
    }
}

extern "C" lf_status lf_render_relaxed(const lf_handle* h, const float* d_residual, const float* d_shift,
                                       const float* d_cams, int32_t n_views, int32_t width, int32_t height, float* d_out,
                                       void* stream)
{
    if (!h || !d_residual || !d_shift || n_views < 0 || width < 1 || height < 1) return lf_fail(LF_EINVAL, "bad argument");
    if (lf_status cs = lf_require_full_chroma(h, "lf_render_relaxed")) return cs;
    if (n_views == 0) return LF_OK;
    if (!d_cams || !d_out) return lf_fail(LF_EINVAL, "null buffer");
    const int64_t total = (int64_t)n_views * width * height;
    if ((total + 255) / 256 > 0x7FFFFFFF) return lf_fail(LF_EINVAL, "too many rays");
    hipLaunchKernelGGL(k_render_relaxed, dim3((unsigned)((total + 255) / 256)), dim3(256), 0, (hipStream_t)stream,
                       h->L.g, h->p, d_residual, (const float2*)d_shift, d_cams, n_views, width, height, d_out);
    return lf_check_launch("render_relaxed");
}

// ---------------------------------------------------------------------------
// adjoint
// ---------------------------------------------------------------------------

struct BwdLayout {
    int64_t n_recs, n_samples;
    int end_bit;
    size_t sort_bytes;
    int64_t o_kin, o_kout, o_vin, o_vout, o_sort, o_start, o_max, o_parts, o_rayf, o_brec, total;
};

static int64_t al256(int64_t v) { return (v + 255) & ~(int64_t)255; }

static lf_status bwd_layout(const lf_handle* h, int nv, int wo, int ho, BwdLayout* B)
{
    const LfGeom& g = h->L.g;
    B->n_recs = (int64_t)nv * wo * ho * 4;
    B->n_samples = (int64_t)g.na * g.nb * g.w * g.h;
    // the record sort takes an int count: at most 2^31 - 1 records (2^29 - 1 rays per call)
    if (B->n_recs > 0x7FFFFFFFll) return lf_fail(LF_EINVAL, "too many rays for one backward call (at most 2^29 - 1)");
    if (B->n_samples >= 0xFFFFFFFFll) return lf_fail(LF_EINVAL, "too many light-field samples");
    // the reference pull indexes its 16x16 tiles with 32-bit integers
    if (3 * (int64_t)g.n_refs * ((g.w + AD_TILE - 1) / AD_TILE) * ((g.h + AD_TILE - 1) / AD_TILE) > 0x7FFFFFFFll)
        return lf_fail(LF_EINVAL, "too many reference tiles for the adjoint");
    int eb = 1;
    while (eb < 32 && ((int64_t)1 << eb) < B->n_samples) eb++;
    B->end_bit = eb;
    size_t sb = 0;
    if (hipcub::DeviceRadixSort::SortPairs(nullptr, sb, (uint32_t*)nullptr, (uint32_t*)nullptr, (uint32_t*)nullptr,
                                           (uint32_t*)nullptr, (int)B->n_recs, 0, eb) != hipSuccess)
        return lf_fail(LF_EDEVICE, "sort workspace query failed");
    B->sort_bytes = sb;
    const int64_t pb = al256(B->n_recs * 4);
    B->o_kin = 0;
    B->o_kout = B->o_kin + pb;
    B->o_vin = B->o_kout + pb;
    B->o_vout = B->o_vin + pb;
    B->o_sort = B->o_vout + pb;
    B->o_start = B->o_sort + al256((int64_t)sb);
    B->o_max = B->o_start + al256(B->n_samples * 4);
    B->o_parts = B->o_max + 256;
    B->o_rayf = B->o_parts + al256(AD_MAX_PARTS * 4);
    B->o_brec = B->o_rayf + al256(B->n_recs / 4 * 16);  // one float4 per ray
    B->total = B->o_brec + al256(h->L.n_rec * 16);         // one split shift per predictive block
    return LF_OK;
}

extern "C" lf_status lf_backward_workspace(const lf_handle* h, int32_t n_views, int32_t width, int32_t height,
                                           int64_t* bytes)
{
    if (!h || !bytes || n_views < 1 || width < 1 || height < 1) return lf_fail(LF_EINVAL, "bad argument");
    if (lf_status cs = lf_require_full_chroma(h, "lf_backward_workspace")) return cs;
    BwdLayout B;
    lf_status st = bwd_layout(h, n_views, width, height, &B);
    if (st != LF_OK) return st;
    *bytes = B.total;
    return LF_OK;
}

__global__ void k_ad_records(LfGeom g, const float* __restrict__ cams, int nv, int wo, int ho,
                             uint32_t* __restrict__ keys, uint32_t* __restrict__ vals, float4* __restrict__ rayf)
{
    const int64_t npix = (int64_t)wo * ho;
    const int64_t r = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (r >= npix * nv) return;
    const int v = (int)(r / npix);
    const int64_t px = r - (int64_t)v * npix;
    const AdRay ry = ad_ray(g, cams + 18 * v, (int)(px % wo), (int)(px / wo));
    rayf[r] = make_float4(ry.fu, ry.fv, ry.fs, ry.ft);  // the blend fractions, for the gather pass
#pragma unroll
    for (int q = 0; q < 4; q++) {
        const int b = (q & 2) ? ry.b1 : ry.b0, a = (q & 1) ? ry.a1 : ry.a0;
        keys[r * 4 + q] = (uint32_t)((((int64_t)b * g.na + a) * g.h + ry.y0) * g.w + ry.x0);
        vals[r * 4 + q] = (uint32_t)(r * 4 + q);
    }
}

__global__ void k_ad_nostart(uint32_t* __restrict__ start, int64_t n)
{
    for (int64_t t = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; t < n; t += (int64_t)gridDim.x * blockDim.x)
        start[t] = 0xFFFFFFFFu;
}

// first record of every key present
__global__ void k_ad_heads(const uint32_t* __restrict__ keys, int64_t n, uint32_t* __restrict__ start)
{
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= n) return;
    const uint32_t k = keys[i];
    if (i == 0 || keys[i - 1] != k) start[k] = (uint32_t)i;
}

// One thread per light-field sample ((b * na + a) * h + y) * w + x, which is
// also the offset of pixel (y, x) in the level-0 node planes of a channel, so
// the YCoCg sample gradients go straight into the residual gradient (channel
// stride cstride); samples no ray reaches get zero.  A record keyed at the
// footprint corner (y0, x0) reaches pixel corner (cy, cx) at (y0 + cy, x0 +
// cx), except along an axis of length 1, where both corners are pixel 0.
__global__ void k_ad_samples(const float4* __restrict__ rayf, int wo, int ho, const float* __restrict__ grad_out,
                             const uint32_t* __restrict__ keys, const uint32_t* __restrict__ vals,
                             const uint32_t* __restrict__ start, int64_t n_recs, int64_t n_samples, int w, int h,
                             int64_t cstride, float* __restrict__ g0 /* level-0 planes of channel 0 */)
{
    const int64_t S = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (S >= n_samples) return;
    const int64_t npix = (int64_t)wo * ho;
    const int x = (int)(S % w), y = (int)((S / w) % h);
    float acc[3] = {0.0f, 0.0f, 0.0f};
    for (int cy = 0; cy < 2; cy++) {
        const int dy = h >= 2 ? cy : 0;
        if (y < dy) continue;
        for (int cx = 0; cx < 2; cx++) {
            const int dx = w >= 2 ? cx : 0;
            if (x < dx) continue;
            const uint32_t K = (uint32_t)(S - (int64_t)dy * w - dx);
            uint32_t j = start[K];
            if (j == 0xFFFFFFFFu) continue;
            for (; (int64_t)j < n_recs && keys[j] == K; j++) {
                const uint32_t val = vals[j];
                const int64_t ray = val >> 2;
                const int q = (int)(val & 3u);
                const int v = (int)(ray / npix);
                const int64_t px = ray - (int64_t)v * npix;
                const float4 f = rayf[ray];  // (fu, fv, fs, ft)
                const float wt = ((q & 2) ? f.y : 1.0f - f.y) * ((q & 1) ? f.x : 1.0f - f.x) *
                                 (cy ? f.w : 1.0f - f.w) * (cx ? f.z : 1.0f - f.z) * (1.0f / 255.0f);
#pragma unroll
                for (int c = 0; c < 3; c++) acc[c] = fmaf(wt, grad_out[((int64_t)v * 3 + c) * npix + px], acc[c]);
            }
        }
    }
    // colour transpose of R = Y + Co/2 - Cg/2, G = Y + Cg/2, B = Y - Co/2 - Cg/2
    g0[S] = acc[0] + acc[1] + acc[2];
    g0[cstride + S] = 0.5f * (acc[0] - acc[2]);
    g0[2 * cstride + S] = 0.5f * (acc[1] - acc[0] - acc[2]);
}

// node gradients of level l >= 1: the sum of its children's (level 0 holds
// the sample gradients themselves)
__global__ void k_ad_tree(LfGeom g, int l, float* __restrict__ gres)
{
    const int64_t plane = (int64_t)g.w * g.h;
    const int64_t nodes_l = (int64_t)g.na_l[l] * g.nb_l[l];
    const int64_t total = 3 * nodes_l * plane;
    for (int64_t t = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; t < total; t += (int64_t)gridDim.x * blockDim.x) {
        const int64_t px = t % plane;
        const int64_t loc = (t / plane) % nodes_l;
        const int c = (int)(t / (plane * nodes_l));
        const int B = (int)(loc / g.na_l[l]), A = (int)(loc % g.na_l[l]);
        float v = 0.0f;
        for (int jj = 0; jj < 2; jj++)
            for (int ii = 0; ii < 2; ii++) {
                const int Bc = 2 * B + jj, Ac = 2 * A + ii;
                if (Bc >= g.nb_l[l - 1] || Ac >= g.na_l[l - 1]) continue;
                v += gres[((int64_t)c * g.n_nodes + g.node_base[l - 1] + Bc * g.na_l[l - 1] + Ac) * plane + px];
            }
        gres[((int64_t)c * g.n_nodes + g.node_base[l] + loc) * plane + px] = v;
    }
}

// largest |shift| component: AD_MAX_PARTS workgroups write partial maxima,
// then one workgroup reduces them (a maximum is exact in any order)
__global__ void k_ad_maxshift(const float2* __restrict__ shift, int64_t n, float* __restrict__ out)
{
    __shared__ float red[256];
    float m = 0.0f;
    for (int64_t t = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; t < n; t += (int64_t)gridDim.x * blockDim.x)
        m = fmaxf(m, fmaxf(fabsf(shift[t].x), fabsf(shift[t].y)));
    red[threadIdx.x] = m;
    __syncthreads();
    for (int s = 128; s > 0; s >>= 1) {
        if ((int)threadIdx.x < s) red[threadIdx.x] = fmaxf(red[threadIdx.x], red[threadIdx.x + s]);
        __syncthreads();
    }
    if (threadIdx.x == 0) out[blockIdx.x] = red[0];
}

__global__ void k_ad_maxparts(const float* __restrict__ parts, int n, float* __restrict__ out)
{
    __shared__ float red[256];
    float m = 0.0f;
    for (int t = threadIdx.x; t < n; t += blockDim.x) m = fmaxf(m, parts[t]);
    red[threadIdx.x] = m;
    __syncthreads();
    for (int s = 128; s > 0; s >>= 1) {
        if ((int)threadIdx.x < s) red[threadIdx.x] = fmaxf(red[threadIdx.x], red[threadIdx.x + s]);
        __syncthreads();
    }
    if (threadIdx.x == 0) out[0] = red[0];
}

// pixel range [lo, hi] of [k0, k1] whose tap (x + fd + o), clamped to [0, n-1], equals X
__device__ __forceinline__ void ad_tap_range(int X, int n, int fd, int o, int k0, int k1, int& lo, int& hi)
{
    if (n == 1) {
        lo = k0;
        hi = k1;
    } else if (X == 0) {
        lo = k0;
        hi = min(k1, -fd - o);
    } else if (X == n - 1) {
        lo = max(k0, n - 1 - fd - o);
        hi = k1;
    } else {
        lo = max(k0, X - fd - o);
        hi = min(k1, X - fd - o);
    }
}

// Phase and split shift of one predictive block: integer part (clamped to
// [-w-1, w] / [-h-1, h], which leaves every clamped tap where it was) and
// fractional part.
struct AdRec {
    int sg, ix, iy;
    float fx, fy;
};

__device__ __forceinline__ int4 ad_pack(const AdRec& d)
{
    return make_int4(d.sg, (d.ix & 0xFFFF) | (d.iy << 16), __float_as_int(d.fx), __float_as_int(d.fy));
}

__device__ __forceinline__ AdRec ad_unpack(int4 v)
{
    return AdRec{v.x, (int)(int16_t)(v.y & 0xFFFF), v.y >> 16, __int_as_float(v.z), __int_as_float(v.w)};
}

// phase and split shift of every predictive block, in record order, decoded
// once for the reference pull (each block is a candidate of several tiles)
__global__ void k_ad_blockrec(LfGeom g, LfPtrs p, const float2* __restrict__ shift, int64_t n_rec,
                              int4* __restrict__ brec)
{
    const int64_t rec = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (rec >= n_rec) return;
    int c = 0, l = g.H - 1;
    while (c < 2 && rec >= g.rec_base[c + 1][g.H - 1]) c++;
    while (l > 0 && rec >= g.rec_base[c][l - 1]) l--;
    int mx, my, sg;
    lf_motion(g, p, c, l, (uint32_t)(rec - g.rec_base[c][l]), mx, my, sg);
    AdRec d{sg, 0, 0, 0.0f, 0.0f};
    if (sg) {
        const float2 s = shift[rec];
        const float fdx = floorf(s.x), fdy = floorf(s.y);
        d.fx = s.x - fdx;
        d.fy = s.y - fdy;
        d.ix = (int)fminf(fmaxf(fdx, (float)(-g.w - 1)), (float)g.w);
        d.iy = (int)fminf(fmaxf(fdy, (float)(-g.h - 1)), (float)g.h);
    }
    brec[rec] = ad_pack(d);
}

// What reference pixel (X, Y) pulls from one predictive block (row ky,
// column kx) with gradient plane gp: the bilinear weights of the block's taps
// that land on the pixel times the gradients of their pixels, phase-signed,
// added to acc.
template <class Get>
__device__ __forceinline__ float ad_block_pull(const LfGeom& g, Get get, int X, int Y, int ky, int kx, const AdRec& d,
                                               float acc)
{
    float blk_acc = 0.0f;
    const int bx0 = kx * g.bs, by0 = ky * g.bs;
    if (X > 0 && X < g.w - 1 && Y > 0 && Y < g.h - 1) {
        // away from the image border no tap is clamped: the tap (oy, ox)
        // landing on the pixel comes from source pixel (Y - iy - oy, X - ix - ox)
        // alone, when that pixel lies in the block
#pragma unroll
        for (int oy = 0; oy < 2; oy++) {
            const int ys = Y - d.iy - oy;
            const float wy = oy ? d.fy : 1.0f - d.fy;
#pragma unroll
            for (int ox = 0; ox < 2; ox++) {
                const int xs = X - d.ix - ox;
                if (ys >= by0 && ys < by0 + g.bs && xs >= bx0 && xs < bx0 + g.bs)
                    blk_acc = fmaf(wy * (ox ? d.fx : 1.0f - d.fx), get(ys, xs), blk_acc);
            }
        }
    } else {
        for (int oy = 0; oy < 2; oy++) {
            int ylo, yhi;
            ad_tap_range(Y, g.h, d.iy, oy, by0, by0 + g.bs - 1, ylo, yhi);
            if (ylo > yhi) continue;
            const float wy = oy ? d.fy : 1.0f - d.fy;
            for (int ox = 0; ox < 2; ox++) {
                int xlo, xhi;
                ad_tap_range(X, g.w, d.ix, ox, bx0, bx0 + g.bs - 1, xlo, xhi);
                if (xlo > xhi) continue;
                const float wxy = wy * (ox ? d.fx : 1.0f - d.fx);
                float sum = 0.0f;
                for (int y = ylo; y <= yhi; y++)
                    for (int x = xlo; x <= xhi; x++) sum += get(y, x);
                blk_acc = fmaf(wxy, sum, blk_acc);
            }
        }
    }
    return acc + (d.sg > 0 ? blk_acc : -blk_acc);
}

// Gradient that reference pixel (X, Y) of the cluster with reference node
// (Br, Ar) pulls from its predictive siblings' gradients: for every sibling
// block whose shifted taps can reach the pixel, the bilinear weights of the
// taps that land on it (phase-signed), added in sibling, block-row,
// block-column order.  fetch(sib, B, A, ky, kx) returns the block's AdRec.
template <class Fetch>
__device__ inline float ad_pull(const LfGeom& g, const float* __restrict__ gres, int c, int l, int Br, int Ar, int X,
                                int Y, int reach, int lky0, int lky1, int lkx0, int lkx1, Fetch fetch, float acc)
{
    // the loops run over [lky0, lky1] x [lkx0, lkx1] (a tile's shared range,
    // uniform across its pixels) and skip the blocks outside this pixel's range
    const int64_t plane = (int64_t)g.w * g.h;
    const int kx0 = max(0, (X - reach) / g.bs), kx1 = min(g.nbx - 1, (X + reach) / g.bs);
    const int nby = g.h / g.bs;
    const int ky0 = max(0, (Y - reach) / g.bs), ky1 = min(nby - 1, (Y + reach) / g.bs);
    for (int sib = 1; sib < 4; sib++) {
        const int B = Br + (sib >> 1), A = Ar + (sib & 1);
        if (B >= g.nb_l[l] || A >= g.na_l[l]) continue;
        const float* gp = gres + ((int64_t)c * g.n_nodes + g.node_base[l] + B * g.na_l[l] + A) * plane;
        for (int ky = lky0; ky <= lky1; ky++)
            for (int kx = lkx0; kx <= lkx1; kx++) {
                if (ky < ky0 || ky > ky1 || kx < kx0 || kx > kx1) continue;
                const AdRec d = fetch(sib, B, A, ky, kx);
                if (!d.sg) continue;
                acc = ad_block_pull(g, [&](int y, int x) { return gp[y * g.w + x]; }, X, Y, ky, kx, d, acc);
            }
    }
    return acc;
}


// reference residual gradient: own node gradient plus the phase-signed
// bilinear transpose of every predictive sibling's gradient (pull form).  A
// workgroup takes 16x16 tiles of one reference plane.  The candidate blocks
// (those within the largest shift of the tile) are read from the decoded
// block records; the ones whose shifted taps land inside the tile are kept, in
// (sibling, block-row, block-column) order, in an LDS list that every pixel
// of the tile walks (the blocks left out add exactly zero to every pixel of
// the tile).  The three sibling gradient windows the taps can come from are
// staged in LDS when they fit; their loads, the candidates' and the pixel's
// own gradient are issued together.  With more candidates than the LDS
// budget holds, every pixel reads its own candidates instead.
__global__ void __launch_bounds__(256) k_ad_reference(LfGeom g, const int4* __restrict__ brec,
                                                      const float* __restrict__ maxshift, float* __restrict__ gres)
{
    // kept block i: windowed tiles: lst_a = (x origin kx bs + ix, y origin
    // ky bs + iy, window offset of source pixel (Y - iy, X - ix) less
    // Y ww + X, packed (sibling, ky, kx)), lst_b = the tap weights (1-fy)(1-fx),
    // (1-fy) fx, fy (1-fx), fy fx times the phase (float bits); otherwise
    // lst_a = the block record, lst_b.x = packed (sibling, ky, kx)
    __shared__ int4 lst_a[AD_CAND_MAX], lst_b[AD_CAND_MAX];
    __shared__ float win[AD_WIN_MAX];  // [sibling - 1][window row][window column]
    __shared__ int wcount[4];
    const int64_t plane = (int64_t)g.w * g.h;
    const int tiles_x = (g.w + AD_TILE - 1) / AD_TILE, tiles_y = (g.h + AD_TILE - 1) / AD_TILE;
    // 32-bit tile indices (the host bounds the tile count by 2^31 - 1)
    const int per_plane = tiles_x * tiles_y;
    const int n_tiles = 3 * g.n_refs * per_plane;
    const int reach = (int)ceilf(fminf(maxshift[0], (float)(g.w + g.h))) + 2;
    const int nby = g.h / g.bs;
    const int lane = threadIdx.x & 63, wv = threadIdx.x >> 6;
    for (int T = blockIdx.x; T < n_tiles; T += gridDim.x) {
        const int rp = T / per_plane;
        const int tt = T - rp * per_plane;
        const int c = rp / g.n_refs, r = rp - c * g.n_refs;
        int l = 0;
        while (l + 1 < g.H && r >= g.ref_base[l + 1]) l++;
        const int loc = r - g.ref_base[l];
        const int Br = 2 * (loc / g.na_l[l + 1]), Ar = 2 * (loc % g.na_l[l + 1]);
        const int tx0 = (tt % tiles_x) * AD_TILE, ty0 = (tt / tiles_x) * AD_TILE;
        const int tx1 = min(tx0 + AD_TILE - 1, g.w - 1), ty1 = min(ty0 + AD_TILE - 1, g.h - 1);
        const int ckx0 = max(0, (tx0 - reach) / g.bs), ckx1 = min(g.nbx - 1, (tx1 + reach) / g.bs);
        const int cky0 = max(0, (ty0 - reach) / g.bs), cky1 = min(nby - 1, (ty1 + reach) / g.bs);
        const int nkx = ckx1 - ckx0 + 1, nk = nkx * (cky1 - cky0 + 1);
        const bool staged = 3 * nk <= AD_CAND_MAX;  // uniform
        // Every tap a pixel of the tile pulls comes from within `reach` of the tile.
        const int wx0 = max(0, tx0 - reach), wx1 = min(g.w - 1, tx1 + reach);
        const int wy0 = max(0, ty0 - reach), wy1 = min(g.h - 1, ty1 + reach);
        const int ww = wx1 - wx0 + 1, nr = wy1 - wy0 + 1, wa = ww * nr;
        const bool windowed = staged && ww <= 64 && 3 * wa <= AD_WIN_MAX;  // uniform

        // loads in flight together: candidate records, the pixel's own
        // gradient, the sibling windows
        constexpr int CR = (AD_CAND_MAX + 255) / 256;
        int4 cv[CR];
        bool cok[CR];
#pragma unroll
        for (int k2 = 0; k2 < CR; k2++) {
            const int e = k2 * 256 + (int)threadIdx.x;
            cok[k2] = false;
            cv[k2] = make_int4(0, 0, 0, 0);
            if (staged && e < 3 * nk) {
                const int sib = 1 + e / nk, k = e - (sib - 1) * nk;
                const int B = Br + (sib >> 1), A = Ar + (sib & 1);
                if (B < g.nb_l[l] && A < g.na_l[l]) {
                    cok[k2] = true;
                    cv[k2] = brec[ad_record(g, c, l, B, A, (cky0 + k / nkx) * g.nbx + ckx0 + k % nkx)];
                }
            }
        }
        // pixel k of this thread: column tid % AD_TILE, row tid / AD_TILE + k AD_TILE / AD_PPT
        constexpr int RSTEP = AD_TILE / AD_PPT;
        const int X = tx0 + (int)threadIdx.x % AD_TILE, Y0 = ty0 + (int)threadIdx.x / AD_TILE;
        const int64_t own0 = ((int64_t)c * g.n_nodes + g.node_base[l] + Br * g.na_l[l] + Ar) * plane + X;
        float own_g[AD_PPT];
#pragma unroll
        for (int k = 0; k < AD_PPT; k++) {
            const int Y = Y0 + k * RSTEP;
            own_g[k] = (X <= tx1 && Y <= ty1) ? gres[own0 + (int64_t)Y * g.w] : 0.0f;
        }
        if (windowed) {
            // all of the three windows' loads in flight at once: value e of
            // the concatenation is value rr of sibling window sw (row rr / ww,
            // column rr % ww; the row from a float reciprocal, exact for
            // rr < 2^13 and ww <= 64)
            constexpr int WL = (AD_WIN_MAX + 255) / 256;
            const float rw = 1.0f / (float)ww;
            const int64_t nb0 = (int64_t)c * g.n_nodes + g.node_base[l];
            const bool h1 = Ar + 1 < g.na_l[l], h2 = Br + 1 < g.nb_l[l], h3 = h1 && h2;
            const float* s1 = gres + (nb0 + Br * g.na_l[l] + Ar + 1) * plane;
            const float* s2 = gres + (nb0 + (Br + 1) * g.na_l[l] + Ar) * plane;
            const float* s3 = gres + (nb0 + (Br + 1) * g.na_l[l] + Ar + 1) * plane;
            float v[WL];
#pragma unroll
            for (int u = 0; u < WL; u++) {
                const int e = u * 256 + (int)threadIdx.x;
                const int sw = e >= 2 * wa ? 2 : (e >= wa ? 1 : 0);
                const int rr = e - sw * wa;
                const int yy = (int)(((float)rr + 0.5f) * rw), xx = rr - yy * ww;
                const bool has = sw == 0 ? h1 : (sw == 1 ? h2 : h3);
                const float* sp = sw == 0 ? s1 : (sw == 1 ? s2 : s3);
                v[u] = (e < 3 * wa && has) ? sp[(int64_t)(wy0 + yy) * g.w + wx0 + xx] : 0.0f;
            }
#pragma unroll
            for (int u = 0; u < WL; u++) {
                const int e = u * 256 + (int)threadIdx.x;
                if (e < 3 * wa) win[e] = v[u];
            }
        }
        // keep the candidates whose taps reach the tile, in order
        int n_list = 0;
        if (staged) {
#pragma unroll
            for (int k2 = 0; k2 < CR; k2++) {
                if (k2 * 256 >= 3 * nk) break;  // uniform
                const int e = k2 * 256 + (int)threadIdx.x;
                const AdRec d = ad_unpack(cv[k2]);
                const int sib = 1 + e / nk, k = e - (sib - 1) * nk;
                const int ky = cky0 + k / nkx, kx = ckx0 + k % nkx;
                // taps of the block's pixels: [k bs + i, k bs + bs + i] per axis, clamped
                const int xlo = lf_clampi(kx * g.bs + d.ix, 0, g.w - 1);
                const int xhi = lf_clampi(kx * g.bs + g.bs + d.ix, 0, g.w - 1);
                const int ylo = lf_clampi(ky * g.bs + d.iy, 0, g.h - 1);
                const int yhi = lf_clampi(ky * g.bs + g.bs + d.iy, 0, g.h - 1);
                const bool keep = cok[k2] && d.sg != 0 && xlo <= tx1 && xhi >= tx0 && ylo <= ty1 && yhi >= ty0;
                const uint64_t m = __ballot(keep);
                if (lane == 0) wcount[wv] = __popcll(m);
                __syncthreads();
                int pos = n_list;
                for (int q = 0; q < wv; q++) pos += wcount[q];
                pos += (int)__builtin_amdgcn_mbcnt_hi((uint32_t)(m >> 32), __builtin_amdgcn_mbcnt_lo((uint32_t)m, 0u));
                if (keep) {
                    const int at = (sib << 28) | (ky << 14) | kx;
                    if (windowed) {
                        const float sg = (float)d.sg, gx = 1.0f - d.fx, gy = 1.0f - d.fy;
                        lst_a[pos] = make_int4(kx * g.bs + d.ix, ky * g.bs + d.iy,
                                               (sib - 1) * wa - (d.iy + wy0) * ww - (d.ix + wx0), at);
                        lst_b[pos] = make_int4(__float_as_int(sg * (gy * gx)), __float_as_int(sg * (gy * d.fx)),
                                               __float_as_int(sg * (d.fy * gx)), __float_as_int(sg * (d.fy * d.fx)));
                    } else {
                        lst_a[pos] = cv[k2];
                        lst_b[pos] = make_int4(at, 0, 0, 0);
                    }
                }
                for (int q = 0; q < 4; q++) n_list += wcount[q];
                __syncthreads();  // wcount is rewritten by the next round; lists and window complete
            }
        }
#pragma unroll
        for (int kp = 0; kp < AD_PPT; kp++) {
        const int Y = Y0 + kp * RSTEP;
        if (X <= tx1 && Y <= ty1) {
            float acc = own_g[kp];
            if (windowed && X > 0 && X < g.w - 1 && Y > 0 && Y < g.h - 1) {
                // away from the image border each tap (oy, ox) landing on the
                // pixel comes from source pixel (Y - iy - oy, X - ix - ox) alone,
                // when it lies in the block: the same products, in the same
                // order, as the general form
                const int base = Y * ww + X;
                for (int i = 0; i < n_list; i++) {
                    const int4 e = lst_a[i];
                    const int dx = X - e.x, dy = Y - e.y;
                    const bool x0 = (unsigned)dx < (unsigned)g.bs, x1 = (unsigned)(dx - 1) < (unsigned)g.bs;
                    const bool y0 = (unsigned)dy < (unsigned)g.bs, y1 = (unsigned)(dy - 1) < (unsigned)g.bs;
                    if (!((x0 || x1) && (y0 || y1))) continue;
                    const int4 wb = lst_b[i];
                    const float* src = win + base + e.z;
                    float blk = 0.0f;
                    if (y0 && x0) blk = fmaf(__int_as_float(wb.x), src[0], blk);
                    if (y0 && x1) blk = fmaf(__int_as_float(wb.y), src[-1], blk);
                    if (y1 && x0) blk = fmaf(__int_as_float(wb.z), src[-ww], blk);
                    if (y1 && x1) blk = fmaf(__int_as_float(wb.w), src[-ww - 1], blk);
                    acc += blk;
                }
            } else if (staged) {
                for (int i = 0; i < n_list; i++) {
                    const int at = windowed ? lst_a[i].w : lst_b[i].x;
                    const int sib = at >> 28, ky = (at >> 14) & 0x3FFF, kx = at & 0x3FFF;
                    const int B = Br + (sib >> 1), A = Ar + (sib & 1);
                    if (windowed) {  // a border pixel
                        const AdRec d = ad_unpack(brec[ad_record(g, c, l, B, A, ky * g.nbx + kx)]);
                        const float* ws = win + (sib - 1) * wa - wy0 * ww - wx0;
                        acc = ad_block_pull(g, [&](int y, int x) { return ws[y * ww + x]; }, X, Y, ky, kx, d, acc);
                    } else {
                        const AdRec d = ad_unpack(lst_a[i]);
                        const float* gp =
                            gres + ((int64_t)c * g.n_nodes + g.node_base[l] + B * g.na_l[l] + A) * plane;
                        acc = ad_block_pull(g, [&](int y, int x) { return gp[y * g.w + x]; }, X, Y, ky, kx, d, acc);
                    }
                }
            } else {
                acc = ad_pull(g, gres, c, l, Br, Ar, X, Y, reach, max(0, (Y - reach) / g.bs),
                              min(nby - 1, (Y + reach) / g.bs), max(0, (X - reach) / g.bs),
                              min(g.nbx - 1, (X + reach) / g.bs),
                              [&](int, int B, int A, int ky, int kx) {
                                  return ad_unpack(brec[ad_record(g, c, l, B, A, ky * g.nbx + kx)]);
                              },
                              acc);
            }
            gres[own0 + (int64_t)Y * g.w] = acc;
        }
        }
        __syncthreads();  // lists and window are rewritten for the next tile
    }
}

// shift gradients: one wave64 per motion record (four per workgroup), each
// lane summing its pixels in order, then a fixed butterfly across the wave
__global__ void __launch_bounds__(256) k_ad_shift(LfGeom g, LfPtrs p, const float* __restrict__ res,
                                                  const float2* __restrict__ shift, const float* __restrict__ gres_pred,
                                                  float2* __restrict__ gshift, int64_t n_rec)
{
    const int64_t rec = (int64_t)blockIdx.x * 4 + (threadIdx.x >> 6);
    const int lane = threadIdx.x & 63;
    if (rec >= n_rec) return;  // uniform per wave
    int c = 0, l = g.H - 1;
    while (c < 2 && rec >= g.rec_base[c + 1][g.H - 1]) c++;
    while (l > 0 && rec >= g.rec_base[c][l - 1]) l--;
    const int64_t j = rec - g.rec_base[c][l];
    const int pord = (int)(j / g.nblk), blk = (int)(j % g.nblk);
    // invert the predictive ordinal: rows with odd B hold na_l nodes, even rows na_l / 2
    const int na = g.na_l[l], pair = na + na / 2;
    int B = 2 * (pord / pair), rem = pord % pair, A;
    if (rem < na / 2) {
        A = 2 * rem + 1;
    } else {
        B += 1;
        A = rem - na / 2;
    }
    const int64_t plane = (int64_t)g.w * g.h;
    int mx, my, sg;
    lf_motion(g, p, c, l, (uint32_t)j, mx, my, sg);
    float sx = 0.0f, sy = 0.0f;
    if (sg) {
        const float2 d = shift[rec];
        const float fdx = floorf(d.x), fdy = floorf(d.y);
        const float fx = d.x - fdx, fy = d.y - fdy;
        const float* R = res + ((int64_t)c * g.n_nodes + g.node_base[l] + (B & ~1) * na + (A & ~1)) * plane;
        const float* gp = gres_pred + ((int64_t)c * g.n_nodes + g.node_base[l] + B * na + A) * plane;
        const int by0 = (blk / g.nbx) * g.bs, bx0 = (blk % g.nbx) * g.bs;
        for (int q = lane; q < g.bs * g.bs; q += 64) {
            const int y = by0 + q / g.bs, x = bx0 + q % g.bs;
            const int x0 = x + (int)fdx, y0 = y + (int)fdy;
            const int xa = lf_clampi(x0, 0, g.w - 1), xb = lf_clampi(x0 + 1, 0, g.w - 1);
            const int ya = lf_clampi(y0, 0, g.h - 1), yb = lf_clampi(y0 + 1, 0, g.h - 1);
            const float t00 = R[ya * g.w + xa], t01 = R[ya * g.w + xb], t10 = R[yb * g.w + xa], t11 = R[yb * g.w + xb];
            const float gv = (float)sg * gp[y * g.w + x];
            sx = fmaf(gv, (1.0f - fy) * (t01 - t00) + fy * (t11 - t10), sx);
            sy = fmaf(gv, (1.0f - fx) * (t10 - t00) + fx * (t11 - t01), sy);
        }
    }
#pragma unroll
    for (int o = 32; o >= 1; o >>= 1) {
        sx += __shfl_xor(sx, o, 64);
        sy += __shfl_xor(sy, o, 64);
    }
    if (lane == 0) gshift[rec] = make_float2(sx, sy);
}

extern "C" lf_status lf_render_backward(const lf_handle* h, const float* d_residual, const float* d_shift,
                                        const float* d_cams, int32_t n_views, int32_t width, int32_t height,
                                        const float* d_grad_out, float* d_grad_residual, float* d_grad_shift,
                                        void* d_workspace, int64_t workspace_bytes, void* stream)
{
    if (!h || !d_residual || !d_shift || !d_cams || !d_grad_out || !d_grad_residual || !d_grad_shift || !d_workspace ||
        n_views < 1 || width < 1 || height < 1)
        return lf_fail(LF_EINVAL, "bad argument");
    if (lf_status cs = lf_require_full_chroma(h, "lf_render_backward")) return cs;
    const LfGeom& g = h->L.g;
    BwdLayout Bl;
    lf_status st = bwd_layout(h, n_views, width, height, &Bl);
    if (st != LF_OK) return st;
    if (workspace_bytes < Bl.total)
        return lf_fail(LF_ENOMEM, "workspace of %lld bytes, %lld needed", (long long)workspace_bytes, (long long)Bl.total);
    if (((uintptr_t)d_workspace) & 255) return lf_fail(LF_EINVAL, "workspace must be 256-byte aligned");
    hipStream_t s = (hipStream_t)stream;
    uint8_t* W = (uint8_t*)d_workspace;
    uint32_t *kin = (uint32_t*)(W + Bl.o_kin), *kout = (uint32_t*)(W + Bl.o_kout);
    uint32_t *vin = (uint32_t*)(W + Bl.o_vin), *vout = (uint32_t*)(W + Bl.o_vout);
    float* mxs = (float*)(W + Bl.o_max);
    float4* rayf = (float4*)(W + Bl.o_rayf);
    const int64_t rays = (int64_t)n_views * width * height;
    hipLaunchKernelGGL(k_ad_records, dim3((unsigned)((rays + 255) / 256)), dim3(256), 0, s, g, d_cams, n_views,
                       width, height, kin, vin, rayf);
    size_t sb = Bl.sort_bytes;
    if (hipcub::DeviceRadixSort::SortPairs(W + Bl.o_sort, sb, kin, kout, vin, vout, (int)Bl.n_recs, 0, Bl.end_bit, s) !=
        hipSuccess)
        return lf_fail(LF_EDEVICE, "radix sort failed");
    uint32_t* start = (uint32_t*)(W + Bl.o_start);
    hipLaunchKernelGGL(k_ad_nostart, dim3(4096), dim3(256), 0, s, start, Bl.n_samples);
    hipLaunchKernelGGL(k_ad_heads, dim3((unsigned)((Bl.n_recs + 255) / 256)), dim3(256), 0, s, kout, Bl.n_recs, start);
    // level-0 node planes of each channel, every sample written
    const int64_t plane = (int64_t)g.w * g.h, cstride = (int64_t)g.n_nodes * plane;
    float* g0 = d_grad_residual + (int64_t)g.node_base[0] * plane;
    hipLaunchKernelGGL(k_ad_samples, dim3((unsigned)((Bl.n_samples + 255) / 256)), dim3(256), 0, s, rayf, width, height,
                       d_grad_out, kout, vout, start, Bl.n_recs, Bl.n_samples, g.w, g.h, cstride, g0);
    for (int l = 1; l < g.H; l++)
        hipLaunchKernelGGL(k_ad_tree, dim3(8192), dim3(256), 0, s, g, l, d_grad_residual);
    float* parts = (float*)(W + Bl.o_parts);
    hipLaunchKernelGGL(k_ad_maxshift, dim3(AD_MAX_PARTS), dim3(256), 0, s, (const float2*)d_shift, h->L.n_rec, parts);
    hipLaunchKernelGGL(k_ad_maxparts, dim3(1), dim3(256), 0, s, parts, AD_MAX_PARTS, mxs);
    // shift gradients read the predictive nodes' gradients, which the
    // reference pass leaves untouched; run them first to keep the order plain
    if (h->L.n_rec > 0)
        hipLaunchKernelGGL(k_ad_shift, dim3((unsigned)((h->L.n_rec + 3) / 4)), dim3(256), 0, s, g, h->p, d_residual,
                           (const float2*)d_shift, d_grad_residual, (float2*)d_grad_shift, h->L.n_rec);
    {
        const int64_t n_tiles = 3 * (int64_t)g.n_refs * ((g.w + AD_TILE - 1) / AD_TILE) * ((g.h + AD_TILE - 1) / AD_TILE);
        int4* brec = (int4*)(W + Bl.o_brec);
        if (h->L.n_rec > 0)
            hipLaunchKernelGGL(k_ad_blockrec, dim3((unsigned)((h->L.n_rec + 255) / 256)), dim3(256), 0, s, g, h->p,
                               (const float2*)d_shift, h->L.n_rec, brec);
        hipLaunchKernelGGL(k_ad_reference, dim3((unsigned)std::min<int64_t>(std::max<int64_t>(n_tiles, 1), 65536)),
                           dim3(256), 0, s, g, (const int4*)brec, mxs, d_grad_residual);
    }
    return lf_check_launch("render_backward");
}
