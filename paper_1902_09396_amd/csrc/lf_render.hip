// Novel-view rendering fused with random-access decoding.
//
// Two kernels compute the same image bit for bit:
//  - k_render_rays: one thread per ray; each ray walks the tree paths of its
//    16 neighbouring samples (the simple reference path, and the fallback for
//    footprints beyond the staging budget);
//  - k_render_batch: a workgroup renders one screen tile for a group of
//    consecutive views.  It decodes the union footprint of those views once:
//    per-block descriptors (table entry, motion vector, reference plane) are
//    staged in LDS, every tree node above the leaf views that the footprint
//    reaches is decoded once per pixel (ancestor deduplication), and each
//    (view, pixel) sample is assembled once as RGBA8 in LDS.  The rays then
//    blend from LDS.
// Blending works on unscaled 8-bit values and scales by 1/255 at the end.
#include <hip/hip_runtime.h>

#include <cstdlib>

#include "lf_internal.h"

__device__ __forceinline__ float lf_lerp(float p, float q, float f) { return fmaf(f, q - p, p); }

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

// quadrilinear blend of 16 samples given as unscaled 8-bit values; order s, t, u, v
__device__ __forceinline__ float lf_blend16(const float (&sm)[16], const Ray& r)
{
    float vw[4];
#pragma unroll
    for (int q = 0; q < 4; q++)
        vw[q] = lf_lerp(lf_lerp(sm[4 * q], sm[4 * q + 1], r.fs), lf_lerp(sm[4 * q + 2], sm[4 * q + 3], r.fs), r.ft);
    return lf_lerp(lf_lerp(vw[0], vw[1], r.fu), lf_lerp(vw[2], vw[3], r.fu), r.fv) * (1.0f / 255.0f);
}

// ---------------------------------------------------------------------------
// per-ray reference path
// ---------------------------------------------------------------------------

__device__ inline void lf_render_one(const LfGeom& g, const LfPtrs& p, const float* __restrict__ cam, int i, int j,
                                     float out[3])
{
    const Ray r = lf_ray_setup(g, cam, i, j);
    uint32_t px[16];
#pragma unroll
    for (int k = 0; k < 16; k++) {
        const int b = (k & 8) ? r.b1 : r.b0, a = (k & 4) ? r.a1 : r.a0;
        const int y = (k & 2) ? r.y1 : r.y0, x = (k & 1) ? r.x1 : r.x0;
        int Y = lf_decode_channel(g, p, 0, b, a, y, x);
        int Co = lf_decode_channel(g, p, 1, b, a, y, x);
        int Cg = lf_decode_channel(g, p, 2, b, a, y, x);
        int R, G, B;
        lf_ycocg_to_rgb(Y, Co, Cg, R, G, B);
        px[k] = (uint32_t)R | ((uint32_t)G << 8) | ((uint32_t)B << 16);
    }
#pragma unroll
    for (int c = 0; c < 3; c++) {
        float sm[16];
#pragma unroll
        for (int k = 0; k < 16; k++) sm[k] = (float)((px[k] >> (8 * c)) & 255u);
        out[c] = lf_blend16(sm, r);
    }
}

__global__ void __launch_bounds__(256) k_render_rays(LfGeom g, LfPtrs p, const float* __restrict__ cams, int nv,
                                                     int wo, int ho, float* __restrict__ out)
{
    const int64_t npix = (int64_t)wo * ho;
    const int64_t r = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (r >= npix * nv) return;
    const int v = (int)(r / npix);
    const int64_t px = r - (int64_t)v * npix;
    const int j = (int)(px / wo), i = (int)(px % wo);
    float o[3];
    lf_render_one(g, p, cams + 18 * v, i, j, o);
#pragma unroll
    for (int c = 0; c < 3; c++) out[((int64_t)v * 3 + c) * npix + px] = o[c];
}

lf_status lf_launch_render_rays(const lf_handle* h, const float* d_cams, int nv, int wo, int ho, float* d_out,
                                hipStream_t s)
{
    int64_t total = (int64_t)nv * wo * ho;
    int64_t blocks = (total + 255) / 256;
    if (blocks > 0x7FFFFFFF) return lf_fail(LF_EINVAL, "too many rays");
    hipLaunchKernelGGL(k_render_rays, dim3((unsigned)blocks), dim3(256), 0, s, h->L.g, h->p, d_cams, nv, wo, ho,
                       d_out);
    return lf_check_launch("render_rays");
}

// ---------------------------------------------------------------------------
// batched tile renderer
// ---------------------------------------------------------------------------

#define TW 32
#define TH 8
#define NT (TW * TH)
#define FMAX 16          // views per workgroup (upper bound of the group size)
#define MODE_PLANE 0xFE  // descriptor of a reference node: read its resident plane

// Staging budgets (entries) for a group of `fpg` views of one 32x8 tile; the
// footprint of one 512x512 orbit view is 33x9 pixels in about 2x2 views.
struct Budget {
    int rgba, sval, desc;
};

__host__ __device__ inline Budget lf_budget(int fpg)
{
    if (fpg <= 1) return Budget{2048, 4096, 192};
    if (fpg == 2) return Budget{2560, 6144, 256};
    if (fpg <= 4) return Budget{3584, 10240, 352};
    if (fpg <= 8) return Budget{5120, 16384, 512};
    return Budget{8192, 28672, 768};
}

__host__ __device__ inline size_t lf_lds_bytes(Budget b)
{
    return (size_t)b.desc * 16 + (size_t)b.rgba * 4 + (size_t)b.sval * 2;
}

__device__ __forceinline__ int wave_min(int v)
{
#pragma unroll
    for (int o = 32; o > 0; o >>= 1) v = min(v, __shfl_xor(v, o, 64));
    return v;
}

__device__ __forceinline__ int wave_max(int v)
{
#pragma unroll
    for (int o = 32; o > 0; o >>= 1) v = max(v, __shfl_xor(v, o, 64));
    return v;
}

// Block descriptor: x = payload word, y = min (16) | step (13) << 16 | phase code << 29,
// z = mx (12, signed) | my (12, signed) << 12 | mode << 24, w = plane offset (elements)
// of the reference plane (predictive node) or of the node's own plane (reference node).
__device__ __forceinline__ uint4 lf_make_desc(const LfGeom& g, const LfPtrs& p, int c, int l, int B, int A, int blk)
{
    const uint32_t plane = (uint32_t)(g.w * g.h);
    const uint32_t ref = (uint32_t)(c * g.n_refs + g.ref_base[l] + (B >> 1) * g.na_l[l + 1] + (A >> 1)) * plane;
    if (!((A | B) & 1)) return make_uint4(0u, 0u, (uint32_t)MODE_PLANE << 24, ref);
    const int node = g.node_base[l] + B * g.na_l[l] + A;
    const uint2 e = p.table[((size_t)c * g.n_nodes + node) * g.nblk + blk];
    int mx, my, sg;
    lf_motion(g, p, c, l, (uint32_t)(pred_ordinal(g.na_l[l], B, A) * g.nblk + blk), mx, my, sg);
    const uint32_t mode = (e.y >> 16) & 0xFFu;
    const uint32_t code = sg == 1 ? 0u : (sg == -1 ? 1u : 2u);
    return make_uint4(e.x, (e.y & 0xFFFFu) | ((uint32_t)g.step[l] << 16) | (code << 29),
                      ((uint32_t)mx & 0xFFFu) | (((uint32_t)my & 0xFFFu) << 12) | (mode << 24), ref);
}

// SRV value at (y, x) of the node a descriptor belongs to.
__device__ __forceinline__ int lf_srv_from_desc(const LfGeom& g, const LfPtrs& p, uint4 d, int y, int x)
{
    const int mode = (int)(d.z >> 24);
    if (mode == MODE_PLANE) return p.refs[d.w + (uint32_t)(y * g.w + x)];
    int r = 0;
    if (mode != LF_MODE_ZERO) {
        const int i = (y % g.bs) * g.bs + (x % g.bs);
        const int mn = (int)(int16_t)(d.y & 0xFFFFu);
        const int step = (int)((d.y >> 16) & 0x1FFFu);
        r = (mn + (int)lf_bise_get(p.payload + d.x, mode, (uint32_t)i)) * step;
    }
    const uint32_t code = d.y >> 29;
    if (code < 2u) {
        const int mx = ((int)(d.z << 20)) >> 20, my = ((int)(d.z << 8)) >> 20;
        const int q = lf_qpel(p.refs + d.w, g.w, g.h, y, x, mx, my);
        r += code == 0u ? q : -q;
    }
    return r;
}

struct Box {
    int amin, amax, bmin, bmax, xmin, xmax, ymin, ymax;
};

struct LevelInfo {
    int B0, nB, A0, nA, sbase, dbase;
};

struct Plan {
    int nva, nvb, sx, sy, npix, nviews;
    int bkx0, bky0, nbkx, nbk;
    int nslots, ndesc;
    bool fits;
};

__device__ __forceinline__ Plan lf_plan(const LfGeom& g, const Box& b, const Budget& bud, LevelInfo* lv /* may be null */)
{
    Plan P;
    P.nva = b.amax - b.amin + 1;
    P.nvb = b.bmax - b.bmin + 1;
    P.sx = b.xmax - b.xmin + 1;
    P.sy = b.ymax - b.ymin + 1;
    P.npix = P.sx * P.sy;
    P.nviews = P.nva * P.nvb;
    P.bkx0 = b.xmin / g.bs;
    P.bky0 = b.ymin / g.bs;
    P.nbkx = b.xmax / g.bs - P.bkx0 + 1;
    P.nbk = P.nbkx * (b.ymax / g.bs - P.bky0 + 1);
    // staged values: nodes of levels 1..H-1 and the root views (level H), per
    // channel and footprint pixel; descriptors: levels 0..H-1, per block
    int ns = 0, nd = 0;
    for (int l = 0; l <= g.H; l++) {
        const int B0 = b.bmin >> l, A0 = b.amin >> l;
        const int nB = (b.bmax >> l) - B0 + 1, nA = (b.amax >> l) - A0 + 1;
        if (lv) lv[l] = LevelInfo{B0, nB, A0, nA, ns, nd};
        if (l >= 1) ns += 3 * nB * nA;
        if (l < g.H) nd += 3 * nB * nA * P.nbk;
    }
    P.nslots = ns;
    P.ndesc = nd;
    P.fits = (int64_t)P.nviews * P.npix <= bud.rgba && (int64_t)ns * P.npix <= bud.sval && nd <= bud.desc;
    return P;
}

__global__ void __launch_bounds__(NT) k_render_batch(LfGeom g, LfPtrs p, const float* __restrict__ cams, int nv,
                                                     int wo, int ho, int tiles_x, int tiles_y, int fpg,
                                                     float* __restrict__ out)
{
    extern __shared__ uint4 lds_dyn[];
    const Budget bud = lf_budget(fpg);
    uint4* desc = lds_dyn;                                   // [bud.desc]
    uint32_t* rgba = reinterpret_cast<uint32_t*>(desc + bud.desc);  // [bud.rgba]
    int16_t* sval = reinterpret_cast<int16_t*>(rgba + bud.rgba);    // [bud.sval]
    __shared__ int fbox[FMAX][8];
    __shared__ int red[FMAX][8][NT / 64];
    __shared__ LevelInfo lvl[LF_MAX_LEVELS + 1];

    // XCD-aware order: workgroup ids go round-robin over the 8 XCDs, so give
    // each XCD a contiguous range of (view group, tile) work: consecutive
    // views and neighbouring tiles share stream data in that XCD's L2.
    const int n_groups_v = (nv + fpg - 1) / fpg;
    const int64_t n_work = (int64_t)tiles_x * tiles_y * n_groups_v;
    const int64_t per_xcd = (n_work + 7) / 8;
    const int64_t work = (int64_t)(blockIdx.x & 7) * per_xcd + (blockIdx.x >> 3);
    if (work >= n_work) return;  // uniform per workgroup
    const int vg = (int)(work / ((int64_t)tiles_x * tiles_y));
    const int tt = (int)(work - (int64_t)vg * tiles_x * tiles_y);
    const int tyi = tt / tiles_x, txi = tt - tyi * tiles_x;
    const int v0 = vg * fpg, nf = min(fpg, nv - v0);
    const int lx = threadIdx.x % TW, ly = threadIdx.x / TW;
    const int i = txi * TW + lx, j = tyi * TH + ly;
    const bool live = i < wo && j < ho;
    const int ii = live ? i : txi * TW, jj = live ? j : tyi * TH;  // dead lanes repeat the tile origin
    const int wid = threadIdx.x >> 6, lane = threadIdx.x & 63;

    // phase 0: footprint box of every view of the group
    for (int f = 0; f < nf; f++) {
        const Ray r = lf_ray_setup(g, cams + 18 * (v0 + f), ii, jj);
        int m[8] = {wave_min(r.a0), wave_max(r.a1), wave_min(r.b0), wave_max(r.b1),
                    wave_min(r.x0), wave_max(r.x1), wave_min(r.y0), wave_max(r.y1)};
        if (lane == 0)
#pragma unroll
            for (int k = 0; k < 8; k++) red[f][k][wid] = m[k];
    }
    __syncthreads();
    if ((int)threadIdx.x < nf * 8) {
        const int f = threadIdx.x >> 3, k = threadIdx.x & 7;
        int v = red[f][k][0];
#pragma unroll
        for (int w = 1; w < NT / 64; w++) v = (k & 1) ? max(v, red[f][k][w]) : min(v, red[f][k][w]);
        fbox[f][k] = v;
    }
    __syncthreads();

    const int64_t npix_out = (int64_t)wo * ho;
    int f = 0;
    while (f < nf) {
        // greedily grow the group of views while the union footprint fits
        Box bx{fbox[f][0], fbox[f][1], fbox[f][2], fbox[f][3], fbox[f][4], fbox[f][5], fbox[f][6], fbox[f][7]};
        int n = 1;
        while (f + n < nf) {
            const int q = f + n;
            Box u{min(bx.amin, fbox[q][0]), max(bx.amax, fbox[q][1]), min(bx.bmin, fbox[q][2]), max(bx.bmax, fbox[q][3]),
                  min(bx.xmin, fbox[q][4]), max(bx.xmax, fbox[q][5]), min(bx.ymin, fbox[q][6]), max(bx.ymax, fbox[q][7])};
            if (!lf_plan(g, u, bud, nullptr).fits) break;
            bx = u;
            n++;
        }
        if (threadIdx.x == 0) lf_plan(g, bx, bud, lvl);
        const Plan P = lf_plan(g, bx, bud, nullptr);
        __syncthreads();
        if (!P.fits) {
            // a single view whose footprint is too large: per-ray decoding
            float o[3];
            lf_render_one(g, p, cams + 18 * (v0 + f), ii, jj, o);
            if (live)
#pragma unroll
                for (int c = 0; c < 3; c++) out[((int64_t)(v0 + f) * 3 + c) * npix_out + (int64_t)j * wo + i] = o[c];
            f += 1;
            continue;
        }
        // phase 1a: block descriptors of every node of every level in the box
        for (int d = threadIdx.x; d < P.ndesc; d += NT) {
            int l = 0;
            while (l + 1 < g.H && d >= lvl[l + 1].dbase) l++;
            const LevelInfo L = lvl[l];
            int loc = d - L.dbase;
            const int kb = loc % P.nbk;
            loc /= P.nbk;
            const int ai = loc % L.nA;
            loc /= L.nA;
            const int bi = loc % L.nB, c = loc / L.nB;
            const int blk = (P.bky0 + kb / P.nbkx) * g.nbx + P.bkx0 + kb % P.nbkx;
            desc[d] = lf_make_desc(g, p, c, l, L.B0 + bi, L.A0 + ai, blk);
        }
        __syncthreads();
        // phase 1b: values shared by several views, once per node and pixel:
        // SRVs of levels 1..H-1 and the root RKV (level H)
        {
            const int total = P.nslots * P.npix;
            auto stage = [&](int it) -> int {
                const int slot = it / P.npix, px = it - slot * P.npix;
                int l = 1;
                while (l < g.H && slot >= lvl[l + 1].sbase) l++;
                const LevelInfo L = lvl[l];
                const int node_c = slot - L.sbase;  // (c * nB + bi) * nA + ai
                const int y = bx.ymin + px / P.sx, x = bx.xmin + px % P.sx;
                if (l == g.H) {
                    const int ai = node_c % L.nA, rest = node_c / L.nA;
                    const int bi = rest % L.nB, c = rest / L.nB;
                    return p.root[((size_t)(c * g.root_nb + L.B0 + bi) * g.root_na + L.A0 + ai) * (size_t)(g.w * g.h) +
                                  y * g.w + x];
                }
                const int kb = (y / g.bs - P.bky0) * P.nbkx + (x / g.bs - P.bkx0);
                return lf_srv_from_desc(g, p, desc[L.dbase + node_c * P.nbk + kb], y, x);
            };
            // two independent items per trip keep more loads in flight
            for (int it = threadIdx.x; it < total; it += 2 * NT) {
                const int it2 = it + NT;
                const int v1 = stage(it);
                const int v2 = it2 < total ? stage(it2) : 0;
                sval[it] = (int16_t)v1;
                if (it2 < total) sval[it2] = (int16_t)v2;
            }
        }
        __syncthreads();
        // phase 2: every (view, pixel) sample: level-0 SRV + staged ancestors and root
        {
            const int total = P.nviews * P.npix;
            auto assemble = [&](int it) -> uint32_t {
                const int vi = it / P.npix, px = it - vi * P.npix;
                const int b = bx.bmin + vi / P.nva, a = bx.amin + vi % P.nva;
                const int y = bx.ymin + px / P.sx, x = bx.xmin + px % P.sx;
                const int kb = (y / g.bs - P.bky0) * P.nbkx + (x / g.bs - P.bkx0);
                const LevelInfo L0 = lvl[0];
                int ch[3];
#pragma unroll
                for (int c = 0; c < 3; c++) {
                    int v = lf_srv_from_desc(g, p, desc[((c * L0.nB + (b - L0.B0)) * L0.nA + (a - L0.A0)) * P.nbk + kb], y, x);
                    for (int l = 1; l <= g.H; l++) {
                        const LevelInfo L = lvl[l];
                        v += sval[(L.sbase + (c * L.nB + ((b >> l) - L.B0)) * L.nA + ((a >> l) - L.A0)) * P.npix + px];
                    }
                    ch[c] = v;
                }
                int R, G, B;
                lf_ycocg_to_rgb(ch[0], ch[1], ch[2], R, G, B);
                return (uint32_t)R | ((uint32_t)G << 8) | ((uint32_t)B << 16);
            };
            for (int it = threadIdx.x; it < total; it += 2 * NT) {
                const int it2 = it + NT;
                const uint32_t v1 = assemble(it);
                const uint32_t v2 = it2 < total ? assemble(it2) : 0u;
                rgba[it] = v1;
                if (it2 < total) rgba[it2] = v2;
            }
        }
        __syncthreads();
        // phase 3: blend every ray of the group's views
        for (int q = f; q < f + n; q++) {
            const Ray r = lf_ray_setup(g, cams + 18 * (v0 + q), ii, jj);
            uint32_t s16[16];
#pragma unroll
            for (int k = 0; k < 16; k++) {
                const int b = (k & 8) ? r.b1 : r.b0, a = (k & 4) ? r.a1 : r.a0;
                const int y = (k & 2) ? r.y1 : r.y0, x = (k & 1) ? r.x1 : r.x0;
                s16[k] = rgba[((b - bx.bmin) * P.nva + (a - bx.amin)) * P.npix + (y - bx.ymin) * P.sx + (x - bx.xmin)];
            }
            if (live) {
#pragma unroll
                for (int c = 0; c < 3; c++) {
                    float sm[16];
#pragma unroll
                    for (int k = 0; k < 16; k++) sm[k] = (float)((s16[k] >> (8 * c)) & 255u);
                    out[((int64_t)(v0 + q) * 3 + c) * npix_out + (int64_t)j * wo + i] = lf_blend16(sm, r);
                }
            }
        }
        __syncthreads();  // LDS is reused by the next group of views
        f += n;
    }
}

static int frames_per_group()
{
    static int fpg = [] {
        const char* e = getenv("HMLFC_VIEWS_PER_GROUP");
        int v = e ? atoi(e) : 8;
        return v < 1 ? 1 : (v > FMAX ? FMAX : v);
    }();
    return fpg;
}

lf_status lf_launch_render_batch(const lf_handle* h, const float* d_cams, int nv, int wo, int ho, float* d_out,
                                 hipStream_t s)
{
    const int tx = (wo + TW - 1) / TW, ty = (ho + TH - 1) / TH;
    const int fpg = frames_per_group();
    const int64_t n_work = (int64_t)tx * ty * ((nv + fpg - 1) / fpg);
    const int64_t grid = ((n_work + 7) / 8) * 8;
    if (grid > 0x7FFFFFFF) return lf_fail(LF_EINVAL, "too many tiles");
    const size_t lds = lf_lds_bytes(lf_budget(fpg));
    static bool attr_set = false;
    if (lds > 65536 && !attr_set) {
        if (hipFuncSetAttribute((const void*)k_render_batch, hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds) !=
            hipSuccess)
            return lf_fail(LF_EDEVICE, "cannot reserve %zu bytes of LDS", lds);
        attr_set = true;
    }
    hipLaunchKernelGGL(k_render_batch, dim3((unsigned)grid), dim3(NT), lf_lds_bytes(lf_budget(fpg)), s, h->L.g, h->p,
                       d_cams, nv, wo, ho, tx, ty, fpg, d_out);
    return lf_check_launch("render_batch");
}

extern "C" lf_status lf_render_views(const lf_handle* h, const float* d_cams, int32_t n_views, int32_t width,
                                     int32_t height, float* d_out, void* stream)
{
    if (!h || n_views < 0 || width < 1 || height < 1) return lf_fail(LF_EINVAL, "bad argument");
    if (n_views == 0) return LF_OK;
    if (!d_cams || !d_out) return lf_fail(LF_EINVAL, "null buffer");
    return lf_launch_render_batch(h, d_cams, n_views, width, height, d_out, (hipStream_t)stream);
}

extern "C" lf_status lf_render_views_per_ray(const lf_handle* h, const float* d_cams, int32_t n_views, int32_t width,
                                             int32_t height, float* d_out, void* stream)
{
    if (!h || n_views < 0 || width < 1 || height < 1) return lf_fail(LF_EINVAL, "bad argument");
    if (n_views == 0) return LF_OK;
    if (!d_cams || !d_out) return lf_fail(LF_EINVAL, "null buffer");
    return lf_launch_render_rays(h, d_cams, n_views, width, height, d_out, (hipStream_t)stream);
}
