// Novel-view rendering fused with random-access decoding, and the per-view
// footprint accounting used for roofline figures.
#include <hip/hip_runtime.h>

#include <vector>

#include "lf_internal.h"

// ---------------------------------------------------------------------------
// Per-ray renderer: every ray decodes its 16 neighbouring samples along their
// full tree paths and blends them.  Simple and independent of tiling; used
// for rays whose footprint does not fit the tiled kernel's staging.
// ---------------------------------------------------------------------------

__device__ __forceinline__ float lf_lerp(float p, float q, float f) { return fmaf(f, q - p, p); }

__device__ inline void lf_render_one(const LfGeom& g, const LfPtrs& p, const float* __restrict__ cam, int i, int j,
                                     float out[3])
{
    float u, v, s, t;
    lf_ray(cam, i, j, u, v, s, t);
    int a0, a1, b0, b1, x0, x1, y0, y1;
    float fu, fv, fs, ft;
    lf_axis(u, g.na, a0, a1, fu);
    lf_axis(v, g.nb, b0, b1, fv);
    lf_axis(s, g.w, x0, x1, fs);
    lf_axis(t, g.h, y0, y1, ft);
    float view[4][3];
#pragma unroll
    for (int q = 0; q < 4; q++) {
        const int b = (q >> 1) ? b1 : b0, a = (q & 1) ? a1 : a0;
        float smp[4][3];
#pragma unroll
        for (int k = 0; k < 4; k++) {
            const int y = (k >> 1) ? y1 : y0, x = (k & 1) ? x1 : x0;
            int Y = lf_decode_channel(g, p, 0, b, a, y, x);
            int Co = lf_decode_channel(g, p, 1, b, a, y, x);
            int Cg = lf_decode_channel(g, p, 2, b, a, y, x);
            int r, gg, bl;
            lf_ycocg_to_rgb(Y, Co, Cg, r, gg, bl);
            smp[k][0] = (float)r / 255.0f;
            smp[k][1] = (float)gg / 255.0f;
            smp[k][2] = (float)bl / 255.0f;
        }
#pragma unroll
        for (int c = 0; c < 3; c++) {
            float top = lf_lerp(smp[0][c], smp[1][c], fs);
            float bot = lf_lerp(smp[2][c], smp[3][c], fs);
            view[q][c] = lf_lerp(top, bot, ft);
        }
    }
#pragma unroll
    for (int c = 0; c < 3; c++) {
        float r0 = lf_lerp(view[0][c], view[1][c], fu);
        float r1 = lf_lerp(view[2][c], view[3][c], fu);
        out[c] = lf_lerp(r0, r1, fv);
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
// Tiled renderer.  A workgroup renders a TW x TH tile of one view.  It first
// finds the tile's footprint (the box of views and of image pixels its rays
// touch), decodes every sample of that box once into LDS as packed RGBA8,
// then each thread blends its ray's 16 samples from LDS.  Rays of one tile
// share nearly all of their samples, so this replaces 16 tree walks per ray
// by about 5.  A tile whose footprint exceeds the LDS budget falls back to
// per-ray decoding (same arithmetic, same result).
// ---------------------------------------------------------------------------

#define TW 32
#define TH 8
#define TILE_THREADS (TW * TH)
#define FOOT_MAX 6144  // packed samples staged per tile (24 KiB)

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

__global__ void __launch_bounds__(TILE_THREADS) k_render_tiles(LfGeom g, LfPtrs p, const float* __restrict__ cams,
                                                                int nv, int wo, int ho, int tiles_x, int tiles_y,
                                                                float* __restrict__ out)
{
    __shared__ uint32_t foot[FOOT_MAX];
    __shared__ int red[8][TILE_THREADS / 64];
    // XCD-aware order: consecutive workgroup ids go round-robin over the 8
    // XCDs; give each XCD a contiguous range of tiles (neighbouring tiles and
    // consecutive views share stream data in that XCD's L2).
    const int64_t n_tiles = (int64_t)tiles_x * tiles_y * nv;
    const int64_t bid = blockIdx.x;
    const int64_t per_xcd = (n_tiles + 7) / 8;
    const int64_t xcd = bid & 7, slot = bid >> 3;
    const int64_t tile = xcd * per_xcd + slot;
    if (tile >= n_tiles) return;  // uniform per workgroup
    const int v = (int)(tile / ((int64_t)tiles_x * tiles_y));
    const int tt = (int)(tile - (int64_t)v * tiles_x * tiles_y);
    const int tyi = tt / tiles_x, txi = tt - tyi * tiles_x;
    const int lx = threadIdx.x % TW, ly = threadIdx.x / TW;
    const int i = txi * TW + lx, j = tyi * TH + ly;
    const bool live = i < wo && j < ho;
    const float* cam = cams + 18 * v;

    float u, vv, s, t;
    lf_ray(cam, live ? i : txi * TW, live ? j : tyi * TH, u, vv, s, t);
    int a0, a1, b0, b1, x0, x1, y0, y1;
    float fu, fv, fs, ft;
    lf_axis(u, g.na, a0, a1, fu);
    lf_axis(vv, g.nb, b0, b1, fv);
    lf_axis(s, g.w, x0, x1, fs);
    lf_axis(t, g.h, y0, y1, ft);

    // footprint box of the tile (dead lanes repeat the tile's first ray)
    const int wid = threadIdx.x >> 6, lane = threadIdx.x & 63;
    int r0 = wave_min(a0), r1 = wave_max(a1), r2 = wave_min(b0), r3 = wave_max(b1);
    int r4 = wave_min(x0), r5 = wave_max(x1), r6 = wave_min(y0), r7 = wave_max(y1);
    if (lane == 0) {
        red[0][wid] = r0;
        red[1][wid] = r1;
        red[2][wid] = r2;
        red[3][wid] = r3;
        red[4][wid] = r4;
        red[5][wid] = r5;
        red[6][wid] = r6;
        red[7][wid] = r7;
    }
    __syncthreads();
    int amin = red[0][0], amax = red[1][0], bmin = red[2][0], bmax = red[3][0];
    int xmin = red[4][0], xmax = red[5][0], ymin = red[6][0], ymax = red[7][0];
#pragma unroll
    for (int k = 1; k < TILE_THREADS / 64; k++) {
        amin = min(amin, red[0][k]);
        amax = max(amax, red[1][k]);
        bmin = min(bmin, red[2][k]);
        bmax = max(bmax, red[3][k]);
        xmin = min(xmin, red[4][k]);
        xmax = max(xmax, red[5][k]);
        ymin = min(ymin, red[6][k]);
        ymax = max(ymax, red[7][k]);
    }
    const int nva = amax - amin + 1, nvb = bmax - bmin + 1;
    const int sx = xmax - xmin + 1, sy = ymax - ymin + 1;
    const int np = sx * sy;
    const int64_t items = (int64_t)nva * nvb * np;
    float o[3];
    if (items <= FOOT_MAX) {
        // decode the footprint once
        for (int it = threadIdx.x; it < (int)items; it += TILE_THREADS) {
            const int vi = it / np, pi = it - vi * np;
            const int b = bmin + vi / nva, a = amin + vi % nva;
            const int y = ymin + pi / sx, x = xmin + pi % sx;
            int Y = lf_decode_channel(g, p, 0, b, a, y, x);
            int Co = lf_decode_channel(g, p, 1, b, a, y, x);
            int Cg = lf_decode_channel(g, p, 2, b, a, y, x);
            int r, gg, bl;
            lf_ycocg_to_rgb(Y, Co, Cg, r, gg, bl);
            foot[it] = (uint32_t)r | ((uint32_t)gg << 8) | ((uint32_t)bl << 16);
        }
        __syncthreads();
        // blend
        float view[4][3];
#pragma unroll
        for (int q = 0; q < 4; q++) {
            const int b = (q >> 1) ? b1 : b0, a = (q & 1) ? a1 : a0;
            const int base = ((b - bmin) * nva + (a - amin)) * np;
            uint32_t sm[4];
#pragma unroll
            for (int k = 0; k < 4; k++) {
                const int y = (k >> 1) ? y1 : y0, x = (k & 1) ? x1 : x0;
                sm[k] = foot[base + (y - ymin) * sx + (x - xmin)];
            }
#pragma unroll
            for (int c = 0; c < 3; c++) {
                float c00 = (float)((sm[0] >> (8 * c)) & 255u) / 255.0f;
                float c01 = (float)((sm[1] >> (8 * c)) & 255u) / 255.0f;
                float c10 = (float)((sm[2] >> (8 * c)) & 255u) / 255.0f;
                float c11 = (float)((sm[3] >> (8 * c)) & 255u) / 255.0f;
                view[q][c] = lf_lerp(lf_lerp(c00, c01, fs), lf_lerp(c10, c11, fs), ft);
            }
        }
#pragma unroll
        for (int c = 0; c < 3; c++) o[c] = lf_lerp(lf_lerp(view[0][c], view[1][c], fu), lf_lerp(view[2][c], view[3][c], fu), fv);
    } else {
        lf_render_one(g, p, cam, i, j, o);
    }
    if (live) {
        const int64_t npix = (int64_t)wo * ho;
        const int64_t px = (int64_t)j * wo + i;
#pragma unroll
        for (int c = 0; c < 3; c++) out[((int64_t)v * 3 + c) * npix + px] = o[c];
    }
}

lf_status lf_launch_render_tiles(const lf_handle* h, const float* d_cams, int nv, int wo, int ho, float* d_out,
                                 hipStream_t s)
{
    const int tx = (wo + TW - 1) / TW, ty = (ho + TH - 1) / TH;
    const int64_t n_tiles = (int64_t)tx * ty * nv;
    const int64_t grid = ((n_tiles + 7) / 8) * 8;
    if (grid > 0x7FFFFFFF) return lf_fail(LF_EINVAL, "too many tiles");
    hipLaunchKernelGGL(k_render_tiles, dim3((unsigned)grid), dim3(TILE_THREADS), 0, s, h->L.g, h->p, d_cams, nv, wo,
                       ho, tx, ty, d_out);
    return lf_check_launch("render_tiles");
}

extern "C" lf_status lf_render_views(const lf_handle* h, const float* d_cams, int32_t n_views, int32_t width,
                                     int32_t height, float* d_out, void* stream)
{
    if (!h || n_views < 0 || width < 1 || height < 1) return lf_fail(LF_EINVAL, "bad argument");
    if (n_views == 0) return LF_OK;
    if (!d_cams || !d_out) return lf_fail(LF_EINVAL, "null buffer");
    return lf_launch_render_tiles(h, d_cams, n_views, width, height, d_out, (hipStream_t)stream);
}

extern "C" lf_status lf_render_views_per_ray(const lf_handle* h, const float* d_cams, int32_t n_views, int32_t width,
                                             int32_t height, float* d_out, void* stream)
{
    if (!h || n_views < 0 || width < 1 || height < 1) return lf_fail(LF_EINVAL, "bad argument");
    if (n_views == 0) return LF_OK;
    if (!d_cams || !d_out) return lf_fail(LF_EINVAL, "null buffer");
    return lf_launch_render_rays(h, d_cams, n_views, width, height, d_out, (hipStream_t)stream);
}

// ---------------------------------------------------------------------------
// Footprint bytes (see hmlfc.h): mark what one view reads, then weigh it.
// ---------------------------------------------------------------------------

__global__ void k_fill_u8(uint8_t* p, int64_t n)
{
    for (int64_t t = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; t < n; t += (int64_t)gridDim.x * blockDim.x)
        p[t] = 0;
}

__global__ void k_fp_mark(LfGeom g, LfPtrs p, const float* __restrict__ cam, int wo, int ho, uint8_t* __restrict__ pred,
                          uint8_t* __restrict__ ref, uint8_t* __restrict__ root)
{
    const int64_t r = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (r >= (int64_t)wo * ho) return;
    const int j = (int)(r / wo), i = (int)(r % wo);
    float u, v, s, t;
    lf_ray(cam, i, j, u, v, s, t);
    int a0, a1, b0, b1, x0, x1, y0, y1;
    float fu, fv, fs, ft;
    lf_axis(u, g.na, a0, a1, fu);
    lf_axis(v, g.nb, b0, b1, fv);
    lf_axis(s, g.w, x0, x1, fs);
    lf_axis(t, g.h, y0, y1, ft);
    for (int k = 0; k < 16; k++) {
        const int b = (k & 8) ? b1 : b0, a = (k & 4) ? a1 : a0, y = (k & 2) ? y1 : y0, x = (k & 1) ? x1 : x0;
        const int blk = (y / g.bs) * g.nbx + x / g.bs;
        for (int c = 0; c < 3; c++) {
            root[((size_t)(c * g.root_nb + (b >> g.H)) * g.root_na + (a >> g.H)) * g.nblk + blk] = 1;
            for (int l = 0; l < g.H; l++) {
                const int B = b >> l, A = a >> l;
                if (!((A | B) & 1)) {
                    int node = g.node_base[l] + B * g.na_l[l] + A;
                    ref[((size_t)c * g.n_nodes + node) * g.nblk + blk] = 1;
                    continue;
                }
                int node = g.node_base[l] + B * g.na_l[l] + A;
                pred[((size_t)c * g.n_nodes + node) * g.nblk + blk] = 1;
                int mx, my, sg;
                lf_motion(g, p, c, l, (uint32_t)(pred_ordinal(g.na_l[l], B, A) * g.nblk + blk), mx, my, sg);
                if (!sg) continue;
                const int rnode = g.node_base[l] + (B & ~1) * g.na_l[l] + (A & ~1);
                const int X = 4 * x + mx, Y = 4 * y + my;
                const int tx0 = X >> 2, ty0 = Y >> 2, fx = X & 3, fy = Y & 3;
                for (int q = 0; q < 4; q++) {
                    const int dx = q & 1, dy = q >> 1;
                    if ((dx ? fx : 4 - fx) * (dy ? fy : 4 - fy) == 0) continue;
                    const int yy = lf_clampi(ty0 + dy, 0, g.h - 1), xx = lf_clampi(tx0 + dx, 0, g.w - 1);
                    ref[((size_t)c * g.n_nodes + rnode) * g.nblk + (yy / g.bs) * g.nbx + xx / g.bs] = 1;
                }
            }
        }
    }
}

struct FpWeights {
    double mv_bytes[3][LF_MAX_LEVELS];
};

__global__ void __launch_bounds__(256) k_fp_sum(LfGeom g, LfPtrs p, FpWeights wts, const uint8_t* __restrict__ pred,
                                                const uint8_t* __restrict__ ref, const uint8_t* __restrict__ root,
                                                int64_t n_ent, int64_t n_root, double* __restrict__ partial)
{
    __shared__ double red[256];
    double acc = 0.0;
    const double tile = 2.0 * g.bs * g.bs;
    for (int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; e < n_ent + n_root;
         e += (int64_t)gridDim.x * blockDim.x) {
        if (e >= n_ent) {
            if (root[e - n_ent]) acc += tile;
            continue;
        }
        if (ref[e]) acc += tile;
        if (pred[e]) {
            const int node = (int)((e / g.nblk) % g.n_nodes);
            const int c = (int)(e / ((int64_t)g.nblk * g.n_nodes));
            int l = 0;
            while (node < g.node_base[l]) l++;
            uint2 t = p.table[e];
            int mode = (int)((t.y >> 16) & 0xFFu);
            double pay = 0.0;
            if (mode != LF_MODE_ZERO) {
                int fam = mode >> 5, b = mode & 31, n = g.bs * g.bs;
                int64_t bits = fam == 0 ? (int64_t)n * b
                                        : (fam == 1 ? (int64_t)((n + 4) / 5) * (8 + 5 * b) : (int64_t)((n + 2) / 3) * (7 + 3 * b));
                pay = 4.0 * (double)((bits + 31) / 32);
            }
            acc += 8.0 + pay + wts.mv_bytes[c][l];
        }
    }
    red[threadIdx.x] = acc;
    __syncthreads();
    for (int s = 128; s > 0; s >>= 1) {
        if ((int)threadIdx.x < s) red[threadIdx.x] += red[threadIdx.x + s];
        __syncthreads();
    }
    if (threadIdx.x == 0) partial[blockIdx.x] = red[0];
}

extern "C" lf_status lf_footprint_bytes(const lf_handle* h, const float* d_cams, int32_t n_views, int32_t width,
                                        int32_t height, double* host_out, void* stream)
{
    if (!h || !d_cams || !host_out || n_views < 0 || width < 1 || height < 1) return lf_fail(LF_EINVAL, "bad argument");
    const LfGeom& g = h->L.g;
    hipStream_t s = (hipStream_t)stream;
    const int64_t n_ent = 3 * (int64_t)g.n_nodes * g.nblk;
    const int64_t n_root = 3 * (int64_t)g.root_na * g.root_nb * g.nblk;
    const int nblocks = 1024;
    uint8_t* buf = nullptr;
    double* part = nullptr;
    if (hipMalloc(&buf, (size_t)(2 * n_ent + n_root)) != hipSuccess ||
        hipMalloc(&part, sizeof(double) * nblocks) != hipSuccess) {
        if (buf) (void)hipFree(buf);
        return lf_fail(LF_EDEVICE, "footprint scratch allocation failed");
    }
    FpWeights w{};
    for (int c = 0; c < 3; c++)
        for (int l = 0; l < g.H; l++) {
            int64_t cnt = (int64_t)((g.nb_l[l] / 2) * g.na_l[l] + ((g.nb_l[l] + 1) / 2) * (g.na_l[l] / 2)) * g.nblk;
            if (cnt == 0) continue;
            int m = g.mv_mode[c][l], fam = m >> 5, b = m & 31;
            int64_t n = 2 * cnt;
            int64_t bits = fam == 0 ? n * b : (fam == 1 ? (n + 4) / 5 * (8 + 5 * b) : (n + 2) / 3 * (7 + 3 * b));
            w.mv_bytes[c][l] = ((double)bits + 2.0 * cnt) / (8.0 * cnt);
        }
    std::vector<double> hp(nblocks);
    lf_status st = LF_OK;
    for (int v = 0; v < n_views && st == LF_OK; v++) {
        hipLaunchKernelGGL(k_fill_u8, dim3(1024), dim3(256), 0, s, buf, 2 * n_ent + n_root);
        int64_t rays = (int64_t)width * height;
        hipLaunchKernelGGL(k_fp_mark, dim3((unsigned)((rays + 255) / 256)), dim3(256), 0, s, g, h->p, d_cams + 18 * v,
                           width, height, buf, buf + n_ent, buf + 2 * n_ent);
        hipLaunchKernelGGL(k_fp_sum, dim3(nblocks), dim3(256), 0, s, g, h->p, w, buf, buf + n_ent, buf + 2 * n_ent,
                           n_ent, n_root, part);
        st = lf_check_launch("footprint");
        if (st != LF_OK) break;
        if (hipMemcpyAsync(hp.data(), part, sizeof(double) * nblocks, hipMemcpyDeviceToHost, s) != hipSuccess ||
            hipStreamSynchronize(s) != hipSuccess) {
            st = lf_fail(LF_EDEVICE, "footprint readback failed");
            break;
        }
        double tot = 12.0 * (double)rays;
        for (int k = 0; k < nblocks; k++) tot += hp[k];
        host_out[v] = tot;
    }
    (void)hipFree(buf);
    (void)hipFree(part);
    return st;
}
