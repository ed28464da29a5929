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

#include <algorithm>
#include <cstdlib>

#include "lf_render_tile.h"

template <int RES>
__global__ void __launch_bounds__(256) k_render_rays(LfGeom g, LfPtrs p, const float* __restrict__ cams, int nv,
                                                     int wo, int ho, float* __restrict__ out, int lod)
{
    const int64_t npix = (int64_t)wo * ho;
    const int64_t r = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (r >= npix * nv) return;
    const int v = (int)(r / npix);
    const int64_t px = r - (int64_t)v * npix;
    const int j = (int)(px / wo), i = (int)(px % wo);
    float o[3];
    lf_render_one<RES>(g, p, cams + 18 * v, i, j, o, lod);
#pragma unroll
    for (int c = 0; c < 3; c++) out[((int64_t)v * 3 + c) * npix + px] = o[c];
}

// 4:2:0 streams, one thread per ray (lf_render_one420).
__global__ void __launch_bounds__(256) k_render_rays420(LfGeom g, LfPtrs p, LfGeom gc, LfPtrs pc,
                                                        const float* __restrict__ cams, int nv, int wo, int ho,
                                                        float* __restrict__ out, int lod)
{
    const int64_t npix = (int64_t)wo * ho;
    const int64_t r = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (r >= npix * nv) return;
    const int v = (int)(r / npix);
    const int64_t px = r - (int64_t)v * npix;
    const int j = (int)(px / wo), i = (int)(px % wo);
    float o[3];
    lf_render_one420(g, p, gc, pc, cams + 18 * v, i, j, o, lod);
#pragma unroll
    for (int c = 0; c < 3; c++) out[((int64_t)v * 3 + c) * npix + px] = o[c];
}

lf_status lf_launch_render_rays(const lf_handle* h, const float* d_cams, int nv, int wo, int ho, float* d_out,
                                hipStream_t s, int lod = 0)
{
    int64_t total = (int64_t)nv * wo * ho;
    int64_t blocks = (total + 255) / 256;
    if (blocks > 0x7FFFFFFF) return lf_fail(LF_EINVAL, "too many rays");
    if (h->L.chroma420)
        hipLaunchKernelGGL(k_render_rays420, dim3((unsigned)blocks), dim3(256), 0, s, h->L.g, h->p, h->L.gc, h->pc,
                           d_cams, nv, wo, ho, d_out, lod);
    else
        hipLaunchKernelGGL(h->L.sparse == LF_RES_CSR     ? k_render_rays<LF_RES_CSR>
                           : h->L.sparse == LF_RES_TILES ? k_render_rays<LF_RES_TILES>
                                                         : k_render_rays<LF_RES_DENSE>,
                           dim3((unsigned)blocks), dim3(256), 0, s, h->L.g, h->p, d_cams, nv, wo, ho, d_out, lod);
    return lf_check_launch("render_rays");
}

// C420: a 4:2:0 stream, chroma geometry gc, pc (unused otherwise).
template <bool SMALL_BLOCKS, bool C420>
__global__ void __launch_bounds__(NT, 3) k_render_batch(LfGeom g, LfPtrs p, LfGeom gc, LfPtrs pc,
                                                     const float* __restrict__ cams, int nv, int wo, int ho,
                                                     int tiles_x, int tiles_y, int chunk, int fpg, int64_t n_full,
                                                     int split, float* __restrict__ out)
{
    // A workgroup renders one screen tile for a chunk of consecutive views
    // (groups of fpg views, decoded values cached between the groups).
    // XCD-aware order: workgroup ids go round-robin over the 8 XCDs, so give
    // each XCD a contiguous range of (view chunk, tile) work: consecutive
    // views and neighbouring tiles share stream data in that XCD's L2.
    // The first n_full (chunk, tile) items go to one workgroup each; the
    // items after them, which would only part-fill the last round of
    // resident workgroups, are cut into `split` runs of views each.
    const int n_chunks = (nv + chunk - 1) / chunk;
    const int64_t n_work = (int64_t)tiles_x * tiles_y * n_chunks;
    const int64_t ga = (n_full + 7) / 8 * 8;  // workgroups of the whole items
    int64_t work;
    int part = 0;
    if ((int64_t)blockIdx.x < ga) {
        const int64_t per_xcd = ga / 8;
        work = (int64_t)(blockIdx.x & 7) * per_xcd + (blockIdx.x >> 3);
        if (work >= n_full) return;  // uniform per workgroup
    } else {
        const int64_t b = blockIdx.x - ga, n_parts = (n_work - n_full) * split;
        const int64_t per_xcd = (n_parts + 7) / 8;
        const int64_t it = (b & 7) * per_xcd + (b >> 3);
        if (it >= n_parts) return;
        work = n_full + it / split;
        part = (int)(it % split);
    }
    TILE_LDS_DECL
    const int vc = (int)(work / ((int64_t)tiles_x * tiles_y));
    const int tt = (int)(work - (int64_t)vc * tiles_x * tiles_y);
    const int tyi = tt / tiles_x, txi = tt - tyi * tiles_x;
    const int c0 = vc * chunk, c1 = min(nv, c0 + chunk);
    int v0 = c0, nf = c1 - c0;
    if (work >= n_full) {
        const int per = (nf + split - 1) / split;
        v0 = c0 + part * per;
        nf = min(per, c1 - v0);
        if (nf <= 0) return;
    }
    lf_tile_views<false, SMALL_BLOCKS, C420>(g, p, gc, pc, cams, v0, nf, fpg, wo, ho, txi, tyi, out, S);
}

// Per-ray rendering of the (view, tile) pairs the batched kernel marked.
// Workgroup b owns pairs [b * per_wg, (b + 1) * per_wg): it checks up to NT
// of them at once (one per thread), compacts the marked ones, and renders
// them one tile at a time, so a launch whose views are mostly marked (tiles
// far minified) still spreads them over the whole grid.
template <bool C420>
__global__ void __launch_bounds__(NT) k_render_fallback(LfGeom g, LfPtrs p, LfGeom gc, LfPtrs pc,
                                                        const float* __restrict__ cams, int nv, int wo, int ho,
                                                        int tiles_x, int tiles_y, int per_wg, float* __restrict__ out)
{
    __shared__ int marked[NT];
    __shared__ int wcount[NT / 64];
    const int64_t n_pairs = (int64_t)nv * tiles_x * tiles_y;
    const int64_t npix = (int64_t)wo * ho;
    const int64_t begin = (int64_t)blockIdx.x * per_wg;
    const int64_t end = min(begin + per_wg, n_pairs);
    const int wid = threadIdx.x >> 6, lane = threadIdx.x & 63;
    for (int64_t base = begin; base < end; base += NT) {
        const int64_t pr = base + threadIdx.x;
        int mine = 0;
        if (pr < end) {
            const int v = (int)(pr / ((int64_t)tiles_x * tiles_y));
            const int tt = (int)(pr - (int64_t)v * tiles_x * tiles_y);
            const int tyi = tt / tiles_x, txi = tt - tyi * tiles_x;
            mine = __float_as_uint(out[(int64_t)v * 3 * npix + (int64_t)(tyi * TH) * wo + txi * TW]) == FALLBACK_MARK;
        }
        // compact the marked pairs in thread order
        const uint64_t bal = __ballot(mine);
        if (lane == 0) wcount[wid] = __popcll(bal);
        __syncthreads();
        int off = 0, total = 0;
        for (int w = 0; w < NT / 64; w++) {
            off += w < wid ? wcount[w] : 0;
            total += wcount[w];
        }
        if (mine) marked[off + __popcll(bal & ((1ull << lane) - 1ull))] = (int)threadIdx.x;
        __syncthreads();
        for (int k = 0; k < total; k++) {
            const int64_t q = base + marked[k];
            const int v = (int)(q / ((int64_t)tiles_x * tiles_y));
            const int tt = (int)(q - (int64_t)v * tiles_x * tiles_y);
            const int tyi = tt / tiles_x, txi = tt - tyi * tiles_x;
            const int i = txi * TW + (int)threadIdx.x % TW, j = tyi * TH + (int)threadIdx.x / TW;
            if (i < wo && j < ho) {
                float o[3];
                if (C420)
                    lf_render_one420(g, p, gc, pc, cams + 18 * v, i, j, o);
                else
                    lf_render_one(g, p, cams + 18 * v, i, j, o);
#pragma unroll
                for (int c = 0; c < 3; c++) out[((int64_t)v * 3 + c) * npix + (int64_t)j * wo + i] = o[c];
            }
        }
        __syncthreads();  // marked[] and wcount[] are rewritten by the next round
    }
}

static int env_int(const char* name, int dflt, int lo, int hi)
{
    const char* e = getenv(name);
    int v = e ? atoi(e) : dflt;
    return v < lo ? lo : (v > hi ? hi : v);
}

// views per group (decoded together) and per chunk (one workgroup, values
// cached between its groups)
static int frames_per_group()
{
    static int v = env_int("HMLFC_VIEWS_PER_GROUP", 12, 1, FMAX);
    return v;
}
// views per chunk: HMLFC_VIEWS_PER_CHUNK if set, else chunks as long as
// possible while the launch still has about 2048 workgroups (balanced, at
// most FMAX views each)
static int frames_per_chunk(int nv, int tiles)
{
    static int v = env_int("HMLFC_VIEWS_PER_CHUNK", 0, 0, FMAX);
    if (v > 0) return v;
    int64_t n_chunks = std::min<int64_t>(nv, std::max<int64_t>(1, (2048 + tiles - 1) / std::max(tiles, 1)));
    n_chunks = std::max<int64_t>(n_chunks, (nv + FMAX - 1) / FMAX);
    return (int)((nv + n_chunks - 1) / n_chunks);
}

// runs each tail item of the batched launch is cut into
static int tail_split()
{
    static int v = env_int("HMLFC_TAIL_SPLIT", 2, 1, 8);
    return v;
}

// compute units of the current device (cached per device id)
static int device_cus()
{
    static int cus[64] = {};
    int dev = 0;
    if (hipGetDevice(&dev) != hipSuccess || dev < 0 || dev >= 64) return 256;
    if (cus[dev] == 0) {
        int n = 0;
        if (hipDeviceGetAttribute(&n, hipDeviceAttributeMultiprocessorCount, dev) != hipSuccess || n < 1) n = 256;
        cus[dev] = n;
    }
    return cus[dev];
}

extern "C" lf_status lf_get_render_config(int32_t n_views, int32_t width, int32_t height, int32_t* views_per_group,
                                          int32_t* views_per_chunk)
{
    if (n_views < 1 || width < 1 || height < 1) return lf_fail(LF_EINVAL, "bad argument");
    const int tiles = ((width + TW - 1) / TW) * ((height + TH - 1) / TH);
    if (views_per_group) *views_per_group = frames_per_group();
    if (views_per_chunk) *views_per_chunk = frames_per_chunk(n_views, tiles);
    return LF_OK;
}

lf_status lf_launch_render_batch(const lf_handle* h, const float* d_cams, int nv, int wo, int ho, float* d_out,
                                 hipStream_t s)
{
    const int tx = (wo + TW - 1) / TW, ty = (ho + TH - 1) / TH;
    const int fpg = frames_per_group(), chunk = frames_per_chunk(nv, tx * ty);
    const int64_t n_work = (int64_t)tx * ty * ((nv + chunk - 1) / chunk);
    // Split the items past the last whole round of resident workgroups
    // (3 per CU) into runs of views, so the tail of the launch is spread
    // over more CUs; chunks too short to split keep one workgroup each.
    const int split = tail_split();
    const int64_t slots = 3 * (int64_t)device_cus();
    int64_t n_full = n_work;
    if (split > 1 && chunk >= 2 * split && n_work > slots && n_work % slots) n_full = n_work - n_work % slots;
    const int sp = n_full < n_work ? split : 1;
    const int64_t grid = (n_full + 7) / 8 * 8 + ((n_work - n_full) * sp + 7) / 8 * 8;
    if (grid > 0x7FFFFFFF) return lf_fail(LF_EINVAL, "too many tiles");
    const bool small = h->L.g.bs < 16, c420 = h->L.chroma420 != 0;
    const size_t lds = small ? LDS_DYN_BYTES_SB : LDS_DYN_BYTES;
    using BatchKernel = void (*)(LfGeom, LfPtrs, LfGeom, LfPtrs, const float*, int, int, int, int, int, int, int,
                                 int64_t, int, float*);
    static const BatchKernel kernels[2][2] = {{k_render_batch<false, false>, k_render_batch<false, true>},
                                              {k_render_batch<true, false>, k_render_batch<true, true>}};
    const BatchKernel kern = kernels[small][c420];
    static bool attr_set[2][2] = {};
    if (lds > 65536 && !attr_set[small][c420]) {
        if (hipFuncSetAttribute((const void*)kern, hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds) != hipSuccess)
            return lf_fail(LF_EDEVICE, "cannot reserve %zu bytes of LDS", lds);
        attr_set[small][c420] = true;
    }
    // a 4:4:4 stream passes its own geometry as the (unused) chroma geometry
    const LfGeom& gc = c420 ? h->L.gc : h->L.g;
    const LfPtrs& pc = c420 ? h->pc : h->p;
    hipLaunchKernelGGL(kern, dim3((unsigned)grid), dim3(NT), lds, s, h->L.g, h->p, gc, pc, d_cams, nv, wo, ho, tx, ty,
                       chunk, fpg, n_full, sp, d_out);
    // marked pairs: workgroups each check a contiguous range.  With 16x16
    // blocks few tiles exceed the staging budget and 1024 workgroups keep the
    // pass short; smaller blocks mark many more tiles, which need the wider grid.
    const int64_t pairs = (int64_t)tx * ty * nv;
    const int64_t fb_grid = std::min<int64_t>(pairs, h->L.g.bs >= 16 ? 1024 : 8192);
    const int64_t per_wg = (pairs + fb_grid - 1) / fb_grid;
    if (per_wg > 0x7FFFFFFF) return lf_fail(LF_EINVAL, "too many tiles");
    hipLaunchKernelGGL(c420 ? k_render_fallback<true> : k_render_fallback<false>, dim3((unsigned)fb_grid), dim3(NT), 0,
                       s, h->L.g, h->p, gc, pc, d_cams, nv, wo, ho, tx, ty, (int)per_wg, d_out);
    return lf_check_launch("render_batch");
}

extern "C" lf_status lf_render_views(const lf_handle* h, const float* d_cams, int32_t n_views, int32_t width,
                                     int32_t height, float* d_out, void* stream)
{
    if (!h || n_views < 0 || width < 1 || height < 1) return lf_fail(LF_EINVAL, "bad argument");
    if (n_views == 0) return LF_OK;
    if (!d_cams || !d_out) return lf_fail(LF_EINVAL, "null buffer");
    // the tile kernel decodes quads of 4 pixels inside one block and reads
    // dense reference planes
    if (h->L.g.bs < 4 || h->L.sparse)
        return lf_launch_render_rays(h, d_cams, n_views, width, height, d_out, (hipStream_t)stream);
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

extern "C" lf_status lf_render_views_lod(const lf_handle* h, int32_t level, const float* d_cams, int32_t n_views,
                                         int32_t width, int32_t height, float* d_out, void* stream)
{
    if (!h || n_views < 0 || width < 1 || height < 1 || level < 0 || level > h->L.g.H)
        return lf_fail(LF_EINVAL, "bad argument");
    if (n_views == 0) return LF_OK;
    if (!d_cams || !d_out) return lf_fail(LF_EINVAL, "null buffer");
    return lf_launch_render_rays(h, d_cams, n_views, width, height, d_out, (hipStream_t)stream, level);
}
