// Stream geometry and device-side decoding primitives of the HMLFC library.
//
// The tree (RLFC: Hierarchical Compression Scheme) has levels 0 (leaf views)
// .. H (root RKVs); level l+1 clusters the 2x2 grid-aligned nodes of level l,
// so node (B, A) of level l has parent (B >> 1, A >> 1).  In every cluster the
// (even, even) node is the reference SRV; the others are predictive SRVs,
// motion-compensated against it (Phase-shifted Motion Compensation).
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

#define LF_MAX_LEVELS 8
#define LF_HDR_BYTES 1024
#define LF_HDR_CHROMA 560  // u32 chroma format: 0 full-size chroma, 1 4:2:0
#define LF_MODE_ZERO 0xFF

struct LfGeom {
    int na, nb, w, h, H, bs, nbx, nblk;
    int nch;  // channels this geometry holds: 3, or 1 (luma) and 2 (Co, Cg at half size) for 4:2:0
    int bsl;  // log2 of the block size (a power of two)
    int na_l[LF_MAX_LEVELS + 1], nb_l[LF_MAX_LEVELS + 1];
    int node_base[LF_MAX_LEVELS];  // first BFS node index of each level
    int ref_base[LF_MAX_LEVELS];   // first reference plane of each level
    int step[LF_MAX_LEVELS];       // dequantisation step
    int bias[LF_MAX_LEVELS];       // 4 * search window: motion-vector offset
    int n_nodes, n_refs;
    int root_na, root_nb;
    uint32_t mv_word[3][LF_MAX_LEVELS];
    uint32_t sig_word[3][LF_MAX_LEVELS];
    int mv_mode[3][LF_MAX_LEVELS];
    int64_t rec_base[3][LF_MAX_LEVELS];  // motion record base (relaxed shift index)
};

struct LfPtrs {
    const int16_t* root;      // [3][root_nb][root_na][h][w]
    const uint2* table;       // [3][n_nodes][nblk]: x = payload word, y = min | mode << 16
    const uint32_t* payload;  // block payload words (+ slack)
    const uint32_t* mv;       // motion-vector section words (+ slack)
    const int16_t* refs;      // dense: [3][n_refs][h][w] decoded reference SRVs;
                              // sparse: [n_tiles][bs][bs] tiles of the significant reference blocks
    const uint4* desc;        // [3][n_nodes][nblk] block descriptors (lf_make_desc), built at load (dense only)
    const int32_t* slots;     // sparse: [3][n_refs][nblk] tile of each reference block, -1 = zero block;
                              // null for dense planes
    const uint32_t* rowptr;   // CSR: first nonzero of every reference row [3][n_refs][h], then the count
    const uint16_t* cols;     // CSR: column of every nonzero, increasing within a row (values in refs)
};

// Reference residency: dense int16 planes, block-sparse tiles, or
// per-pixel compressed sparse rows.
#define LF_RES_DENSE 0
#define LF_RES_TILES 1
#define LF_RES_CSR 2

// Ordinal of predictive node (B, A) among the predictive nodes of its level,
// raster order: rows with odd B are entirely predictive, rows with even B
// only at odd A.
__host__ __device__ inline int pred_ordinal(int na_l, int B, int A)
{
    return (B >> 1) * na_l + ((B + 1) >> 1) * (na_l >> 1) + ((B & 1) ? A : (A >> 1));
}

// ---------------------------------------------------------------------------
// Bounded integer sequences (Bounded Integer Sequence Encoding).  Mode byte:
// family in bits 7..5 (0: b-bit fields; 1: groups of 5 = 8-bit base-3 high
// part + five b-bit low parts; 2: groups of 3 = 7-bit base-5 high part +
// three b-bit low parts), b in bits 4..0.  LSB-first bit order; every field
// lies inside a 64-bit window starting at its word.
// ---------------------------------------------------------------------------

__device__ __forceinline__ uint32_t lf_field(const uint32_t* __restrict__ w, uint32_t pos, int n)
{
    uint32_t q = pos >> 5;
    uint64_t x = ((uint64_t)w[q + 1] << 32) | w[q];
    return (uint32_t)(x >> (pos & 31u)) & ((1u << n) - 1u);
}

__device__ __forceinline__ uint32_t lf_bise_get(const uint32_t* __restrict__ w, int mode, uint32_t i)
{
    const int fam = mode >> 5, b = mode & 31;
    if (fam == 0) return lf_field(w, i * (uint32_t)b, b);
    if (fam == 1) {
        uint32_t g = i / 5u, k = i - 5u * g;
        uint32_t base = g * (uint32_t)(8 + 5 * b);
        uint32_t t = lf_field(w, base, 8);
        for (uint32_t s = 0; s < k; s++) t /= 3u;
        uint32_t lo = lf_field(w, base + 8u + k * (uint32_t)b, b);
        return ((t % 3u) << b) | lo;
    }
    uint32_t g = i / 3u, k = i - 3u * g;
    uint32_t base = g * (uint32_t)(7 + 3 * b);
    uint32_t q = lf_field(w, base, 7);
    for (uint32_t s = 0; s < k; s++) q /= 5u;
    uint32_t lo = lf_field(w, base + 7u + k * (uint32_t)b, b);
    return ((q % 5u) << b) | lo;
}

// Dequantised residual of pixel i of block blk of BFS node `node` (level l).
__device__ __forceinline__ int lf_residual(const LfGeom& g, const LfPtrs& p, int c, int l, int node, int blk,
                                           int i)
{
    uint2 e = p.table[((size_t)c * g.n_nodes + node) * g.nblk + blk];
    int mode = (int)((e.y >> 16) & 0xFFu);
    if (mode == LF_MODE_ZERO) return 0;
    int mn = (int)(int16_t)(e.y & 0xFFFFu);
    return (mn + (int)lf_bise_get(p.payload + e.x, mode, (uint32_t)i)) * g.step[l];
}

// Motion record j of (channel c, level l): quarter-pel vector and phase.
__device__ __forceinline__ void lf_motion(const LfGeom& g, const LfPtrs& p, int c, int l, uint32_t j, int& mx,
                                          int& my, int& sg)
{
    const uint32_t* w = p.mv + g.mv_word[c][l];
    const int mode = g.mv_mode[c][l];
    mx = (int)lf_bise_get(w, mode, 2u * j) - g.bias[l];
    my = (int)lf_bise_get(w, mode, 2u * j + 1u) - g.bias[l];
    uint32_t code = lf_field(p.mv + g.sig_word[c][l], 2u * j, 2);
    sg = code == 0u ? 1 : (code == 1u ? -1 : 0);
}

__device__ __forceinline__ int lf_clampi(int v, int lo, int hi) { return min(max(v, lo), hi); }

// Pixel (y, x) of reference plane rp (index into [3][n_refs]).  Dense
// residency reads the plane; block-sparse residency (the paper's
// reduced-memory reference storage, Decompression Analysis) reads the tile of
// the pixel's block, a zero block having no tile; CSR residency (the paper's
// sparse matrix, per pixel) binary-searches the row's nonzero columns.
template <int RES>
__device__ __forceinline__ int lf_ref_tap(const LfGeom& g, const LfPtrs& p, uint32_t rp, int y, int x)
{
    if (RES == LF_RES_DENSE) return p.refs[(size_t)rp * (size_t)(g.w * g.h) + y * g.w + x];
    if (RES == LF_RES_TILES) {
        const int t = p.slots[(size_t)rp * g.nblk + (y >> g.bsl) * g.nbx + (x >> g.bsl)];
        return t < 0 ? 0 : p.refs[((size_t)t << (2 * g.bsl)) + (((y & (g.bs - 1)) << g.bsl) | (x & (g.bs - 1)))];
    }
    const size_t row = (size_t)rp * g.h + y;
    const uint32_t end = p.rowptr[row + 1];
    uint32_t lo = p.rowptr[row], hi = end;
    while (lo < hi) {
        const uint32_t mid = (lo + hi) >> 1;
        if ((int)p.cols[mid] < x)
            lo = mid + 1;
        else
            hi = mid;
    }
    return (lo < end && (int)p.cols[lo] == x) ? p.refs[lo] : 0;
}

// Quarter-pel bilinear prediction from reference plane rp, taps clamped to
// the plane, rounded as (sum w * tap + 8) >> 4 with weights (4 - fx)(4 - fy),
// fx(4 - fy), (4 - fx)fy, fx fy.
template <int RES>
__device__ __forceinline__ int lf_qpel(const LfGeom& g, const LfPtrs& p, uint32_t rp, int y, int x, int mx, int my)
{
    int X = 4 * x + mx, Y = 4 * y + my;
    int x0 = X >> 2, y0 = Y >> 2, fx = X & 3, fy = Y & 3;
    int xa = lf_clampi(x0, 0, g.w - 1), xb = lf_clampi(x0 + 1, 0, g.w - 1);
    int ya = lf_clampi(y0, 0, g.h - 1), yb = lf_clampi(y0 + 1, 0, g.h - 1);
    int acc = (4 - fx) * (4 - fy) * lf_ref_tap<RES>(g, p, rp, ya, xa) +
              fx * (4 - fy) * lf_ref_tap<RES>(g, p, rp, ya, xb) +
              (4 - fx) * fy * lf_ref_tap<RES>(g, p, rp, yb, xa) + fx * fy * lf_ref_tap<RES>(g, p, rp, yb, xb);
    return (acc + 8) >> 4;
}

__device__ __forceinline__ uint32_t lf_ref_index(const LfGeom& g, int c, int l, int Bp, int Ap)
{
    return (uint32_t)(c * g.n_refs + g.ref_base[l] + Bp * g.na_l[l + 1] + Ap);
}

// One YCoCg channel of sample (b, a, y, x) (Decoding Procedure): the root
// RKV plus the SRVs of levels lod .. H-1 on the path from leaf view (b, a) up
// (lod = 0: the leaf view itself; lod = l: the reconstructed RKV of the
// level-l ancestor, the progressive decode).  Reference SRVs come from the
// resident reference storage; predictive SRVs are residual + phase *
// prediction.
template <int RES = LF_RES_DENSE>
__device__ inline int lf_decode_channel(const LfGeom& g, const LfPtrs& p, int c, int b, int a, int y, int x,
                                        int lod = 0)
{
    const int plane = g.w * g.h;
    int v = p.root[((size_t)(c * g.root_nb + (b >> g.H)) * g.root_na + (a >> g.H)) * plane + y * g.w + x];
    const int blk = (y >> g.bsl) * g.nbx + (x >> g.bsl);
    const int i = ((y & (g.bs - 1)) << g.bsl) | (x & (g.bs - 1));
    for (int l = lod; l < g.H; l++) {
        int B = b >> l, A = a >> l;
        const uint32_t rp = lf_ref_index(g, c, l, B >> 1, A >> 1);
        if (!((A | B) & 1)) {
            v += lf_ref_tap<RES>(g, p, rp, y, x);
            continue;
        }
        int node = g.node_base[l] + B * g.na_l[l] + A;
        int r = lf_residual(g, p, c, l, node, blk, i);
        int mx, my, sg;
        lf_motion(g, p, c, l, (uint32_t)(pred_ordinal(g.na_l[l], B, A) * g.nblk + blk), mx, my, sg);
        if (sg) r += sg * lf_qpel<RES>(g, p, rp, y, x, mx, my);
        v += r;
    }
    return v;
}

// 4:2:0 chroma (Compressing HMLFC tree: the chroma channels are
// sub-sampled): channel c of the chroma geometry (0: Co, 1: Cg, coded at
// half width and height) at full-resolution sample (y, x), by centred
// bilinear up-sampling.  Half-resolution sample (Y, X) sits at full
// resolution (2Y + 1/2, 2X + 1/2), so an even row y blends half rows
// y/2 - 1 and y/2 with weights 1 and 3, an odd row y/2 and y/2 + 1 with 3
// and 1 (clamped to the plane), columns likewise; (sum + 8) >> 4.
template <int RES = LF_RES_DENSE>
__device__ inline int lf_chroma_up(const LfGeom& gc, const LfPtrs& pc, int c, int b, int a, int y, int x, int lod = 0)
{
    const int y0 = (y & 1) ? (y >> 1) : (y >> 1) - 1, x0 = (x & 1) ? (x >> 1) : (x >> 1) - 1;
    const int wy0 = (y & 1) ? 3 : 1, wx0 = (x & 1) ? 3 : 1;
    int acc = 0;
    for (int j = 0; j < 2; j++) {
        const int yy = lf_clampi(y0 + j, 0, gc.h - 1), wy = j ? 4 - wy0 : wy0;
        for (int i = 0; i < 2; i++) {
            const int xx = lf_clampi(x0 + i, 0, gc.w - 1), wx = i ? 4 - wx0 : wx0;
            acc += wy * wx * lf_decode_channel<RES>(gc, pc, c, b, a, yy, xx, lod);
        }
    }
    return (acc + 8) >> 4;
}

// Inverse reversible YCoCg lifting, then clamp to 8 bits.
__device__ __forceinline__ void lf_ycocg_to_rgb(int Y, int Co, int Cg, int& r, int& gg, int& b)
{
    int t = Y - (Cg >> 1);
    gg = Cg + t;
    b = t - (Co >> 1);
    r = b + Co;
    r = lf_clampi(r, 0, 255);
    gg = lf_clampi(gg, 0, 255);
    b = lf_clampi(b, 0, 255);
}

#define MODE_PLANE 0xFE  // descriptor of a reference node: read its resident plane

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
    uint32_t mode = (e.y >> 16) & 0xFFu, word = e.x, mn = e.y & 0xFFFFu;
    if (mode == LF_MODE_ZERO) mode = word = mn = 0u;  // insignificant: zero-bit values, minimum 0
    const uint32_t code = sg == 1 ? 0u : (sg == -1 ? 1u : 2u);
    return make_uint4(word, mn | ((uint32_t)g.step[l] << 16) | (code << 29),
                      ((uint32_t)mx & 0xFFFu) | (((uint32_t)my & 0xFFFu) << 12) | (mode << 24), ref);
}

// Ray coordinates: (h0 px + h1 py) + h2 per row, each product and sum
// rounded separately (no fused multiply-add), then one IEEE division.  When a
// homography's third row is exactly (0, 0, 1) its third component is exactly 1
// at every pixel and x / 1 == x, so it is neither formed nor divided by.
// lf_ray_h maps the pixel centre through one homography h (row-major 3x3).
__device__ __forceinline__ void lf_ray_h(const float* __restrict__ h, float px, float py, float& x, float& y)
{
#pragma clang fp contract(off)
    float q[3];
#pragma unroll
    for (int r = 0; r < 2; r++) {
        float a = h[3 * r] * px;
        float bb = h[3 * r + 1] * py;
        float sum = a + bb;
        q[r] = sum + h[3 * r + 2];
    }
    if (h[6] == 0.0f && h[7] == 0.0f && h[8] == 1.0f) {
        q[2] = 1.0f;
    } else {
        float a = h[6] * px;
        float bb = h[7] * py;
        float sum = a + bb;
        q[2] = sum + h[8];
    }
    if (q[2] == 1.0f) {
        x = q[0];
        y = q[1];
    } else {
        x = q[0] / q[2];
        y = q[1] / q[2];
    }
}

__device__ inline void lf_ray(const float* __restrict__ cam, int i, int j, float& u, float& v, float& s, float& t)
{
    const float px = (float)i + 0.5f, py = (float)j + 0.5f;
    lf_ray_h(cam, px, py, u, v);
    lf_ray_h(cam + 9, px, py, s, t);
}

// Clamp a coordinate to [0, n-1]; lower neighbour k (<= n-2), upper
// neighbour, fraction c - k.
__device__ __forceinline__ void lf_axis(float c, int n, int& k0, int& k1, float& f)
{
    c = fminf(fmaxf(c, 0.0f), (float)(n - 1));
    int k = (int)floorf(c);
    k = min(k, n - 2);
    k = max(k, 0);
    k0 = k;
    k1 = min(k + 1, n - 1);
    f = c - (float)k;
}
