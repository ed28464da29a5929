// HMLFC encoder on the GPU: builds the compressed stream the library decodes.
//
// The pipeline is the paper's (Fig. 1 caption):
//   1. reversible YCoCg per sample (Compressing HMLFC tree);
//   2. the RLFC hierarchy: each level-(l+1) RKV is the rounded mean of a 2x2
//      grid-aligned cluster of level-l views, ragged at odd edges, up to the
//      tree height (RLFC: Hierarchical Compression Scheme);
//   3. top-down from the lossless root, level by level: SRV = view minus the
//      reconstructed parent RKV; the (even, even) member of each cluster is
//      the reference and is quantised directly; every block of the other
//      members is predicted from the coded reference with the phase-shifted
//      search of Eq. 1-2 (Phase-shifted Motion Compensation; the quarter-pel
//      refinement is the sub-pel compensation of Future Work) and its
//      residual is quantised (the replacement step);
//   4. uniform quantisation per level, and a block whose dequantised energy
//      is below the level's threshold is dropped (Compressing HMLFC tree);
//   5. every block, then the motion vectors, as bounded integer sequences in
//      breadth-first node order (Bounded Integer Sequence Encoding;
//      Compressed Stream Structure).
//
// Every stage is a kernel over planes kept in the caller's device workspace:
// one thread per sample for the colour, pyramid and SRV stages; one wave64
// per block for quantisation, thresholding and packing; the motion search is
// k_mc_search (lf_search.hip).  Block payload offsets come from a device
// prefix sum over the per-block word counts.  Packing builds each output word
// from the fields that overlap it, so no word is written twice and nothing
// needs zeroing.  The host sequences the launches, writes the 1 KiB header
// and copies the sections back.
#include <hip/hip_runtime.h>

#include <cstddef>
#include <cstdlib>
#include <cstring>

#include <algorithm>

#include "lf_internal.h"

namespace {

constexpr int kMaxLevels = LF_MAX_LEVELS;

enum : int32_t {
    ST_RANGE = 1,   // a quantised value, coded SRV or reconstruction left int16
    ST_SEARCH = 2,  // the search reported an error for a block
    ST_MV = 4,      // a motion vector outside +-4W
};

__host__ __device__ inline int64_t align256(int64_t v) { return (v + 255) & ~(int64_t)255; }

__device__ __forceinline__ bool fits16(int v) { return v >= -32768 && v <= 32767; }

// ---------------------------------------------------------------------------
// bounded-integer-sequence modes (format: family in bits 7..5, b in 4..0)
// ---------------------------------------------------------------------------

__host__ __device__ inline int64_t seq_bits(int fam, int b, int64_t n)
{
    switch (fam) {
        case 0: return n * b;                    // b-bit fields
        case 1: return ((n + 4) / 5) * (8 + 5 * b);  // 5 values: base-3 high field + 5 b-bit parts
        default: return ((n + 2) / 3) * (7 + 3 * b); // 3 values: base-5 high field + 3 b-bit parts
    }
}

// Cheapest family for n values in [0, vmax]: family f covers m_f * 2^b
// values (m = 1, 3, 5), so b is the bit length of vmax / m_f; b above 20 is
// not representable.  Equal sizes keep the lower family number.
__host__ __device__ inline int pick_mode(uint32_t vmax, int64_t n, int64_t* bits)
{
    int mode = -1;
    int64_t size = 0;
    for (int fam = 0; fam < 3; fam++) {
        const uint32_t q = vmax / (uint32_t)(2 * fam + 1);
        const int b = q ? 32 - __builtin_clz(q) : 0;
        if (b > 20) continue;
        const int64_t s = seq_bits(fam, b, n);
        if (mode < 0 || s < size) {
            mode = (fam << 5) | b;
            size = s;
        }
    }
    if (bits) *bits = size;
    return mode;
}

// Word k (bits 32k .. 32k + 31) of the sequence val(0 .. n-1) coded with
// mode (fam, b): every field overlapping the word contributes its bits.
template <class Val>
__device__ uint32_t seq_word(const Val& val, int64_t n, int fam, int b, int64_t k)
{
    const int64_t lo = 32 * k, hi = lo + 32;
    uint32_t word = 0;
    auto put = [&](int64_t pos, int nbits, uint32_t v) {
        if (nbits == 0 || pos >= hi || pos + nbits <= lo) return;
        const int64_t sh = pos - lo;
        word |= sh >= 0 ? (uint32_t)((uint64_t)v << sh) : (v >> (int)(-sh));
    };
    if (fam == 0) {
        if (b == 0) return 0;
        const int64_t last = min(n, (hi + b - 1) / b);
        for (int64_t i = lo / b; i < last; i++) put(i * b, b, val(i));
        return word;
    }
    const int per = fam == 1 ? 5 : 3, hbits = fam == 1 ? 8 : 7;
    const uint32_t radix = fam == 1 ? 3u : 5u, mask = (1u << b) - 1u;
    const int64_t gbits = hbits + per * b, groups = (n + per - 1) / per;
    for (int64_t g = lo / gbits; g < groups && g * gbits < hi; g++) {
        uint32_t high = 0, weight = 1;
        for (int t = 0; t < per; t++) {
            const int64_t i = g * per + t;
            const uint32_t v = i < n ? val(i) : 0u;
            high += (v >> b) * weight;
            weight *= radix;
            put(g * gbits + hbits + (int64_t)t * b, b, v & mask);
        }
        put(g * gbits, hbits, high);
    }
    return word;
}

// ---------------------------------------------------------------------------
// plan: level grids, entry counts and the workspace layout
// ---------------------------------------------------------------------------

// Channels coded at one plane size: all three, or for 4:2:0 chroma the luma
// (group 0) and Co, Cg at half width and height (group 1).
struct Group {
    int nch, c0;  // channels, first stream channel
    int w, h, nbx, nblk;
    int64_t plane;
    int64_t npred[kMaxLevels];     // predictive blocks per channel and level
    int64_t rec_base[kMaxLevels];  // first motion record of each level, [channel][record] inside
    int64_t ebase;                 // first table entry of the group
    int64_t o_I[kMaxLevels + 1], o_shat;  // workspace: YCoCg planes per level, coded SRVs
};

struct Plan {
    int H, bs, bsl, n, w, h, na, nb, c420, ngroups;
    Group grp[2];
    int na_l[kMaxLevels + 1], nb_l[kMaxLevels + 1];
    int64_t views[kMaxLevels + 1], node_base[kMaxLevels], n_nodes, nent, n_rec;
    int64_t payload_bound;  // payload words without slack, upper bound
    // motion-vector section (word offsets, modes), [stream channel][level]
    uint32_t mv_word[3][kMaxLevels], sig_word[3][kMaxLevels];
    int mv_mode[3][kMaxLevels];
    int64_t mv_words;  // without slack
    int64_t n_tiles;   // prefix-sum tiles
    // workspace sections (byte offsets)
    int64_t o_status, o_rgb, o_q, o_ext, o_wm, o_woff, o_table, o_tile, o_rec, o_items, o_payload, o_mv, o_full,
        total;
    const Group& of(int c) const { return grp[(c420 && c > 0) ? 1 : 0]; }
};

constexpr int SCAN_PER_THREAD = 16, SCAN_THREADS = 256, SCAN_TILE = SCAN_PER_THREAD * SCAN_THREADS;

lf_status make_plan(int32_t nb, int32_t na, int32_t h, int32_t w, const lf_encode_params* prm, Plan* P)
{
    if (!prm) return lf_fail(LF_EINVAL, "null argument");
    const int H = prm->levels, bs = prm->block, c420 = prm->chroma420 != 0;
    if (H < 1 || H > kMaxLevels || bs < 1 || bs > 64 || (bs & (bs - 1)) || w < 1 || h < 1 || w % bs || h % bs ||
        na < 1 || nb < 1 || na > 4096 || nb > 4096 || w > 16384 || h > 16384)
        return lf_fail(LF_EINVAL, "bad geometry (block a power of two up to 64 dividing the image sides)");
    if (c420 && (w % (2 * bs) || h % (2 * bs)))
        return lf_fail(LF_EINVAL, "4:2:0 chroma needs image sides that are multiples of twice the block size");
    if (prm->chroma420 < 0 || prm->chroma420 > 1) return lf_fail(LF_EINVAL, "chroma420 must be 0 or 1");
    for (int l = 0; l < H; l++)
        if (prm->step[l] < 1 || prm->step[l] > 4096 || prm->win[l] < 0 || prm->win[l] > 255)
            return lf_fail(LF_EINVAL, "bad step or window at level %d", l);
    if (!prm->no_mc) {
        if (bs < 2) return lf_fail(LF_EINVAL, "the motion search needs blocks of at least 2x2");
        for (int l = 0; l < H; l++)
            if (bs + 2 * prm->win[l] + 1 > 96)
                return lf_fail(LF_EINVAL, "search window too large at level %d (block + 2W + 1 > 96)", l);
    }
    Plan& p = *P;
    memset(&p, 0, sizeof p);
    p.H = H;
    p.bs = bs;
    while ((1 << p.bsl) < bs) p.bsl++;
    p.n = bs * bs;
    p.w = w;
    p.h = h;
    p.na = na;
    p.nb = nb;
    p.c420 = c420;
    p.ngroups = c420 ? 2 : 1;
    p.na_l[0] = na;
    p.nb_l[0] = nb;
    for (int l = 1; l <= H; l++) {
        p.na_l[l] = (p.na_l[l - 1] + 1) >> 1;
        p.nb_l[l] = (p.nb_l[l - 1] + 1) >> 1;
    }
    for (int l = 0; l <= H; l++) p.views[l] = (int64_t)p.na_l[l] * p.nb_l[l];
    for (int l = H - 1; l >= 0; l--) {
        p.node_base[l] = p.n_nodes;
        p.n_nodes += p.views[l];
    }
    int64_t items_max = 0;
    for (int gi = 0; gi < p.ngroups; gi++) {
        Group& G = p.grp[gi];
        G.nch = c420 ? (gi == 0 ? 1 : 2) : 3;
        G.c0 = gi == 0 ? 0 : 1;
        G.w = gi == 0 ? w : w / 2;
        G.h = gi == 0 ? h : h / 2;
        G.nbx = G.w / bs;
        G.nblk = G.nbx * (G.h / bs);
        G.plane = (int64_t)G.w * G.h;
        G.ebase = p.nent;
        p.nent += G.nch * p.n_nodes * G.nblk;
        for (int l = 0; l < H; l++) {
            // predictive nodes: every node of an odd row, odd columns of an even row
            const int64_t pn =
                (int64_t)(p.nb_l[l] >> 1) * p.na_l[l] + (int64_t)((p.nb_l[l] + 1) >> 1) * (p.na_l[l] >> 1);
            G.npred[l] = pn * G.nblk;
            G.rec_base[l] = p.n_rec;
            p.n_rec += G.nch * G.npred[l];
        }
        items_max = std::max(items_max, G.nch * G.npred[0]);
    }
    if (items_max > 0x7FFFFFF0ll) return lf_fail(LF_EINVAL, "too many blocks per level");
    // every quantised value fits int16 (checked), so a block never needs
    // more than 16 bits per value: the 16-bit plain family already fits
    p.payload_bound = p.nent * (((int64_t)16 * p.n + 31) / 32);
    int64_t mw = 0;
    for (int c = 0; c < 3; c++)
        for (int l = H - 1; l >= 0; l--) {
            const int64_t nv = 2 * p.of(c).npred[l];
            p.mv_mode[c][l] = pick_mode((uint32_t)(8 * prm->win[l]), nv > 0 ? nv : 2, nullptr);
            const int64_t bits = seq_bits(p.mv_mode[c][l] >> 5, p.mv_mode[c][l] & 31, nv);
            p.mv_word[c][l] = (uint32_t)mw;
            mw += (bits + 31) / 32;
            p.sig_word[c][l] = (uint32_t)mw;
            mw += (nv + 31) / 32;
        }
    p.mv_words = mw;
    if (mw + 2 > 0xFFFFFFFFll) return lf_fail(LF_EINVAL, "motion-vector section too large");
    p.n_tiles = (p.nent + SCAN_TILE - 1) / SCAN_TILE;
    int64_t o = 0;
    auto take = [&](int64_t bytes) {
        const int64_t at = o;
        o = align256(o + bytes);
        return at;
    };
    Group& G0 = p.grp[0];
    p.o_status = take(256);
    p.o_rgb = take(p.views[0] * (int64_t)w * h * 3);
    for (int l = 0; l <= H; l++) G0.o_I[l] = take(G0.nch * p.views[l] * G0.plane * 2);
    G0.o_shat = take(G0.nch * p.views[0] * G0.plane * 2);
    p.o_q = take(p.nent * p.n * 2);
    p.o_ext = take(p.nent * 8);
    p.o_wm = take(p.nent * 4);
    p.o_woff = take(p.nent * 8);
    p.o_table = take(p.nent * 8);
    p.o_tile = take((p.n_tiles + 1) * 8);
    p.o_rec = take(p.n_rec * 16);
    p.o_items = take(items_max * 12);
    p.o_payload = take(p.payload_bound * 4);
    p.o_mv = take(p.mv_words * 4);
    if (c420) {
        Group& G1 = p.grp[1];
        for (int l = 0; l <= H; l++) G1.o_I[l] = take(G1.nch * p.views[l] * G1.plane * 2);
        G1.o_shat = take(G1.nch * p.views[0] * G1.plane * 2);
        p.o_full = take(2 * p.views[0] * (int64_t)w * h * 2);  // full-size Co, Cg before sub-sampling
    }
    p.total = o;
    return LF_OK;
}

// ---------------------------------------------------------------------------
// kernels
// ---------------------------------------------------------------------------

inline unsigned grid_for(int64_t n, int per_block)
{
    int64_t g = (n + per_block - 1) / per_block;
    return (unsigned)(g < 1 ? 1 : (g > 0x7FFFFFFF ? 0x7FFFFFFF : g));
}

__global__ void k_enc_clear(int32_t* p, int n)
{
    if ((int)threadIdx.x < n) p[threadIdx.x] = 0;
}

// RGB uint8 [views][plane][3] -> YCoCg-R int16 planes [views][plane] of Y,
// Co and Cg (three destinations):
// Co = R - B, t = B + (Co >> 1), Cg = G - t, Y = t + (Cg >> 1)
__global__ void k_enc_colour(const uint8_t* __restrict__ rgb, int16_t* __restrict__ Y, int16_t* __restrict__ Co,
                             int16_t* __restrict__ Cg, int64_t npx)
{
    for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < npx; i += (int64_t)gridDim.x * blockDim.x) {
        const int r = rgb[3 * i], g = rgb[3 * i + 1], b = rgb[3 * i + 2];
        const int co = r - b;
        const int t = b + (co >> 1);
        const int cg = g - t;
        Y[i] = (int16_t)(t + (cg >> 1));
        Co[i] = (int16_t)co;
        Cg[i] = (int16_t)cg;
    }
}

// 4:2:0 chroma: each half-size sample is the rounded mean of its 2x2
// full-size samples, floor((sum + 2) / 4); planes [n_planes][h][w] ->
// [n_planes][h / 2][w / 2].
__global__ void k_enc_chroma_down(const int16_t* __restrict__ full, int16_t* __restrict__ half, int64_t n_planes,
                                  int w, int h)
{
    const int hw = w / 2, hh = h / 2;
    const int64_t total = n_planes * hw * hh;
    for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < total;
         i += (int64_t)gridDim.x * blockDim.x) {
        const int64_t pl = i / ((int64_t)hw * hh), px = i - pl * hw * hh;
        const int Y = (int)(px / hw), X = (int)(px - (int64_t)Y * hw);
        const int16_t* f = full + pl * w * (int64_t)h + (int64_t)(2 * Y) * w + 2 * X;
        const int num = f[0] + f[1] + f[w] + f[w + 1] + 2;
        int q = num / 4;
        if (q * 4 > num) q--;  // floor for negative sums
        half[i] = (int16_t)q;
    }
}

// Level l+1 RKV: mean of the cluster's present members, rounded half up
// (floor((sum + floor(m / 2)) / m) for m members).
__global__ void k_enc_rkv(const int16_t* __restrict__ lo, int16_t* __restrict__ hi, int nch, int nal, int nbl, int nau,
                          int nbu, int64_t plane)
{
    const int64_t total = nch * (int64_t)nau * nbu * plane;
    for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < total;
         i += (int64_t)gridDim.x * blockDim.x) {
        const int64_t px = i % plane, node = i / plane;
        const int A = (int)(node % nau), B = (int)((node / nau) % nbu), c = (int)(node / ((int64_t)nau * nbu));
        const int16_t* base = lo + (int64_t)c * nal * nbl * plane + px;
        int sum = 0, m = 0;
        for (int bb = 2 * B; bb < min(2 * B + 2, nbl); bb++)
            for (int aa = 2 * A; aa < min(2 * A + 2, nal); aa++) {
                sum += base[((int64_t)bb * nal + aa) * plane];
                m++;
            }
        const int num = sum + m / 2;
        int q = num / m;
        if (q * m > num) q--;  // floor for negative sums
        hi[i] = (int16_t)q;
    }
}

// dst[c][v] = a[c][v] + sign * up[c][parent(v)] over a level's planes:
// sign -1 forms the SRVs (view - parent RKV), sign +1 the reconstruction
// (parent RKV + coded SRV).
// (dst may be a: each element is read before it is written, by one thread)
__global__ void k_enc_parent(int16_t* dst, const int16_t* a, const int16_t* __restrict__ up, int sign, int nch,
                             int nal, int nbl, int nau, int nbu, int64_t plane, int32_t* __restrict__ status)
{
    const int64_t total = nch * (int64_t)nal * nbl * plane;
    bool bad = false;
    for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < total;
         i += (int64_t)gridDim.x * blockDim.x) {
        const int64_t px = i % plane, node = i / plane;
        const int A = (int)(node % nal), B = (int)((node / nal) % nbl), c = (int)(node / ((int64_t)nal * nbl));
        const int64_t par = (((int64_t)c * nbu + (B >> 1)) * nau + (A >> 1)) * plane + px;
        const int v = a[i] + sign * up[par];
        bad |= !fits16(v);
        dst[i] = (int16_t)v;
    }
    if (bad) atomicOr(status, ST_RANGE);
}

// Search items of a level: (predictive plane, its reference plane, block),
// planes indexed [channel][view]; items ordered (channel, predictive node in
// raster order, block), the stream's motion-record order.
__device__ __forceinline__ void pred_node(int64_t ord, int nal, int* B, int* A)
{
    // row pairs (2r, 2r + 1) hold nal / 2 (odd columns) + nal predictive nodes
    const int64_t half = nal >> 1, pair = half + nal;
    const int64_t r = ord / pair, e = ord - r * pair;
    if (e < half) {
        *B = (int)(2 * r);
        *A = (int)(2 * e + 1);
    } else {
        *B = (int)(2 * r + 1);
        *A = (int)(e - half);
    }
}

__global__ void k_enc_items(int32_t* __restrict__ items, int nch, int64_t npred, int nal, int nbl, int nblk)
{
    const int64_t nv = (int64_t)nal * nbl;
    for (int64_t it = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; it < nch * npred;
         it += (int64_t)gridDim.x * blockDim.x) {
        const int c = (int)(it / npred);
        const int64_t j = it - c * npred;
        int B, A;
        pred_node(j / nblk, nal, &B, &A);
        items[3 * it] = (int32_t)(c * nv + (int64_t)B * nal + A);
        items[3 * it + 1] = (int32_t)(c * nv + (int64_t)(B & ~1) * nal + (A & ~1));
        items[3 * it + 2] = (int32_t)(j % nblk);
    }
}

// quarter-pel bilinear prediction of pixel (y, x) from plane R shifted by
// (mx, my) quarter pixels: taps at clamped coordinates, weights
// (4 - fx)(4 - fy), fx (4 - fy), (4 - fx) fy, fx fy, rounded (+8) >> 4
__device__ __forceinline__ int qpel_pred(const int16_t* __restrict__ R, int w, int h, int y, int x, int mx, int my)
{
    const int X = 4 * x + mx, Y = 4 * y + my;
    const int fx = X & 3, fy = Y & 3;
    const int xl = min(max(X >> 2, 0), w - 1), xr = min(max((X >> 2) + 1, 0), w - 1);
    const int yt = min(max(Y >> 2, 0), h - 1), yb = min(max((Y >> 2) + 1, 0), h - 1);
    const int16_t* rt = R + (int64_t)yt * w;
    const int16_t* rb = R + (int64_t)yb * w;
    const int top = (4 - fx) * rt[xl] + fx * rt[xr], bot = (4 - fx) * rb[xl] + fx * rb[xr];
    return ((4 - fy) * top + fy * bot + 8) >> 4;
}

__device__ __forceinline__ int quantise(int e, int step)
{
    const int m = (abs(e) + (step >> 1)) / step;  // round half away from zero
    return e < 0 ? -m : m;
}

__device__ __forceinline__ int64_t wave_sum64(int64_t v)
{
#pragma unroll
    for (int o = 32; o >= 1; o >>= 1) v += __shfl_xor(v, o, 64);
    return v;
}

__device__ __forceinline__ int wave_min(int v)
{
#pragma unroll
    for (int o = 32; o >= 1; o >>= 1) v = min(v, __shfl_xor(v, o, 64));
    return v;
}

__device__ __forceinline__ int wave_max(int v)
{
#pragma unroll
    for (int o = 32; o >= 1; o >>= 1) v = max(v, __shfl_xor(v, o, 64));
    return v;
}

struct LevelArgs {
    const int16_t* S;   // SRV planes of the level [3][nv][h][w]
    int16_t* shat;      // coded SRV planes [3][nv][h][w]
    int16_t* q;         // quantised values [entry][n]
    int2* ext;          // per entry (min, max) of the quantised values
    int4* rec;          // motion records of the level [3][npred] (mx, my, sigma, cost)
    int32_t* status;
    int64_t plane, npred, node_base, n_nodes, ebase;
    int nch, nal, nbl, nau, nbx, nblk, bs, bsl, n, w, h, step, thr, no_mc, bias;
};

// One wave64 per block: quantise (PRED: the residual after the phase-signed
// quarter-pel prediction from the coded reference), drop the block when its
// dequantised energy sum |q * step| is below the threshold, store the
// quantised values and the coded SRV.
template <bool PRED>
__global__ void __launch_bounds__(256) k_enc_code(LevelArgs a)
{
    const int lane = threadIdx.x & 63;
    const int64_t it = (int64_t)blockIdx.x * 4 + (threadIdx.x >> 6);
    const int64_t nv = (int64_t)a.nal * a.nbl;
    const int64_t items = PRED ? a.nch * a.npred : a.nch * (int64_t)a.nau * ((a.nbl + 1) >> 1) * a.nblk;
    if (it >= items) return;
    int c, B, A, k;
    int mx = 0, my = 0, sg = 0;
    if (PRED) {
        c = (int)(it / a.npred);
        const int64_t j = it - c * a.npred;
        k = (int)(j % a.nblk);
        pred_node(j / a.nblk, a.nal, &B, &A);
        if (!a.no_mc) {
            const int4 r = a.rec[it];
            mx = r.x;
            my = r.y;
            sg = r.z;
            if (lane == 0 && r.w < 0) atomicOr(a.status, ST_SEARCH);
            if (lane == 0 && (abs(mx) > a.bias || abs(my) > a.bias)) atomicOr(a.status, ST_MV);
        }
    } else {
        const int64_t per_c = (int64_t)a.nau * ((a.nbl + 1) >> 1) * a.nblk;
        c = (int)(it / per_c);
        const int64_t j = it - c * per_c;
        k = (int)(j % a.nblk);
        const int64_t r = j / a.nblk;
        B = 2 * (int)(r / a.nau);
        A = 2 * (int)(r % a.nau);
    }
    const int64_t v = (int64_t)B * a.nal + A;
    const int16_t* P = a.S + ((int64_t)c * nv + v) * a.plane;
    const int16_t* R = a.shat + ((int64_t)c * nv + (int64_t)(B & ~1) * a.nal + (A & ~1)) * a.plane;
    int16_t* D = a.shat + ((int64_t)c * nv + v) * a.plane;
    const int by0 = (k / a.nbx) * a.bs, bx0 = (k % a.nbx) * a.bs;
    const int msk = a.bs - 1;

    auto value = [&](int i, int* pred) {
        const int y = by0 + (i >> a.bsl), x = bx0 + (i & msk);
        int e = P[(int64_t)y * a.w + x];
        *pred = 0;
        if (PRED && sg != 0) {
            *pred = sg * qpel_pred(R, a.w, a.h, y, x, mx, my);
            e -= *pred;
        }
        return quantise(e, a.step);
    };
    int64_t energy = 0;
    for (int i = lane; i < a.n; i += 64) {
        int pr;
        energy += (int64_t)abs(value(i, &pr)) * a.step;
    }
    const bool keep = wave_sum64(energy) >= a.thr;
    const int64_t entry = a.ebase + ((int64_t)c * a.n_nodes + a.node_base + v) * a.nblk + k;
    int16_t* Q = a.q + entry * a.n;
    int qmin = 0x7FFFFFFF, qmax = -0x7FFFFFFF - 1;
    bool bad = false;
    for (int i = lane; i < a.n; i += 64) {
        int pr;
        int qv = value(i, &pr);
        if (!keep) qv = 0;
        const int s = pr + qv * a.step;
        bad |= !fits16(qv) || !fits16(s);
        Q[i] = (int16_t)qv;
        D[(int64_t)(by0 + (i >> a.bsl)) * a.w + bx0 + (i & msk)] = (int16_t)s;
        qmin = min(qmin, qv);
        qmax = max(qmax, qv);
    }
    qmin = wave_min(qmin);
    qmax = wave_max(qmax);
    if (__ballot(bad) != 0 && lane == 0) atomicOr(a.status, ST_RANGE);
    if (lane == 0) {
        a.ext[entry] = make_int2(qmin, qmax);
        if (PRED && a.no_mc) a.rec[it] = make_int4(0, 0, 0, 0);
    }
}

// Per entry: mode and payload words (low 24 bits: words; high byte: mode).
// A range beyond 16 bits only follows a value that left int16, already
// flagged; such a block gets no payload, so the payload bound holds.
__global__ void k_enc_modes(const int2* __restrict__ ext, uint32_t* __restrict__ wm, int64_t nent, int n,
                            int32_t* __restrict__ status)
{
    for (int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; e < nent; e += (int64_t)gridDim.x * blockDim.x) {
        const int2 x = ext[e];
        const int64_t range = (int64_t)x.y - x.x;
        if ((x.x == 0 && x.y == 0) || range > 65535) {
            if (range > 65535) atomicOr(status, ST_RANGE);
            wm[e] = (uint32_t)LF_MODE_ZERO << 24;
            continue;
        }
        int64_t bits;
        const int mode = pick_mode((uint32_t)range, n, &bits);
        wm[e] = (uint32_t)((bits + 31) / 32) | ((uint32_t)mode << 24);
    }
}

// ---- exclusive prefix sum of the entries' word counts (int64) ----

__device__ int64_t block_scan_excl(int64_t v, int64_t* total)
{
    __shared__ int64_t wsum[SCAN_THREADS / 64];
    const int lane = threadIdx.x & 63, wv = threadIdx.x >> 6;
    int64_t inc = v;
#pragma unroll
    for (int o = 1; o < 64; o <<= 1) {
        const int64_t t = __shfl_up(inc, o, 64);
        if (lane >= o) inc += t;
    }
    if (lane == 63) wsum[wv] = inc;
    __syncthreads();
    int64_t before = 0, all = 0;
    for (int i = 0; i < SCAN_THREADS / 64; i++) {
        if (i < wv) before += wsum[i];
        all += wsum[i];
    }
    __syncthreads();
    if (total) *total = all;
    return before + inc - v;
}

__device__ __forceinline__ uint32_t words_of(uint32_t x) { return x & 0xFFFFFFu; }

__global__ void __launch_bounds__(SCAN_THREADS) k_scan_tiles(const uint32_t* __restrict__ wm, int64_t n,
                                                             int64_t* __restrict__ tile_sum)
{
    const int64_t base = (int64_t)blockIdx.x * SCAN_TILE + (int64_t)threadIdx.x * SCAN_PER_THREAD;
    int64_t s = 0;
    for (int i = 0; i < SCAN_PER_THREAD; i++)
        if (base + i < n) s += words_of(wm[base + i]);
    int64_t total;
    block_scan_excl(s, &total);
    if (threadIdx.x == 0) tile_sum[blockIdx.x] = total;
}

// one workgroup: tile sums -> exclusive tile offsets; the grand total at [n_tiles]
__global__ void __launch_bounds__(SCAN_THREADS) k_scan_top(int64_t* __restrict__ tile, int64_t n_tiles)
{
    int64_t carry = 0;
    for (int64_t b = 0; b < n_tiles; b += SCAN_THREADS) {
        const int64_t i = b + threadIdx.x;
        const int64_t v = i < n_tiles ? tile[i] : 0;
        int64_t total;
        const int64_t ex = block_scan_excl(v, &total);
        if (i < n_tiles) tile[i] = carry + ex;
        carry += total;
    }
    if (threadIdx.x == 0) tile[n_tiles] = carry;
}

__global__ void __launch_bounds__(SCAN_THREADS) k_scan_apply(const uint32_t* __restrict__ wm, int64_t n,
                                                             const int64_t* __restrict__ tile,
                                                             int64_t* __restrict__ woff)
{
    const int64_t base = (int64_t)blockIdx.x * SCAN_TILE + (int64_t)threadIdx.x * SCAN_PER_THREAD;
    int64_t s = 0;
    for (int i = 0; i < SCAN_PER_THREAD; i++)
        if (base + i < n) s += words_of(wm[base + i]);
    int64_t run = tile[blockIdx.x] + block_scan_excl(s, nullptr);
    for (int i = 0; i < SCAN_PER_THREAD; i++)
        if (base + i < n) {
            woff[base + i] = run;
            run += words_of(wm[base + i]);
        }
}

// table entry: u32 payload word, i16 minimum, u8 mode, u8 0
__global__ void k_enc_table(const uint32_t* __restrict__ wm, const int64_t* __restrict__ woff,
                            const int2* __restrict__ ext, uint2* __restrict__ table, int64_t nent)
{
    for (int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; e < nent; e += (int64_t)gridDim.x * blockDim.x) {
        const uint32_t mode = wm[e] >> 24;
        if (mode == LF_MODE_ZERO)
            table[e] = make_uint2(0u, (uint32_t)LF_MODE_ZERO << 16);
        else
            table[e] = make_uint2((uint32_t)woff[e], ((uint32_t)ext[e].x & 0xFFFFu) | (mode << 16));
    }
}

// One wave64 per entry: stage q - min in LDS, then each lane builds words.
__global__ void __launch_bounds__(64) k_enc_pack(const int16_t* __restrict__ q, const uint32_t* __restrict__ wm,
                                                 const int64_t* __restrict__ woff, const int2* __restrict__ ext,
                                                 uint32_t* __restrict__ payload, int n)
{
    extern __shared__ uint32_t vals[];
    const int64_t e = blockIdx.x;
    const uint32_t x = wm[e];
    const int mode = (int)(x >> 24);
    const uint32_t words = words_of(x);
    if (mode == LF_MODE_ZERO || words == 0) return;
    const int qmin = ext[e].x;
    const int16_t* src = q + e * n;
    for (int i = threadIdx.x; i < n; i += 64) vals[i] = (uint32_t)(src[i] - qmin);
    __syncthreads();
    uint32_t* dst = payload + woff[e];
    auto val = [&](int64_t i) { return vals[i]; };
    for (uint32_t k = threadIdx.x; k < words; k += 64) dst[k] = seq_word(val, n, mode >> 5, mode & 31, k);
}

// Motion vectors of one (channel, level): the (mx + 4W, my + 4W) sequence.
__global__ void k_enc_mv_words(const int4* __restrict__ rec, int64_t nrec, int bias, int mode,
                               uint32_t* __restrict__ dst, int64_t words)
{
    auto val = [&](int64_t i) {
        const int4 r = rec[i >> 1];
        return (uint32_t)((i & 1 ? r.y : r.x) + bias);
    };
    for (int64_t k = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; k < words;
         k += (int64_t)gridDim.x * blockDim.x)
        dst[k] = seq_word(val, 2 * nrec, mode >> 5, mode & 31, k);
}

// ... and its 2-bit phase codes (0: +1, 1: -1, 2: no prediction), 16 per word.
__global__ void k_enc_sig_words(const int4* __restrict__ rec, int64_t nrec, uint32_t* __restrict__ dst, int64_t words)
{
    for (int64_t k = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; k < words;
         k += (int64_t)gridDim.x * blockDim.x) {
        uint32_t word = 0;
        for (int t = 0; t < 16; t++) {
            const int64_t r = 16 * k + t;
            if (r >= nrec) break;
            const int s = rec[r].z;
            word |= (uint32_t)(s > 0 ? 0 : (s < 0 ? 1 : 2)) << (2 * t);
        }
        dst[k] = word;
    }
}

// ---------------------------------------------------------------------------
// header (1 KiB): the layout lf_parse reads
// ---------------------------------------------------------------------------

#pragma pack(push, 1)
struct MvDir {
    uint32_t mv_word, sig_word, count;
    uint8_t mode, pad[3];
};
struct StreamHeader {
    char magic[8];  // "HMLFCv1\0"
    uint32_t header_bytes, version;
    int32_t na, nb, w, h, levels, block, channels, mv_units;  // mv_units: motion vectors in 1/4 pixel
    uint32_t step[kMaxLevels], win[kMaxLevels];
    uint64_t root_off, root_bytes, table_off, table_bytes, payload_off, payload_bytes, mv_off, mv_bytes;
    MvDir dir[3][kMaxLevels];
    uint32_t chroma_format;  // 0: full-size chroma, 1: 4:2:0
    uint8_t reserved[LF_HDR_BYTES - 564];
};
#pragma pack(pop)
static_assert(sizeof(StreamHeader) == LF_HDR_BYTES, "header size");
static_assert(offsetof(StreamHeader, step) == 48 && offsetof(StreamHeader, win) == 80, "header layout");
static_assert(offsetof(StreamHeader, root_off) == 112 && offsetof(StreamHeader, dir) == 176, "header layout");
static_assert(offsetof(StreamHeader, chroma_format) == LF_HDR_CHROMA, "header layout");

}  // namespace

extern "C" lf_status lf_encode_workspace_bytes(int32_t nb, int32_t na, int32_t height, int32_t width,
                                               const lf_encode_params* prm, int64_t* bytes)
{
    if (!bytes) return lf_fail(LF_EINVAL, "null argument");
    Plan p;
    lf_status st = make_plan(nb, na, height, width, prm, &p);
    if (st != LF_OK) return st;
    *bytes = p.total;
    return LF_OK;
}

extern "C" lf_status lf_encode_device(const uint8_t* host_lf, int32_t nb, int32_t na, int32_t height, int32_t width,
                                      const lf_encode_params* prm, void* d_work, int64_t work_bytes, void* stream,
                                      uint8_t** out_stream, size_t* out_bytes)
{
    if (!host_lf || !out_stream || !out_bytes) return lf_fail(LF_EINVAL, "null argument");
    Plan p;
    lf_status st = make_plan(nb, na, height, width, prm, &p);
    if (st != LF_OK) return st;
    if (!d_work || work_bytes < p.total) return lf_fail(LF_ENOMEM, "workspace too small (%lld bytes needed)",
                                                         (long long)p.total);
    if (((uintptr_t)d_work) & 255) return lf_fail(LF_EINVAL, "workspace must be 256-byte aligned");
    hipStream_t s = (hipStream_t)stream;
    uint8_t* W = (uint8_t*)d_work;
    int32_t* status = (int32_t*)(W + p.o_status);
    auto I = [&](const Group& G, int l) { return (int16_t*)(W + G.o_I[l]); };
    int16_t* q = (int16_t*)(W + p.o_q);
    int2* ext = (int2*)(W + p.o_ext);
    uint32_t* wm = (uint32_t*)(W + p.o_wm);
    int64_t* woff = (int64_t*)(W + p.o_woff);
    int64_t* tile = (int64_t*)(W + p.o_tile);
    int4* rec = (int4*)(W + p.o_rec);
    int32_t* items = (int32_t*)(W + p.o_items);
    uint32_t* payload = (uint32_t*)(W + p.o_payload);
    uint32_t* mvsec = (uint32_t*)(W + p.o_mv);
    const unsigned T = 256;
    const unsigned GRID = 8192;  // grid-stride kernels: 32 workgroups per CU
    const int64_t fplane = (int64_t)p.w * p.h, nv0 = p.views[0];

    hipLaunchKernelGGL(k_enc_clear, dim3(1), dim3(64), 0, s, status, 64);
    if (hipMemcpyAsync(W + p.o_rgb, host_lf, (size_t)(nv0 * fplane * 3), hipMemcpyHostToDevice, s) != hipSuccess)
        return lf_fail(LF_EDEVICE, "upload failed");
    // colour transform; 4:2:0 chroma goes through a full-size buffer and the 2x2 mean
    {
        int16_t* y = I(p.grp[0], 0);
        int16_t* co = p.c420 ? (int16_t*)(W + p.o_full) : y + nv0 * fplane;
        int16_t* cg = co + nv0 * fplane;
        hipLaunchKernelGGL(k_enc_colour, dim3(GRID), dim3(T), 0, s, (const uint8_t*)(W + p.o_rgb), y, co, cg,
                           nv0 * fplane);
        if (p.c420)
            hipLaunchKernelGGL(k_enc_chroma_down, dim3(GRID), dim3(T), 0, s, (const int16_t*)co, I(p.grp[1], 0),
                               2 * nv0, p.w, p.h);
    }
    for (int gi = 0; gi < p.ngroups; gi++) {
        const Group& Gp = p.grp[gi];
        for (int l = 0; l < p.H; l++)
            hipLaunchKernelGGL(k_enc_rkv, dim3(GRID), dim3(T), 0, s, (const int16_t*)I(Gp, l), I(Gp, l + 1), Gp.nch,
                               p.na_l[l], p.nb_l[l], p.na_l[l + 1], p.nb_l[l + 1], Gp.plane);
    }
    if ((st = lf_check_launch("encode: hierarchy")) != LF_OK) return st;

    // closed loop, per channel group: I(l + 1) holds the reconstruction of
    // level l + 1 (the root is lossless); I(l) becomes the SRVs, then the
    // reconstruction
    for (int gi = 0; gi < p.ngroups; gi++) {
        const Group& Gp = p.grp[gi];
        int16_t* shat = (int16_t*)(W + Gp.o_shat);
        for (int l = p.H - 1; l >= 0; l--) {
            const int nal = p.na_l[l], nbl = p.nb_l[l], nau = p.na_l[l + 1], nbu = p.nb_l[l + 1];
            hipLaunchKernelGGL(k_enc_parent, dim3(GRID), dim3(T), 0, s, I(Gp, l), (const int16_t*)I(Gp, l),
                               (const int16_t*)I(Gp, l + 1), -1, Gp.nch, nal, nbl, nau, nbu, Gp.plane, status);
            LevelArgs a;
            a.S = I(Gp, l);
            a.shat = shat;
            a.q = q;
            a.ext = ext;
            a.rec = rec + Gp.rec_base[l];
            a.status = status;
            a.plane = Gp.plane;
            a.npred = Gp.npred[l];
            a.node_base = p.node_base[l];
            a.n_nodes = p.n_nodes;
            a.ebase = Gp.ebase;
            a.nch = Gp.nch;
            a.nal = nal;
            a.nbl = nbl;
            a.nau = nau;
            a.nbx = Gp.nbx;
            a.nblk = Gp.nblk;
            a.bs = p.bs;
            a.bsl = p.bsl;
            a.n = p.n;
            a.w = Gp.w;
            a.h = Gp.h;
            a.step = prm->step[l];
            a.thr = prm->t_ref[l];
            a.no_mc = prm->no_mc != 0;
            a.bias = 4 * prm->win[l];
            const int64_t nref_items = Gp.nch * (int64_t)nau * ((nbl + 1) >> 1) * Gp.nblk;
            hipLaunchKernelGGL(k_enc_code<false>, dim3(grid_for(nref_items, 4)), dim3(256), 0, s, a);
            const int64_t npi = Gp.nch * Gp.npred[l];
            if (npi > 0) {
                if (!prm->no_mc) {
                    hipLaunchKernelGGL(k_enc_items, dim3(grid_for(npi, T)), dim3(T), 0, s, items, Gp.nch, Gp.npred[l],
                                       nal, nbl, Gp.nblk);
                    const int64_t nv = Gp.nch * (int64_t)nal * nbl;
                    st = lf_search_launch(I(Gp, l), shat, nv, nv, Gp.w, Gp.h, p.bs, prm->win[l], prm->subpel,
                                          prm->zero_phase, items, npi, (int32_t*)a.rec, stream);
                    if (st != LF_OK) return st;
                }
                a.thr = prm->t_pred[l];
                hipLaunchKernelGGL(k_enc_code<true>, dim3(grid_for(npi, 4)), dim3(256), 0, s, a);
            }
            hipLaunchKernelGGL(k_enc_parent, dim3(GRID), dim3(T), 0, s, I(Gp, l), (const int16_t*)shat,
                               (const int16_t*)I(Gp, l + 1), 1, Gp.nch, nal, nbl, nau, nbu, Gp.plane, status);
            if ((st = lf_check_launch("encode: level")) != LF_OK) return st;
        }
    }

    // block payloads: word counts, offsets, table, packing
    hipLaunchKernelGGL(k_enc_modes, dim3(grid_for(p.nent, T)), dim3(T), 0, s, (const int2*)ext, wm, p.nent, p.n,
                       status);
    hipLaunchKernelGGL(k_scan_tiles, dim3((unsigned)p.n_tiles), dim3(SCAN_THREADS), 0, s, (const uint32_t*)wm, p.nent,
                       tile);
    hipLaunchKernelGGL(k_scan_top, dim3(1), dim3(SCAN_THREADS), 0, s, tile, p.n_tiles);
    hipLaunchKernelGGL(k_scan_apply, dim3((unsigned)p.n_tiles), dim3(SCAN_THREADS), 0, s, (const uint32_t*)wm, p.nent,
                       (const int64_t*)tile, woff);
    hipLaunchKernelGGL(k_enc_table, dim3(grid_for(p.nent, T)), dim3(T), 0, s, (const uint32_t*)wm,
                       (const int64_t*)woff, (const int2*)ext, (uint2*)(W + p.o_table), p.nent);
    hipLaunchKernelGGL(k_enc_pack, dim3((unsigned)p.nent), dim3(64), (size_t)p.n * 4, s, (const int16_t*)q,
                       (const uint32_t*)wm, (const int64_t*)woff, (const int2*)ext, payload, p.n);
    // motion vectors, [stream channel][level H-1 .. 0]
    for (int c = 0; c < 3; c++)
        for (int l = p.H - 1; l >= 0; l--) {
            const Group& Gp = p.of(c);
            const int64_t nrec = Gp.npred[l];
            if (nrec == 0) continue;
            const int4* r = rec + Gp.rec_base[l] + (c - Gp.c0) * nrec;
            const int mode = p.mv_mode[c][l];
            const int64_t mvw = (seq_bits(mode >> 5, mode & 31, 2 * nrec) + 31) / 32;
            if (mvw > 0)
                hipLaunchKernelGGL(k_enc_mv_words, dim3(grid_for(mvw, T)), dim3(T), 0, s, r, nrec, 4 * prm->win[l],
                                   mode, mvsec + p.mv_word[c][l], mvw);
            const int64_t sgw = (2 * nrec + 31) / 32;
            hipLaunchKernelGGL(k_enc_sig_words, dim3(grid_for(sgw, T)), dim3(T), 0, s, r, nrec,
                               mvsec + p.sig_word[c][l], sgw);
        }
    if ((st = lf_check_launch("encode: packing")) != LF_OK) return st;
    int32_t flags = 0;
    int64_t pwords = 0;
    if (hipMemcpyAsync(&flags, status, 4, hipMemcpyDeviceToHost, s) != hipSuccess ||
        hipMemcpyAsync(&pwords, tile + p.n_tiles, 8, hipMemcpyDeviceToHost, s) != hipSuccess ||
        hipStreamSynchronize(s) != hipSuccess)
        return lf_fail(LF_EDEVICE, "encode failed");
    if (flags & ST_SEARCH) return lf_fail(LF_EINVAL, "motion search rejected a block");
    if (flags) return lf_fail(LF_EINVAL, "values exceed the stream's integer ranges");
    if (pwords > 0xFFFFFFFFll - 2) return lf_fail(LF_EINVAL, "payload exceeds 16 GiB");

    // stream: header, root (the level-H RKVs), table, payload + 2 slack
    // words, motion vectors + 2 slack words
    StreamHeader hd;
    memset(&hd, 0, sizeof hd);
    memcpy(hd.magic, "HMLFCv1", 8);
    hd.header_bytes = LF_HDR_BYTES;
    hd.version = 1;
    hd.na = p.na;
    hd.nb = p.nb;
    hd.w = p.w;
    hd.h = p.h;
    hd.levels = p.H;
    hd.block = p.bs;
    hd.channels = 3;
    hd.mv_units = 4;
    for (int l = 0; l < p.H; l++) {
        hd.step[l] = (uint32_t)prm->step[l];
        hd.win[l] = (uint32_t)prm->win[l];
    }
    hd.chroma_format = (uint32_t)p.c420;
    hd.root_off = LF_HDR_BYTES;
    uint64_t group_root[2] = {0, 0};
    for (int gi = 0; gi < p.ngroups; gi++) group_root[gi] = (uint64_t)(p.grp[gi].nch * p.views[p.H] * p.grp[gi].plane * 2);
    hd.root_bytes = group_root[0] + group_root[1];
    hd.table_off = hd.root_off + hd.root_bytes;
    hd.table_bytes = (uint64_t)p.nent * 8;
    hd.payload_off = hd.table_off + hd.table_bytes;
    hd.payload_bytes = (uint64_t)(pwords + 2) * 4;
    hd.mv_off = hd.payload_off + hd.payload_bytes;
    hd.mv_bytes = (uint64_t)(p.mv_words + 2) * 4;
    for (int c = 0; c < 3; c++)
        for (int l = 0; l < p.H; l++) {
            hd.dir[c][l].mv_word = p.mv_word[c][l];
            hd.dir[c][l].sig_word = p.sig_word[c][l];
            hd.dir[c][l].count = (uint32_t)p.of(c).npred[l];
            hd.dir[c][l].mode = (uint8_t)p.mv_mode[c][l];
        }
    const size_t total = (size_t)(hd.mv_off + hd.mv_bytes);
    uint8_t* out = (uint8_t*)calloc(total, 1);
    if (!out) return lf_fail(LF_ENOMEM, "out of host memory");
    memcpy(out, &hd, sizeof hd);
    const bool ok = hipMemcpyAsync(out + hd.root_off, I(p.grp[0], p.H), group_root[0], hipMemcpyDeviceToHost, s) ==
                        hipSuccess &&
                    (!p.c420 || hipMemcpyAsync(out + hd.root_off + group_root[0], I(p.grp[1], p.H), group_root[1],
                                               hipMemcpyDeviceToHost, s) == hipSuccess) &&
                    hipMemcpyAsync(out + hd.table_off, W + p.o_table, hd.table_bytes, hipMemcpyDeviceToHost, s) ==
                        hipSuccess &&
                    (pwords == 0 || hipMemcpyAsync(out + hd.payload_off, payload, (size_t)pwords * 4,
                                                   hipMemcpyDeviceToHost, s) == hipSuccess) &&
                    (p.mv_words == 0 || hipMemcpyAsync(out + hd.mv_off, mvsec, (size_t)p.mv_words * 4,
                                                       hipMemcpyDeviceToHost, s) == hipSuccess) &&
                    hipStreamSynchronize(s) == hipSuccess;
    if (!ok) {
        free(out);
        return lf_fail(LF_EDEVICE, "copy of the stream failed");
    }
    *out_stream = out;
    *out_bytes = total;
    return LF_OK;
}

extern "C" void lf_encode_free(uint8_t* p) { free(p); }
