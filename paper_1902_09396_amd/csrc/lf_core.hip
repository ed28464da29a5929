// HMLFC light-field library: stream loading, random-access decoding and the
// per-ray reference renderer, behind the C ABI of include/hmlfc.h.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cstdio>
#include <cstring>
#include <new>
#include <string>
#include <vector>

#include "../../include/hmlfc.h"
#include "lf_geom.h"
#include "lf_internal.h"

// ---------------------------------------------------------------------------
// errors
// ---------------------------------------------------------------------------

static thread_local std::string g_err;

lf_status lf_fail(lf_status s, const char* fmt, ...)
{
    char buf[512];
    va_list ap;
    va_start(ap, fmt);
    vsnprintf(buf, sizeof buf, fmt, ap);
    va_end(ap);
    g_err = buf;
    return s;
}

extern "C" const char* lf_last_error(void) { return g_err.c_str(); }

lf_status lf_check_launch(const char* what)
{
    hipError_t e = hipGetLastError();
    if (e != hipSuccess) return lf_fail(LF_EDEVICE, "%s: %s", what, hipGetErrorString(e));
    return LF_OK;
}

// ---------------------------------------------------------------------------
// host-side stream parsing (every offset and size is checked before upload)
// ---------------------------------------------------------------------------

static uint32_t rd32(const uint8_t* p) { uint32_t v; memcpy(&v, p, 4); return v; }
static uint64_t rd64(const uint8_t* p) { uint64_t v; memcpy(&v, p, 8); return v; }

static int64_t bise_bits_host(int mode, int64_t n)
{
    int fam = mode >> 5, b = mode & 31;
    if (fam == 0) return n * b;
    if (fam == 1) return (n + 4) / 5 * (8 + 5 * b);
    return (n + 2) / 3 * (7 + 3 * b);
}

static int64_t align256(int64_t v) { return (v + 255) & ~(int64_t)255; }

// Largest dequantised residual magnitude a block's mode may hold.  With at
// most 8 levels, a root value (int16) and reference taps of at most
// LF_REF_LIMIT, every int32 sum of the decoders stays far from overflow.
// A stream of 8-bit content has residuals of a few thousand at most.
#define LF_RES_LIMIT (1 << 24)

lf_status lf_parse(const uint8_t* s, size_t n, LfLayout* L)
{
    memset(L, 0, sizeof *L);
    if (!s) return lf_fail(LF_EINVAL, "null stream");
    if (n < LF_HDR_BYTES || memcmp(s, "HMLFCv1\0", 8) != 0) return lf_fail(LF_EFORMAT, "bad magic");
    if (rd32(s + 8) != LF_HDR_BYTES || rd32(s + 12) != 1) return lf_fail(LF_EFORMAT, "bad header size/version");
    int32_t d[8];
    memcpy(d, s + 16, 32);
    LfGeom& g = L->g;
    g.na = d[0];
    g.nb = d[1];
    g.w = d[2];
    g.h = d[3];
    g.H = d[4];
    g.bs = d[5];
    if (g.na < 1 || g.nb < 1 || g.w < 1 || g.h < 1 || g.H < 1 || g.H > LF_MAX_LEVELS || g.bs < 1 || g.bs > 64 ||
        g.w % g.bs || g.h % g.bs || d[6] != 3 || d[7] != 4 || g.na > 4096 || g.nb > 4096 || g.w > 16384 ||
        g.h > 16384)
        return lf_fail(LF_EFORMAT, "bad geometry");
    if (g.bs & (g.bs - 1)) return lf_fail(LF_EFORMAT, "block size %d is not a power of two", g.bs);
    const uint32_t cf = rd32(s + LF_HDR_CHROMA);
    if (cf > 1) return lf_fail(LF_EFORMAT, "unknown chroma format %u", cf);
    if (cf == 1 && (g.w % (2 * g.bs) || g.h % (2 * g.bs)))
        return lf_fail(LF_EFORMAT, "4:2:0 chroma planes are not whole blocks");
    L->chroma420 = (int32_t)cf;
    g.nch = cf ? 1 : 3;
    g.bsl = 0;
    while ((1 << g.bsl) < g.bs) g.bsl++;
    g.nbx = g.w / g.bs;
    g.nblk = g.nbx * (g.h / g.bs);
    g.na_l[0] = g.na;
    g.nb_l[0] = g.nb;
    for (int l = 0; l < g.H; l++) {
        g.na_l[l + 1] = (g.na_l[l] + 1) / 2;
        g.nb_l[l + 1] = (g.nb_l[l] + 1) / 2;
    }
    g.root_na = g.na_l[g.H];
    g.root_nb = g.nb_l[g.H];
    int64_t nodes = 0, refs = 0;
    for (int l = g.H - 1; l >= 0; l--) {
        g.node_base[l] = (int)nodes;
        nodes += (int64_t)g.na_l[l] * g.nb_l[l];
    }
    for (int l = 0; l < g.H; l++) {
        g.ref_base[l] = (int)refs;
        refs += (int64_t)g.na_l[l + 1] * g.nb_l[l + 1];
    }
    g.n_nodes = (int)nodes;
    g.n_refs = (int)refs;
    // device code addresses reference planes with 32-bit element offsets
    if (3 * refs * (int64_t)g.w * g.h >= ((int64_t)1 << 32)) return lf_fail(LF_EFORMAT, "light field too large");
    for (int l = 0; l < g.H; l++) {
        int32_t st, wn;
        memcpy(&st, s + 48 + 4 * l, 4);
        memcpy(&wn, s + 80 + 4 * l, 4);
        if (st < 1 || st > 4096 || wn < 0 || wn > 255) return lf_fail(LF_EFORMAT, "bad step/window at level %d", l);
        g.step[l] = st;
        g.bias[l] = 4 * wn;
    }
    // chroma geometry: the same tree at half width and height
    LfGeom& gc = L->gc;
    if (cf) {
        gc = g;
        gc.nch = 2;
        gc.w = g.w / 2;
        gc.h = g.h / 2;
        gc.nbx = gc.w / g.bs;
        gc.nblk = gc.nbx * (gc.h / g.bs);
    }
    // stream channel c: its geometry, its index there, first table entry and root sample
    auto geo = [&](int c) -> LfGeom& { return (cf && c > 0) ? gc : g; };
    auto local = [&](int c) { return (cf && c > 0) ? c - 1 : c; };
    int64_t tfirst[3], rfirst[3], tb = 0, rb = 0;
    for (int c = 0; c < 3; c++) {
        tfirst[c] = tb;
        rfirst[c] = rb;
        tb += nodes * geo(c).nblk;
        rb += (int64_t)g.root_na * g.root_nb * geo(c).w * geo(c).h;
    }
    L->root_off = rd64(s + 112);
    L->root_bytes = rd64(s + 120);
    L->table_off = rd64(s + 128);
    L->table_bytes = rd64(s + 136);
    L->payload_off = rd64(s + 144);
    L->payload_bytes = rd64(s + 152);
    L->mv_off = rd64(s + 160);
    L->mv_bytes = rd64(s + 168);
    const uint64_t N = n;
    if (L->root_bytes != (uint64_t)(rb * 2) || L->table_bytes != (uint64_t)(tb * 8))
        return lf_fail(LF_EFORMAT, "section sizes do not match the geometry");
    struct {
        uint64_t o, b;
    } sec[4] = {{L->root_off, L->root_bytes}, {L->table_off, L->table_bytes}, {L->payload_off, L->payload_bytes},
                {L->mv_off, L->mv_bytes}};
    for (auto& x : sec)
        if (x.o < LF_HDR_BYTES || x.o > N || x.b > N - x.o) return lf_fail(LF_EFORMAT, "section outside the stream");
    if ((L->root_off & 1) || (L->table_off & 3) || (L->payload_off & 3) || (L->mv_off & 3) || (L->payload_bytes & 3) ||
        (L->mv_bytes & 3) || L->payload_bytes < 8 || L->mv_bytes < 8)
        return lf_fail(LF_EFORMAT, "misaligned section");
    const int64_t pwords = (int64_t)(L->payload_bytes / 4), mwords = (int64_t)(L->mv_bytes / 4);
    // block payloads: every 64-bit read window must stay inside the payload
    // section, and every value the mode can hold, (min + v) * step, must
    // stay within LF_RES_LIMIT so that the decoders' int32 sums cannot wrap
    const uint8_t* tab = s + L->table_off;
    for (int c = 0; c < 3; c++)
        for (int l = g.H - 1; l >= 0; l--) {
            const int nblk = geo(c).nblk;
            const int64_t first = tfirst[c] + (int64_t)g.node_base[l] * nblk;
            const int64_t count = (int64_t)g.na_l[l] * g.nb_l[l] * nblk;
            for (int64_t e = first; e < first + count; e++) {
                const uint8_t* t = tab + 8 * e;
                const int mode = t[6];
                if (mode == LF_MODE_ZERO) continue;
                if ((mode >> 5) > 2 || (mode & 31) > 20)
                    return lf_fail(LF_EFORMAT, "bad block mode at entry %lld", (long long)e);
                const int64_t words = (bise_bits_host(mode, (int64_t)g.bs * g.bs) + 31) / 32;
                if ((int64_t)rd32(t) + words + 1 > pwords) return lf_fail(LF_EFORMAT, "block payload out of range");
                int16_t mn;
                memcpy(&mn, t + 4, 2);
                const int64_t cap = (int64_t)(2 * (mode >> 5) + 1) << (mode & 31);  // values 0 .. cap - 1
                const int64_t lo = (int64_t)mn * g.step[l], hi = ((int64_t)mn + cap - 1) * g.step[l];
                if (std::max(std::llabs(lo), std::llabs(hi)) > LF_RES_LIMIT)
                    return lf_fail(LF_EFORMAT, "block residual range beyond %d at entry %lld", LF_RES_LIMIT,
                                   (long long)e);
            }
        }
    int64_t rec = 0;
    for (int c = 0; c < 3; c++)
        for (int l = g.H - 1; l >= 0; l--) {
            LfGeom& gg = geo(c);
            const int lc = local(c);
            const uint8_t* dd = s + 176 + (c * LF_MAX_LEVELS + l) * 16;
            gg.mv_word[lc][l] = rd32(dd);
            gg.sig_word[lc][l] = rd32(dd + 4);
            uint32_t count = rd32(dd + 8);
            gg.mv_mode[lc][l] = dd[12];
            int64_t npn = (int64_t)(g.nb_l[l] / 2) * g.na_l[l] + (int64_t)((g.nb_l[l] + 1) / 2) * (g.na_l[l] / 2);
            int64_t expect = npn * gg.nblk;
            if ((int64_t)count != expect) return lf_fail(LF_EFORMAT, "motion record count mismatch");
            if (expect > 0) {
                int m = gg.mv_mode[lc][l];
                if ((m >> 5) > 2 || (m & 31) > 20) return lf_fail(LF_EFORMAT, "bad motion-vector mode");
                if ((int64_t)gg.mv_word[lc][l] + (bise_bits_host(m, 2 * expect) + 31) / 32 + 1 > mwords ||
                    (int64_t)gg.sig_word[lc][l] + (2 * expect + 31) / 32 + 1 > mwords)
                    return lf_fail(LF_EFORMAT, "motion-vector section out of range");
            }
            gg.rec_base[lc][l] = rec;
            rec += expect;
        }
    L->n_rec = rec;
    // arena: [root][table][payload][mv][refs][desc][status], 256-byte
    // aligned; desc holds one 16-byte block descriptor per (channel, node,
    // block), expanded from the table and motion vectors at load; the status
    // tail keeps the multi-word loads at the end of the last section inside
    // the arena.  4:2:0: [refs] holds the luma reference planes, then the
    // chroma ones at a_refs_c, and there are no descriptors.
    const int64_t plane = (int64_t)g.w * g.h;
    L->a_root = 0;
    L->a_table = align256(L->a_root + (int64_t)L->root_bytes);
    L->a_payload = align256(L->a_table + (int64_t)L->table_bytes);
    L->a_mv = align256(L->a_payload + (int64_t)L->payload_bytes);
    L->a_refs = align256(L->a_mv + (int64_t)L->mv_bytes);
    if (cf) {
        L->a_refs_c = align256(L->a_refs + refs * plane * 2);
        L->a_desc = align256(L->a_refs_c + 2 * refs * (int64_t)gc.w * gc.h * 2);
        L->a_status = L->a_desc;
    } else {
        L->a_desc = align256(L->a_refs + 3 * refs * plane * 2);
        L->a_status = align256(L->a_desc + 3 * nodes * (int64_t)g.nblk * 16);
    }
    L->arena = L->a_status + 256;
    L->stream_bytes = (int64_t)n;
    (void)rfirst;
    return LF_OK;
}

lf_status lf_require_full_chroma(const lf_handle* h, const char* what)
{
    if (h && h->L.chroma420) return lf_fail(LF_EINVAL, "%s needs full-size chroma planes (a 4:4:4 stream)", what);
    return LF_OK;
}

// Sparse reference residency: significant blocks of the reference SRVs take
// consecutive tiles in (channel, reference node, block) order; a block coded
// as insignificant decodes to zero and takes none.  Writes the tile of every
// reference block to slots (when given) and returns the tile count.
static int64_t lf_ref_slots(const uint8_t* s, const LfLayout& L, int32_t* slots)
{
    const LfGeom& g = L.g;
    const uint8_t* tab = s + L.table_off;
    int64_t n = 0;
    for (int c = 0; c < 3; c++)
        for (int l = 0; l < g.H; l++)
            for (int Bp = 0; Bp < g.nb_l[l + 1]; Bp++)
                for (int Ap = 0; Ap < g.na_l[l + 1]; Ap++) {
                    const int64_t node = g.node_base[l] + 2 * Bp * g.na_l[l] + 2 * Ap;
                    const int64_t rp = (int64_t)c * g.n_refs + g.ref_base[l] + (int64_t)Bp * g.na_l[l + 1] + Ap;
                    const uint8_t* e = tab + 8 * (((int64_t)c * g.n_nodes + node) * g.nblk);
                    for (int blk = 0; blk < g.nblk; blk++) {
                        const bool sig = e[8 * blk + 6] != LF_MODE_ZERO;
                        if (slots) slots[rp * g.nblk + blk] = sig ? (int32_t)n : -1;
                        n += sig;
                    }
                }
    return n;
}

// Re-lay a parsed layout for sparse residency: [root][table][payload][mv]
// [tiles][slots][status].
static lf_status lf_layout_sparse(const uint8_t* s, LfLayout* L)
{
    const LfGeom& g = L->g;
    L->n_tiles = lf_ref_slots(s, *L, nullptr);
    if (L->n_tiles > 0x7FFFFFFF) return lf_fail(LF_EFORMAT, "too many reference blocks");
    L->sparse = LF_RES_TILES;
    L->a_slots = align256(L->a_refs + L->n_tiles * (int64_t)g.bs * g.bs * 2);
    L->a_desc = L->a_status = align256(L->a_slots + 3 * (int64_t)g.n_refs * g.nblk * 4);
    L->arena = L->a_status + 256;
    return LF_OK;
}

// Re-lay a parsed layout for CSR residency: [root][table][payload][mv]
// [values][columns][row starts][status].  The
// nonzero count is known only after decoding, so values and columns are
// sized for every pixel of the significant reference blocks.
static lf_status lf_layout_csr(const uint8_t* s, LfLayout* L)
{
    const LfGeom& g = L->g;
    if (g.w > 65535) return lf_fail(LF_EINVAL, "CSR residency stores 16-bit columns");
    L->nnz_bound = lf_ref_slots(s, *L, nullptr) * (int64_t)g.bs * g.bs;
    if (L->nnz_bound > 0xFFFFFFF0ll) return lf_fail(LF_EFORMAT, "too many reference pixels for 32-bit row starts");
    const int64_t rows = 3 * (int64_t)g.n_refs * g.h;
    L->sparse = LF_RES_CSR;
    L->a_cols = align256(L->a_refs + L->nnz_bound * 2);
    L->a_rowptr = align256(L->a_cols + L->nnz_bound * 2);
    L->a_desc = L->a_status = align256(L->a_rowptr + (rows + 1) * 4);
    L->arena = L->a_status + 256;
    return LF_OK;
}

static lf_status lf_parse_ex(const uint8_t* s, size_t n, int32_t flags, LfLayout* L)
{
    if ((flags & ~(LF_LOAD_SPARSE_REFS | LF_LOAD_CSR_REFS)) ||
        (flags & (LF_LOAD_SPARSE_REFS | LF_LOAD_CSR_REFS)) == (LF_LOAD_SPARSE_REFS | LF_LOAD_CSR_REFS))
        return lf_fail(LF_EINVAL, "unknown or conflicting load flags 0x%x", flags);
    lf_status st = lf_parse(s, n, L);
    if (st != LF_OK || !flags) return st;
    if (L->chroma420) return lf_fail(LF_EINVAL, "sparse reference residency needs full-size chroma planes");
    return (flags & LF_LOAD_CSR_REFS) ? lf_layout_csr(s, L) : lf_layout_sparse(s, L);
}

extern "C" lf_status lf_query_arena_ex(const void* host_stream, size_t nbytes, int32_t flags, int64_t* arena_bytes)
{
    if (!arena_bytes) return lf_fail(LF_EINVAL, "null output");
    LfLayout L;
    lf_status st = lf_parse_ex((const uint8_t*)host_stream, nbytes, flags, &L);
    if (st != LF_OK) return st;
    *arena_bytes = L.arena;
    return LF_OK;
}

extern "C" lf_status lf_query_arena(const void* host_stream, size_t nbytes, int64_t* arena_bytes)
{
    return lf_query_arena_ex(host_stream, nbytes, 0, arena_bytes);
}

// ---------------------------------------------------------------------------
// reference planes (Decompression Memory Overhead)
// ---------------------------------------------------------------------------

// Reference SRVs must satisfy |v| <= LF_REF_LIMIT: the tile renderer forms
// 16-weighted prediction sums of them in 16-bit lanes.  SRVs of 8-bit
// content stay near +-520; a larger value flags the stream as malformed.
#define LF_REF_LIMIT 2047
#define LF_SAMPLE_LIMIT 8191
// load status bits
#define LF_ST_REF 1     // a reference SRV beyond LF_REF_LIMIT
#define LF_ST_MV 2      // a motion vector beyond 12 signed bits
#define LF_ST_SAMPLE 4  // a decoded sample channel beyond LF_SAMPLE_LIMIT

__global__ void k_load_refs(LfGeom g, LfPtrs p, int16_t* __restrict__ refs, int* __restrict__ status)
{
    bool bad = false;
    const int64_t plane = (int64_t)g.w * g.h;
    const int64_t total = g.nch * (int64_t)g.n_refs * plane;
    for (int64_t t = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; t < total; t += (int64_t)gridDim.x * blockDim.x) {
        int64_t px = t % plane;
        int64_t r = (t / plane) % g.n_refs;
        int c = (int)(t / (plane * g.n_refs));
        int l = 0;
        while (l + 1 < g.H && r >= g.ref_base[l + 1]) l++;
        int local = (int)(r - g.ref_base[l]);
        int Bp = local / g.na_l[l + 1], Ap = local % g.na_l[l + 1];
        int node = g.node_base[l] + (2 * Bp) * g.na_l[l] + 2 * Ap;
        int y = (int)(px / g.w), x = (int)(px % g.w);
        int blk = (y / g.bs) * g.nbx + x / g.bs;
        int i = (y % g.bs) * g.bs + x % g.bs;
        const int v = lf_residual(g, p, c, l, node, blk, i);
        bad |= v < -LF_REF_LIMIT || v > LF_REF_LIMIT;
        refs[t] = (int16_t)v;
    }
    if (bad) atomicOr(status, LF_ST_REF);
}

// Sparse residency: the tile of every significant reference block.
__global__ void k_load_tiles(LfGeom g, LfPtrs p, int16_t* __restrict__ tiles, int* __restrict__ status)
{
    bool bad = false;
    const int n = g.bs * g.bs;
    const int64_t total = 3 * (int64_t)g.n_refs * g.nblk * n;
    for (int64_t t = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; t < total; t += (int64_t)gridDim.x * blockDim.x) {
        const int64_t rb = t / n;  // (reference plane, block)
        const int tile = p.slots[rb];
        if (tile < 0) continue;
        const int i = (int)(t - rb * n);
        const int blk = (int)(rb % g.nblk);
        const int64_t rp = rb / g.nblk;
        const int c = (int)(rp / g.n_refs), r = (int)(rp % g.n_refs);
        int l = 0;
        while (l + 1 < g.H && r >= g.ref_base[l + 1]) l++;
        const int local = r - g.ref_base[l];
        const int Bp = local / g.na_l[l + 1], Ap = local % g.na_l[l + 1];
        const int node = g.node_base[l] + (2 * Bp) * g.na_l[l] + 2 * Ap;
        const int v = lf_residual(g, p, c, l, node, blk, i);
        bad |= v < -LF_REF_LIMIT || v > LF_REF_LIMIT;
        tiles[(int64_t)tile * n + i] = (int16_t)v;
    }
    if (bad) atomicOr(status, LF_ST_REF);
}

// Dequantised value of pixel (y, x) of reference plane rp (index into
// [3][n_refs]) straight from the stream.
__device__ __forceinline__ int lf_ref_value(const LfGeom& g, const LfPtrs& p, int64_t rp, int y, int x)
{
    const int c = (int)(rp / g.n_refs), r = (int)(rp % g.n_refs);
    int l = 0;
    while (l + 1 < g.H && r >= g.ref_base[l + 1]) l++;
    const int local = r - g.ref_base[l];
    const int Bp = local / g.na_l[l + 1], Ap = local % g.na_l[l + 1];
    const int node = g.node_base[l] + (2 * Bp) * g.na_l[l] + 2 * Ap;
    return lf_residual(g, p, c, l, node, (y >> g.bsl) * g.nbx + (x >> g.bsl),
                       ((y & (g.bs - 1)) << g.bsl) | (x & (g.bs - 1)));
}

// CSR residency, pass 1: nonzero pixels of every reference row (one wave per
// row), range-checked like the dense planes.
__global__ void __launch_bounds__(256) k_csr_count(LfGeom g, LfPtrs p, uint32_t* __restrict__ counts, int64_t rows,
                                                   int* __restrict__ status)
{
    const int64_t row = (int64_t)blockIdx.x * 4 + (threadIdx.x >> 6);
    const int lane = threadIdx.x & 63;
    if (row == 0 && threadIdx.x == 0) counts[rows] = 0;
    if (row >= rows) return;
    const int64_t rp = row / g.h;
    const int y = (int)(row - rp * g.h);
    uint32_t cnt = 0;
    bool bad = false;
    for (int x = lane; x < g.w; x += 64) {
        const int v = lf_ref_value(g, p, rp, y, x);
        cnt += v != 0;
        bad |= v < -LF_REF_LIMIT || v > LF_REF_LIMIT;
    }
#pragma unroll
    for (int o = 32; o >= 1; o >>= 1) cnt += __shfl_xor(cnt, o, 64);
    if (lane == 0) counts[row] = cnt;
    if (__ballot(bad) != 0ull && lane == 0) atomicOr(status, LF_ST_REF);
}

// CSR residency, pass 2: columns and values of every row's nonzero pixels in
// increasing column order, from the row's start (one wave per row).
__global__ void __launch_bounds__(256) k_csr_fill(LfGeom g, LfPtrs p, const uint32_t* __restrict__ rowptr,
                                                  uint16_t* __restrict__ cols, int16_t* __restrict__ vals, int64_t rows)
{
    const int64_t row = (int64_t)blockIdx.x * 4 + (threadIdx.x >> 6);
    const int lane = threadIdx.x & 63;
    if (row >= rows) return;
    const int64_t rp = row / g.h;
    const int y = (int)(row - rp * g.h);
    uint32_t at = rowptr[row];
    for (int x0 = 0; x0 < g.w; x0 += 64) {
        const int x = x0 + lane;
        const int v = x < g.w ? lf_ref_value(g, p, rp, y, x) : 0;
        const uint64_t m = __ballot(v != 0);
        if (v != 0) {
            const uint32_t k = at + (uint32_t)__popcll(m & ((1ull << lane) - 1ull));
            cols[k] = (uint16_t)x;
            vals[k] = (int16_t)v;
        }
        at += (uint32_t)__popcll(m);
    }
}

// Block descriptors of every (channel, node, block), BFS node order.  A
// descriptor holds each vector component in 12 signed bits: a motion vector
// beyond +-2047 quarter pixels (a stream can code one when 4W + 2047 is
// below its sequence's range) is flagged.
__global__ void k_load_desc(LfGeom g, LfPtrs p, uint4* __restrict__ desc, int* __restrict__ status)
{
    const int64_t total = 3 * (int64_t)g.n_nodes * g.nblk;
    bool bad = false;
    for (int64_t t = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; t < total; t += (int64_t)gridDim.x * blockDim.x) {
        const int blk = (int)(t % g.nblk);
        const int node = (int)((t / g.nblk) % g.n_nodes);
        const int c = (int)(t / ((int64_t)g.nblk * g.n_nodes));
        int l = 0;
        while (l + 1 < g.H && node < g.node_base[l]) l++;  // levels are stored H-1 first
        const int local = node - g.node_base[l];
        const int B = local / g.na_l[l], A = local % g.na_l[l];
        desc[t] = lf_make_desc(g, p, c, l, B, A, blk);
        if ((A | B) & 1) {
            int mx, my, sg;
            lf_motion(g, p, c, l, (uint32_t)(pred_ordinal(g.na_l[l], B, A) * g.nblk + blk), mx, my, sg);
            bad |= mx < -2047 || mx > 2047 || my < -2047 || my > 2047;
        }
    }
    if (bad) atomicOr(status, LF_ST_MV);
}

// Every decoded sample's Y, Co and Cg must lie within +-LF_SAMPLE_LIMIT:
// the tile renderer adds a sample's SRVs in 16-bit lanes, which is exact
// modulo 2^16, and its colour inverse (two halvings, sums of at most three
// terms) stays inside int16 from such values, so its result then equals the
// int32 decode.  Decoded values of 8-bit content are within 255 + step / 2
// of the source.  One thread per sample of every leaf view, all channels.
__global__ void k_load_check(LfGeom g, LfPtrs p, int* __restrict__ status)
{
    const int64_t plane = (int64_t)g.w * g.h;
    const int64_t total = (int64_t)g.na * g.nb * plane;
    bool bad = false;
    for (int64_t t = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; t < total; t += (int64_t)gridDim.x * blockDim.x) {
        const int64_t view = t / plane, px = t - view * plane;
        const int b = (int)(view / g.na), a = (int)(view - (int64_t)b * g.na);
        const int y = (int)(px / g.w), x = (int)(px - (int64_t)y * g.w);
        for (int c = 0; c < 3; c++) {
            const int v = lf_decode_channel<LF_RES_DENSE>(g, p, c, b, a, y, x);
            bad |= v < -LF_SAMPLE_LIMIT || v > LF_SAMPLE_LIMIT;
        }
    }
    if (bad) atomicOr(status, LF_ST_SAMPLE);
}

extern "C" lf_status lf_load_compressed_ex(const void* host_stream, size_t nbytes, int32_t flags, void* d_arena,
                                           int64_t arena_bytes, void* stream, lf_handle** out)
{
    if (!out || !d_arena) return lf_fail(LF_EINVAL, "null argument");
    *out = nullptr;
    LfLayout L;
    lf_status st = lf_parse_ex((const uint8_t*)host_stream, nbytes, flags, &L);
    if (st != LF_OK) return st;
    if (arena_bytes < L.arena)
        return lf_fail(LF_ENOMEM, "arena of %lld bytes, %lld needed", (long long)arena_bytes, (long long)L.arena);
    if (((uintptr_t)d_arena) & 255) return lf_fail(LF_EINVAL, "arena must be 256-byte aligned");
    hipStream_t s = (hipStream_t)stream;
    uint8_t* A = (uint8_t*)d_arena;
    const uint8_t* S = (const uint8_t*)host_stream;
    struct {
        int64_t dst;
        uint64_t src, n;
    } cp[4] = {{L.a_root, L.root_off, L.root_bytes},
               {L.a_table, L.table_off, L.table_bytes},
               {L.a_payload, L.payload_off, L.payload_bytes},
               {L.a_mv, L.mv_off, L.mv_bytes}};
    for (auto& c : cp)
        if (hipMemcpyAsync(A + c.dst, S + c.src, c.n, hipMemcpyHostToDevice, s) != hipSuccess)
            return lf_fail(LF_EDEVICE, "upload failed");
    lf_handle* h = new (std::nothrow) lf_handle;
    if (!h) return lf_fail(LF_EINVAL, "out of host memory");
    h->L = L;
    h->arena = A;
    h->p.root = (const int16_t*)(A + L.a_root);
    h->p.table = (const uint2*)(A + L.a_table);
    h->p.payload = (const uint32_t*)(A + L.a_payload);
    h->p.mv = (const uint32_t*)(A + L.a_mv);
    h->p.refs = (const int16_t*)(A + L.a_refs);
    h->p.desc = (L.sparse || L.chroma420) ? nullptr : (const uint4*)(A + L.a_desc);
    h->p.slots = L.sparse == LF_RES_TILES ? (const int32_t*)(A + L.a_slots) : nullptr;
    h->p.rowptr = L.sparse == LF_RES_CSR ? (const uint32_t*)(A + L.a_rowptr) : nullptr;
    h->p.cols = L.sparse == LF_RES_CSR ? (const uint16_t*)(A + L.a_cols) : nullptr;
    h->pc = LfPtrs{};
    if (L.chroma420) {
        // chroma sections follow the luma ones inside the root and table
        const int64_t luma_root = (int64_t)L.g.root_na * L.g.root_nb * L.g.w * L.g.h;
        h->pc.root = h->p.root + luma_root;
        h->pc.table = h->p.table + (int64_t)L.g.n_nodes * L.g.nblk;
        h->pc.payload = h->p.payload;
        h->pc.mv = h->p.mv;
        h->pc.refs = (const int16_t*)(A + L.a_refs_c);
    }
    const int64_t total = L.g.nch * (int64_t)L.g.n_refs * L.g.w * L.g.h;
    int64_t blocks = (total + 255) / 256;
    if (blocks > 65536) blocks = 65536;
    int* status = (int*)(A + L.a_status);
    if (hipMemsetAsync(status, 0, 256, s) != hipSuccess) {
        delete h;
        return lf_fail(LF_EDEVICE, "status clear failed");
    }
    std::vector<int32_t> slots;
    if (L.sparse == LF_RES_CSR && total > 0) {
        // row counts on the device, row starts by a prefix sum on the host
        // (load time only), then the columns and values
        const int64_t rows = 3 * (int64_t)L.g.n_refs * L.g.h;
        uint32_t* rowptr = (uint32_t*)(A + L.a_rowptr);
        const unsigned rblocks = (unsigned)((rows + 3) / 4);
        hipLaunchKernelGGL(k_csr_count, dim3(rblocks), dim3(256), 0, s, L.g, h->p, rowptr, rows, status);
        std::vector<uint32_t> rp((size_t)rows + 1);
        st = lf_check_launch("load_csr");
        if (st == LF_OK && (hipMemcpyAsync(rp.data(), rowptr, rp.size() * 4, hipMemcpyDeviceToHost, s) != hipSuccess ||
                            hipStreamSynchronize(s) != hipSuccess))
            st = lf_fail(LF_EDEVICE, "CSR row counts failed");
        uint64_t run = 0;
        for (size_t r = 0; r < rp.size() && st == LF_OK; r++) {
            const uint32_t cnt = rp[r];
            rp[r] = (uint32_t)run;
            run += cnt;
        }
        if (st == LF_OK && (int64_t)run > L.nnz_bound) st = lf_fail(LF_EFORMAT, "more nonzero reference pixels than blocks hold");
        if (st == LF_OK && hipMemcpyAsync(rowptr, rp.data(), rp.size() * 4, hipMemcpyHostToDevice, s) != hipSuccess)
            st = lf_fail(LF_EDEVICE, "CSR row starts upload failed");
        if (st == LF_OK) {
            hipLaunchKernelGGL(k_csr_fill, dim3(rblocks), dim3(256), 0, s, L.g, h->p, (const uint32_t*)rowptr,
                               (uint16_t*)(A + L.a_cols), (int16_t*)h->p.refs, rows);
            st = lf_check_launch("load_csr");
        }
        if (st != LF_OK) {
            delete h;
            return st;
        }
        h->L.nnz = (int64_t)run;
    } else if (L.sparse && total > 0) {
        slots.resize((size_t)(3 * (int64_t)L.g.n_refs * L.g.nblk));
        lf_ref_slots(S, L, slots.data());
        if (hipMemcpyAsync(A + L.a_slots, slots.data(), slots.size() * 4, hipMemcpyHostToDevice, s) != hipSuccess) {
            delete h;
            return lf_fail(LF_EDEVICE, "upload failed");
        }
        hipLaunchKernelGGL(k_load_tiles, dim3((unsigned)blocks), dim3(256), 0, s, L.g, h->p, (int16_t*)h->p.refs,
                           status);
        st = lf_check_launch("load_tiles");
        if (st != LF_OK) {
            delete h;
            return st;
        }
    } else if (total > 0) {
        hipLaunchKernelGGL(k_load_refs, dim3((unsigned)blocks), dim3(256), 0, s, L.g, h->p, (int16_t*)h->p.refs,
                           status);
        if (L.chroma420)
            hipLaunchKernelGGL(k_load_refs, dim3((unsigned)blocks), dim3(256), 0, s, L.gc, h->pc,
                               (int16_t*)h->pc.refs, status);
        st = lf_check_launch("load_refs");
        if (st != LF_OK) {
            delete h;
            return st;
        }
    }
    if (!L.sparse && !L.chroma420) {
        const int64_t nd = 3 * (int64_t)L.g.n_nodes * L.g.nblk;
        const int64_t dblocks = std::min<int64_t>((nd + 255) / 256, 65536);
        hipLaunchKernelGGL(k_load_desc, dim3((unsigned)dblocks), dim3(256), 0, s, L.g, h->p, (uint4*)(A + L.a_desc),
                           status);
        // the range check reads reference planes: only meaningful when they are in range
        const int64_t ns = (int64_t)L.g.na * L.g.nb * L.g.w * L.g.h;
        const int64_t cblocks = std::min<int64_t>((ns + 255) / 256, 65536);
        hipLaunchKernelGGL(k_load_check, dim3((unsigned)cblocks), dim3(256), 0, s, L.g, h->p, status);
        st = lf_check_launch("load_desc");
        if (st != LF_OK) {
            delete h;
            return st;
        }
    }
    // the caller may free host_stream on return: finish the copies
    int flag = 0;
    if (hipMemcpyAsync(&flag, status, sizeof(int), hipMemcpyDeviceToHost, s) != hipSuccess ||
        hipStreamSynchronize(s) != hipSuccess) {
        delete h;
        return lf_fail(LF_EDEVICE, "stream synchronise failed");
    }
    if (flag) {
        delete h;
        if (flag & LF_ST_REF) return lf_fail(LF_EFORMAT, "reference residual magnitude above %d", LF_REF_LIMIT);
        if (flag & LF_ST_MV) return lf_fail(LF_EFORMAT, "motion vector beyond +-2047 quarter pixels");
        return lf_fail(LF_EFORMAT, "decoded sample channel value beyond +-%d", LF_SAMPLE_LIMIT);
    }
    *out = h;
    return LF_OK;
}

extern "C" lf_status lf_load_compressed(const void* host_stream, size_t nbytes, void* d_arena, int64_t arena_bytes,
                                        void* stream, lf_handle** out)
{
    return lf_load_compressed_ex(host_stream, nbytes, 0, d_arena, arena_bytes, stream, out);
}

extern "C" lf_status lf_free(lf_handle* h)
{
    delete h;
    return LF_OK;
}

// Requested coordinates outside the grid are clamped and counted: one
// 64-bit counter at byte 8 of the status section, cleared at load.
static unsigned long long* lf_clamp_counter(const lf_handle* h)
{
    return reinterpret_cast<unsigned long long*>(h->arena + h->L.a_status + 8);
}

extern "C" lf_status lf_get_info(const lf_handle* h, lf_info* o)
{
    if (!h || !o) return lf_fail(LF_EINVAL, "null argument");
    const LfGeom& g = h->L.g;
    o->na = g.na;
    o->nb = g.nb;
    o->width = g.w;
    o->height = g.h;
    o->levels = g.H;
    o->block = g.bs;
    o->root_na = g.root_na;
    o->root_nb = g.root_nb;
    o->n_nodes = g.n_nodes;
    o->n_pred_records = h->L.n_rec;
    o->n_refs = g.n_refs;
    o->arena_bytes = h->L.arena;
    o->stream_bytes = h->L.stream_bytes;
    o->payload_bytes = (int64_t)h->L.payload_bytes;
    o->sparse_refs = h->L.sparse;
    o->chroma420 = h->L.chroma420;
    if (h->L.sparse == LF_RES_CSR)
        o->ref_bytes = h->L.nnz * 4 + (3 * (int64_t)g.n_refs * g.h + 1) * 4;  // values, columns, row starts
    else
        o->ref_bytes = h->L.sparse ? h->L.a_status - h->L.a_refs : h->L.a_desc - h->L.a_refs;
    unsigned long long clamps = 0;
    if (hipMemcpy(&clamps, lf_clamp_counter(h), sizeof clamps, hipMemcpyDeviceToHost) != hipSuccess)
        return lf_fail(LF_EDEVICE, "reading the clamp counter failed");
    o->clamped_coords = (int64_t)clamps;
    return LF_OK;
}

// ---------------------------------------------------------------------------
// random-access sample decoding
// ---------------------------------------------------------------------------

// each wave adds its clamped lanes to the counter with one atomic
__device__ __forceinline__ void lf_count_clamps(unsigned long long* counter, bool clamped)
{
    const unsigned long long m = __ballot(clamped);
    if (m && __lane_id() == (unsigned)(__ffsll((long long)m) - 1)) atomicAdd(counter, (unsigned long long)__popcll(m));
}

template <int RES>
__global__ void k_decode_pixels(LfGeom g, LfPtrs p, const int32_t* __restrict__ coords, int64_t n,
                                uint8_t* __restrict__ rgb, unsigned long long* __restrict__ clamps)
{
    int64_t k = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (k >= n) return;
    int4 q = reinterpret_cast<const int4*>(coords)[k];
    int b = lf_clampi(q.x, 0, g.nb - 1), a = lf_clampi(q.y, 0, g.na - 1);
    int y = lf_clampi(q.z, 0, g.h - 1), x = lf_clampi(q.w, 0, g.w - 1);
    lf_count_clamps(clamps, b != q.x || a != q.y || y != q.z || x != q.w);
    int Y = lf_decode_channel<RES>(g, p, 0, b, a, y, x);
    int Co = lf_decode_channel<RES>(g, p, 1, b, a, y, x);
    int Cg = lf_decode_channel<RES>(g, p, 2, b, a, y, x);
    int r, gg, bl;
    lf_ycocg_to_rgb(Y, Co, Cg, r, gg, bl);
    rgb[3 * k] = (uint8_t)r;
    rgb[3 * k + 1] = (uint8_t)gg;
    rgb[3 * k + 2] = (uint8_t)bl;
}

// 4:2:0 streams: luma from the luma geometry, Co and Cg up-sampled from the
// half-size chroma geometry; lod > 0 reads level-lod node images (B, A).
__global__ void k_decode_pixels420(LfGeom g, LfPtrs p, LfGeom gc, LfPtrs pc, int lod,
                                   const int32_t* __restrict__ coords, int64_t n, uint8_t* __restrict__ rgb,
                                   unsigned long long* __restrict__ clamps)
{
    int64_t k = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (k >= n) return;
    int4 q = reinterpret_cast<const int4*>(coords)[k];
    int B = lf_clampi(q.x, 0, g.nb_l[lod] - 1), A = lf_clampi(q.y, 0, g.na_l[lod] - 1);
    int y = lf_clampi(q.z, 0, g.h - 1), x = lf_clampi(q.w, 0, g.w - 1);
    lf_count_clamps(clamps, B != q.x || A != q.y || y != q.z || x != q.w);
    const int b = B << lod, a = A << lod;
    int Y = lf_decode_channel(g, p, 0, b, a, y, x, lod);
    int Co = lf_chroma_up(gc, pc, 0, b, a, y, x, lod);
    int Cg = lf_chroma_up(gc, pc, 1, b, a, y, x, lod);
    int r, gg, bl;
    lf_ycocg_to_rgb(Y, Co, Cg, r, gg, bl);
    rgb[3 * k] = (uint8_t)r;
    rgb[3 * k + 1] = (uint8_t)gg;
    rgb[3 * k + 2] = (uint8_t)bl;
}

static lf_status lf_launch_decode420(const lf_handle* h, int lod, const int32_t* d_coords, int64_t n, uint8_t* d_rgb,
                                     void* stream)
{
    const int64_t blocks = (n + 255) / 256;
    if (blocks > 0x7FFFFFFF) return lf_fail(LF_EINVAL, "too many samples");
    hipLaunchKernelGGL(k_decode_pixels420, dim3((unsigned)blocks), dim3(256), 0, (hipStream_t)stream, h->L.g, h->p,
                       h->L.gc, h->pc, lod, d_coords, n, d_rgb, lf_clamp_counter(h));
    return lf_check_launch("decode_pixels");
}

extern "C" lf_status lf_decode_pixels(const lf_handle* h, const int32_t* d_coords, int64_t n, uint8_t* d_rgb,
                                      void* stream)
{
    if (!h || n < 0) return lf_fail(LF_EINVAL, "bad argument");
    if (n == 0) return LF_OK;
    if (!d_coords || !d_rgb) return lf_fail(LF_EINVAL, "null buffer");
    if (((uintptr_t)d_coords) & 15) return lf_fail(LF_EINVAL, "coords must be 16-byte aligned");
    if (h->L.chroma420) return lf_launch_decode420(h, 0, d_coords, n, d_rgb, stream);
    int64_t blocks = (n + 255) / 256;
    if (blocks > 0x7FFFFFFF) return lf_fail(LF_EINVAL, "too many samples");
    hipLaunchKernelGGL(h->L.sparse == LF_RES_CSR     ? k_decode_pixels<LF_RES_CSR>
                       : h->L.sparse == LF_RES_TILES ? k_decode_pixels<LF_RES_TILES>
                                                     : k_decode_pixels<LF_RES_DENSE>,
                       dim3((unsigned)blocks), dim3(256),
                       0, (hipStream_t)stream, h->L.g, h->p, d_coords, n, d_rgb, lf_clamp_counter(h));
    return lf_check_launch("decode_pixels");
}

// Progressive decode: samples of the level-`lod` node images.
template <int RES>
__global__ void k_decode_nodes(LfGeom g, LfPtrs p, int lod, const int32_t* __restrict__ coords, int64_t n,
                               uint8_t* __restrict__ rgb, unsigned long long* __restrict__ clamps)
{
    int64_t k = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (k >= n) return;
    int4 q = reinterpret_cast<const int4*>(coords)[k];
    int B = lf_clampi(q.x, 0, g.nb_l[lod] - 1), A = lf_clampi(q.y, 0, g.na_l[lod] - 1);
    int y = lf_clampi(q.z, 0, g.h - 1), x = lf_clampi(q.w, 0, g.w - 1);
    lf_count_clamps(clamps, B != q.x || A != q.y || y != q.z || x != q.w);
    int Y = lf_decode_channel<RES>(g, p, 0, B << lod, A << lod, y, x, lod);
    int Co = lf_decode_channel<RES>(g, p, 1, B << lod, A << lod, y, x, lod);
    int Cg = lf_decode_channel<RES>(g, p, 2, B << lod, A << lod, y, x, lod);
    int r, gg, bl;
    lf_ycocg_to_rgb(Y, Co, Cg, r, gg, bl);
    rgb[3 * k] = (uint8_t)r;
    rgb[3 * k + 1] = (uint8_t)gg;
    rgb[3 * k + 2] = (uint8_t)bl;
}

extern "C" lf_status lf_decode_pixels_lod(const lf_handle* h, int32_t level, const int32_t* d_coords, int64_t n,
                                          uint8_t* d_rgb, void* stream)
{
    if (!h || n < 0 || level < 0 || level > h->L.g.H) return lf_fail(LF_EINVAL, "bad argument");
    if (n == 0) return LF_OK;
    if (!d_coords || !d_rgb) return lf_fail(LF_EINVAL, "null buffer");
    if (((uintptr_t)d_coords) & 15) return lf_fail(LF_EINVAL, "coords must be 16-byte aligned");
    if (h->L.chroma420) return lf_launch_decode420(h, level, d_coords, n, d_rgb, stream);
    const int64_t blocks = (n + 255) / 256;
    if (blocks > 0x7FFFFFFF) return lf_fail(LF_EINVAL, "too many samples");
    hipLaunchKernelGGL(h->L.sparse == LF_RES_CSR     ? k_decode_nodes<LF_RES_CSR>
                       : h->L.sparse == LF_RES_TILES ? k_decode_nodes<LF_RES_TILES>
                                                     : k_decode_nodes<LF_RES_DENSE>,
                       dim3((unsigned)blocks), dim3(256), 0,
                       (hipStream_t)stream, h->L.g, h->p, (int)level, d_coords, n, d_rgb, lf_clamp_counter(h));
    return lf_check_launch("decode_pixels_lod");
}

// ---------------------------------------------------------------------------
// ray coordinates (exposed for checking the renderer's arithmetic)
// ---------------------------------------------------------------------------

__global__ void k_ray_coords(const float* __restrict__ cams, int nv, int wo, int ho, float4* __restrict__ out)
{
    int64_t r = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    int64_t npix = (int64_t)wo * ho;
    if (r >= npix * nv) return;
    int v = (int)(r / npix);
    int j = (int)((r % npix) / wo), i = (int)(r % wo);
    float u, vv, s, t;
    lf_ray(cams + 18 * v, i, j, u, vv, s, t);
    out[r] = make_float4(u, vv, s, t);
}

extern "C" lf_status lf_ray_coords(const float* d_cams, int32_t n_views, int32_t width, int32_t height,
                                   float* d_uvst, void* stream)
{
    if (!d_cams || !d_uvst || n_views < 0 || width < 1 || height < 1) return lf_fail(LF_EINVAL, "bad argument");
    int64_t total = (int64_t)n_views * width * height;
    if (total == 0) return LF_OK;
    hipLaunchKernelGGL(k_ray_coords, dim3((unsigned)((total + 255) / 256)), dim3(256), 0, (hipStream_t)stream,
                       d_cams, n_views, width, height, (float4*)d_uvst);
    return lf_check_launch("ray_coords");
}
