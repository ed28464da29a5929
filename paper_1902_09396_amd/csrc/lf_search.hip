// Phase-shifted motion search on the device (Phase-shifted Motion
// Compensation, Eq. 1 and 2), the encoder's costly step.
//
// For each predictive block: the integer displacement in [-W, W]^2 and phase
// sigma in {+1, -1} minimising the sum of absolute errors against the
// reconstructed reference SRV (sigma = +1: prediction +R; sigma = -1:
// prediction -R), then a +-3 quarter-pel refinement around each phase's
// best.  The decisions are the host search's: candidates rank by (cost,
// |mx| + |my|, my, mx); phase -1 wins only on a strictly lower cost; the
// optional zero phase (no prediction) only when strictly cheaper still.
//
// One wave64 per block.  The reference window (the block, W pixels on each
// side and one more for the bilinear taps; coordinates clamped to the plane,
// as the prediction clamps them) is staged in LDS as 16-bit values biased by
// 32768, twice: as pixel pairs starting at even and at odd columns, so every
// pair a candidate needs is one aligned dword.
//  - integer candidates: v_sad_u16 adds |p - r| for two pixels per
//    instruction; the -1 phase compares the packed negation of the biased
//    block, 32768 - p = -(p + 32768) mod 2^16, with the same reference pair,
//    since |p + r| = |(32768 - p) - (r + 32768)|;
//  - quarter-pel candidates: v_dot2_u32_u16 applies two bilinear weights per
//    instruction to biased taps; the weights sum to 16, so the bias passes
//    through the rounding shift exactly.  Two lanes share a candidate (eight
//    rows each), and each lane carries the lower tap row to the next row.
// A ranking key packs (cost, |mx| + |my|, my, mx) into 64 bits; each phase's
// best is a wave-wide minimum.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <vector>

#include "lf_internal.h"

namespace {

typedef unsigned short u16x2 __attribute__((ext_vector_type(2)));

constexpr int SEARCH_DMAX = 96;  // largest window side bs + 2W + 1
constexpr uint32_t BIAS2 = 0x80008000u;

__device__ __forceinline__ uint32_t pk_neg(uint32_t v)
{
    return __builtin_bit_cast(uint32_t, (u16x2)(0) - __builtin_bit_cast(u16x2, v));
}

__device__ __forceinline__ uint32_t sad2(uint32_t a, uint32_t b, uint32_t acc)
{
    return __builtin_amdgcn_sad_u16(a, b, acc);
}

__device__ __forceinline__ uint32_t dot2(uint32_t a, u16x2 w, uint32_t acc)
{
    return __builtin_amdgcn_udot2(__builtin_bit_cast(u16x2, a), w, acc, false);
}

// (cost, |mx| + |my|, my, mx), lexicographic: cost < 2^29, |mx|, |my| < 1024
__device__ __forceinline__ uint64_t mv_key(uint32_t cost, int mx, int my)
{
    const uint32_t n = (uint32_t)(abs(mx) + abs(my));
    return ((uint64_t)cost << 33) | ((uint64_t)n << 22) | ((uint64_t)(my + 1024) << 11) | (uint64_t)(mx + 1024);
}
__device__ __forceinline__ int key_mx(uint64_t k) { return (int)(k & 2047u) - 1024; }
__device__ __forceinline__ int key_my(uint64_t k) { return (int)((k >> 11) & 2047u) - 1024; }

__device__ __forceinline__ uint64_t wave_min64(uint64_t v)
{
#pragma unroll
    for (int o = 32; o >= 1; o >>= 1) {
        const uint64_t t = __shfl_xor(v, o, 64);
        v = t < v ? t : v;
    }
    return v;
}

__device__ __forceinline__ uint32_t wave_sum32(uint32_t v)
{
#pragma unroll
    for (int o = 32; o >= 1; o >>= 1) v += __shfl_xor(v, o, 64);
    return v;
}

// Window rows hold Dj dwords per copy: pairs starting at columns 0, 2, 4, ..
// (even copy) and 1, 3, 5, .. (odd copy).  Dj is odd, so neighbouring rows
// fall in different banks.
__host__ __device__ inline int window_dwords(int D) { return (D / 2) | 1; }

__host__ __device__ inline int search_lds_dwords(int bs, int win)
{
    const int D = bs + 2 * win + 1;
    return 2 * D * window_dwords(D) + bs * bs;
}

template <int BS>
__global__ void __launch_bounds__(64, BS >= 32 ? 3 : 8) k_mc_search(const int16_t* __restrict__ pred, const int16_t* __restrict__ ref,
                                                  int64_t n_pred, int64_t n_ref, int w, int h, int win, int subpel,
                                                  int zero_phase, const int32_t* __restrict__ items, int64_t n,
                                                  int32_t* __restrict__ out)
{
    extern __shared__ uint32_t lds[];
    // XCD-contiguous item ranges: neighbouring blocks share reference rows in L2
    const int64_t per_xcd = (int64_t)gridDim.x >> 3;
    const int64_t it = (int64_t)(blockIdx.x & 7) * per_xcd + (blockIdx.x >> 3);
    if (it >= n) return;
    const int lane = threadIdx.x;
    const int D = BS + 2 * win + 1, Dj = window_dwords(D);
    uint32_t* E = lds;
    uint32_t* O = lds + D * Dj;
    constexpr int HB = BS / 2;  // pixel pairs per block row
    uint32_t* Pb = lds + 2 * D * Dj;
    uint32_t* Pn = Pb + BS * HB;  // negated block: 32768 - p

    const int64_t pi = items[3 * it], ri = items[3 * it + 1];
    const int k = items[3 * it + 2];
    const int nbx = w / BS, nblk = nbx * (h / BS);
    if (pi < 0 || pi >= n_pred || ri < 0 || ri >= n_ref || k < 0 || k >= nblk) {
        if (lane == 0) reinterpret_cast<int4*>(out)[it] = make_int4(0, 0, 0, -2);
        return;
    }
    const int by0 = (k / nbx) * BS, bx0 = (k - (k / nbx) * nbx) * BS;
    const int64_t plane = (int64_t)w * h;
    const int16_t* P = pred + pi * plane;
    const int16_t* R = ref + ri * plane;

    bool bad = false;
    for (int e = lane; e < D * Dj; e += 64) {
        const int ry = e / Dj, j = e - ry * Dj;
        const int16_t* row = R + (int64_t)min(max(by0 - win + ry, 0), h - 1) * w;
        const int c0 = bx0 - win + 2 * j;
        const int v0 = row[min(max(c0, 0), w - 1)], v1 = row[min(max(c0 + 1, 0), w - 1)],
                  v2 = row[min(max(c0 + 2, 0), w - 1)];
        E[e] = (uint32_t)(v0 + 32768) | ((uint32_t)(v1 + 32768) << 16);
        O[e] = (uint32_t)(v1 + 32768) | ((uint32_t)(v2 + 32768) << 16);
    }
    for (int e = lane; e < BS * HB; e += 64) {
        const int y = e / HB, i = e - y * HB;
        const int16_t* px = P + (int64_t)(by0 + y) * w + bx0 + 2 * i;
        const int p0 = px[0], p1 = px[1];
        bad |= p0 == -32768 || p1 == -32768;
        Pb[e] = (uint32_t)(p0 + 32768) | ((uint32_t)(p1 + 32768) << 16);
        Pn[e] = (uint32_t)(32768 - p0) | ((uint32_t)(32768 - p1) << 16);
    }
    bad = __ballot(bad) != 0;
    __syncthreads();

    // ---- integer displacements, both phases in one pass ----
    // A task is one window row offset dy and three offsets dx0, dx0 + 2,
    // dx0 + 4 of one parity: the three share the reference dwords of a row
    // (offset dx0 + 2u starts u dwords later), so each loaded dword serves
    // six absolute-difference instructions.
    const int ne = win + 1, no = win;  // even / odd offsets in [0, 2W]
    const int ge = (ne + 2) / 3, go = (no + 2) / 3, gpr = ge + go;
    const int n_tasks = (2 * win + 1) * gpr;
    uint64_t bestp = ~0ull, bestm = ~0ull;
    for (int t = lane; t - lane < n_tasks; t += 64) {
        const bool active = t < n_tasks;
        const int tt = active ? t : 0;
        const int dy = tt / gpr, g = tt - dy * gpr;
        const int par = g >= ge;
        const int dx0 = par + 6 * (par ? g - ge : g);
        const uint32_t* r = lds + (par ? D * Dj : 0) + dy * Dj + (dx0 >> 1);
        uint32_t acc[3][2] = {{0, 0}, {0, 0}, {0, 0}};
#pragma unroll 2
        for (int y = 0; y < BS; y++) {
            uint32_t rv[HB + 2];
#pragma unroll
            for (int i = 0; i < HB + 2; i++) rv[i] = r[y * Dj + i];
            // the block row is the same for every lane: scalar loads from the
            // plane (4-byte aligned: w and bx0 are even), biased and negated
            // per 16-bit half in scalar registers
            const uint32_t* prow = reinterpret_cast<const uint32_t*>(P + (int64_t)(by0 + y) * w + bx0);
#pragma unroll
            for (int i = 0; i < HB; i++) {
                const uint32_t raw = prow[i];
                const uint32_t pp = raw ^ BIAS2;
                const uint32_t pm = ((0x8000u - (raw & 0xFFFFu)) & 0xFFFFu) | ((0x8000u - (raw >> 16)) << 16);
#pragma unroll
                for (int u = 0; u < 3; u++) {
                    acc[u][0] = sad2(pp, rv[i + u], acc[u][0]);
                    acc[u][1] = sad2(pm, rv[i + u], acc[u][1]);
                }
            }
        }
        if (active) {
#pragma unroll
            for (int u = 0; u < 3; u++) {
                const int dx = dx0 + 2 * u;
                if (dx <= 2 * win) {
                    const int mx = 4 * (dx - win), my = 4 * (dy - win);
                    const uint64_t kp = mv_key(acc[u][0], mx, my), km = mv_key(acc[u][1], mx, my);
                    bestp = kp < bestp ? kp : bestp;
                    bestm = km < bestm ? km : bestm;
                }
            }
        }
    }
    bestp = wave_min64(bestp);
    bestm = wave_min64(bestm);

    // ---- quarter-pel refinement: 48 offsets around each phase's best ----
    // 96 candidates x 2 row halves = 3 rounds of the wave; lanes 2m and 2m + 1
    // take the two halves of one candidate
    if (subpel && win > 0) {
        const int lim = 4 * win;
        const int cxp = key_mx(bestp), cyp = key_my(bestp), cxm = key_mx(bestm), cym = key_my(bestm);
        uint64_t kq0 = ~0ull, kq1 = ~0ull;
        constexpr int HR = BS / 2;  // rows per half
        for (int u = lane; u < 192; u += 64) {
            const int c = u >> 1, half = u & 1;
            const int s = c >= 48;
            const int o = c - 48 * s;
            const int oo = o + (o >= 24);  // skip the centre of the 7x7 neighbourhood
            const int qx = (s ? cxm : cxp) + oo % 7 - 3, qy = (s ? cym : cyp) + oo / 7 - 3;
            const bool ok = qx >= -lim && qx <= lim && qy >= -lim && qy <= lim;
            uint32_t acc = 0;
            if (ok) {
                const int fx = qx & 3, fy = qy & 3;
                const int ox = win + (qx >> 2), oy = win + (qy >> 2) + half * HR;  // window position of the first tap
                const u16x2 wa = {(unsigned short)((4 - fx) * (4 - fy)), (unsigned short)(fx * (4 - fy))};
                const u16x2 wb = {(unsigned short)((4 - fx) * fy), (unsigned short)(fx * fy)};
                // pixel x of a row starts its tap pair at column ox + x: even x in
                // the copy of ox's parity, odd x in the other one
                const uint32_t* A = ((ox & 1) ? O : E) + (ox >> 1) + oy * Dj;
                const uint32_t* B = ((ox & 1) ? E : O) + ((ox + 1) >> 1) + oy * Dj;
                const uint32_t* Pp = (s ? Pn : Pb) + half * HR * HB;
                uint32_t a0[HB], b0[HB];
#pragma unroll
                for (int i = 0; i < HB; i++) {
                    a0[i] = A[i];
                    b0[i] = B[i];
                }
                for (int y = 0; y < HR; y++) {
                    const int r1 = (y + 1) * Dj;
#pragma unroll
                    for (int i = 0; i < HB; i++) {
                        const uint32_t a1 = A[r1 + i], b1 = B[r1 + i];
                        const uint32_t t0 = dot2(a0[i], wa, dot2(a1, wb, 8u)) >> 4;
                        const uint32_t t1 = dot2(b0[i], wa, dot2(b1, wb, 8u)) >> 4;
                        acc = sad2(Pp[y * HB + i], t0 | (t1 << 16), acc);
                        a0[i] = a1;
                        b0[i] = b1;
                    }
                }
            }
            acc += __shfl_xor(acc, 1, 64);
            if (ok && half == 0) {
                const uint64_t key = mv_key(acc, qx, qy);
                if (s)
                    kq1 = key < kq1 ? key : kq1;
                else
                    kq0 = key < kq0 ? key : kq0;
            }
        }
        const uint64_t k0 = wave_min64(kq0), k1 = wave_min64(kq1);
        bestp = k0 < bestp ? k0 : bestp;
        bestm = k1 < bestm ? k1 : bestm;
    }

    uint32_t z = 0;
    if (zero_phase) {
        for (int e = lane; e < BS * HB; e += 64) z = sad2(Pb[e], BIAS2, z);
        z = wave_sum32(z);
    }
    if (lane == 0) {
        const uint32_t cp = (uint32_t)(bestp >> 33), cm = (uint32_t)(bestm >> 33);
        const bool minus = cm < cp;
        const uint64_t kb = minus ? bestm : bestp;
        int4 r = make_int4(key_mx(kb), key_my(kb), minus ? -1 : 1, (int)(minus ? cm : cp));
        if (zero_phase && z < (uint32_t)r.w) r = make_int4(0, 0, 0, (int)z);
        if (bad) r = make_int4(0, 0, 0, -1);
        reinterpret_cast<int4*>(out)[it] = r;
    }
}

template <int BS>
void launch_search(const int16_t* pred, const int16_t* ref, int64_t n_pred, int64_t n_ref, int w, int h, int win,
                   int subpel, int zero_phase, const int32_t* items, int64_t n, int32_t* out, hipStream_t s)
{
    const int64_t grid = ((n + 7) / 8) * 8;
    const size_t lds = (size_t)search_lds_dwords(BS, win) * 4;
    hipLaunchKernelGGL(k_mc_search<BS>, dim3((unsigned)grid), dim3(64), lds, s, pred, ref, n_pred, n_ref, w, h, win,
                       subpel, zero_phase, items, n, out);
}

lf_status search_args(int32_t w, int32_t h, int32_t bs, int32_t win, int64_t n)
{
    if (w < 1 || h < 1 || n < 0) return lf_fail(LF_EINVAL, "bad argument");
    if (bs != 2 && bs != 4 && bs != 8 && bs != 16 && bs != 32 && bs != 64)
        return lf_fail(LF_EINVAL, "block size must be 2, 4, 8, 16, 32 or 64");
    if (w % bs || h % bs) return lf_fail(LF_EINVAL, "plane sides must be multiples of the block size");
    if (win < 0 || bs + 2 * win + 1 > SEARCH_DMAX)
        return lf_fail(LF_EINVAL, "search window too large (block + 2W + 1 must be at most %d)", SEARCH_DMAX);
    if ((n + 7) / 8 * 8 > 0x7FFFFFFF) return lf_fail(LF_EINVAL, "too many blocks");
    return LF_OK;
}

lf_status launch_any(const int16_t* pred, const int16_t* ref, int64_t n_pred, int64_t n_ref, int w, int h, int bs,
                     int win, int subpel, int zero_phase, const int32_t* items, int64_t n, int32_t* out,
                     hipStream_t s)
{
    switch (bs) {
        case 2: launch_search<2>(pred, ref, n_pred, n_ref, w, h, win, subpel, zero_phase, items, n, out, s); break;
        case 4: launch_search<4>(pred, ref, n_pred, n_ref, w, h, win, subpel, zero_phase, items, n, out, s); break;
        case 8: launch_search<8>(pred, ref, n_pred, n_ref, w, h, win, subpel, zero_phase, items, n, out, s); break;
        case 16: launch_search<16>(pred, ref, n_pred, n_ref, w, h, win, subpel, zero_phase, items, n, out, s); break;
        case 32: launch_search<32>(pred, ref, n_pred, n_ref, w, h, win, subpel, zero_phase, items, n, out, s); break;
        default: launch_search<64>(pred, ref, n_pred, n_ref, w, h, win, subpel, zero_phase, items, n, out, s); break;
    }
    return lf_check_launch("mc_search");
}

}  // namespace

extern "C" lf_status lf_mc_search(const int16_t* d_pred, int64_t n_pred, const int16_t* d_ref, int64_t n_ref,
                                  int32_t width, int32_t height, int32_t block, int32_t win, int32_t subpel,
                                  int32_t zero_phase, const int32_t* d_items, int64_t n, int32_t* d_out, void* stream)
{
    lf_status st = search_args(width, height, block, win, n);
    if (st != LF_OK) return st;
    if (n == 0) return LF_OK;
    if (!d_pred || !d_ref || !d_items || !d_out || n_pred < 1 || n_ref < 1) return lf_fail(LF_EINVAL, "null buffer");
    if (((uintptr_t)d_out) & 15) return lf_fail(LF_EINVAL, "output must be 16-byte aligned");
    return launch_any(d_pred, d_ref, n_pred, n_ref, width, height, block, win, subpel != 0, zero_phase != 0, d_items,
                      n, d_out, (hipStream_t)stream);
}

lf_status lf_search_launch(const int16_t* pred, const int16_t* ref, int64_t n_pred, int64_t n_ref, int w, int h,
                           int bs, int win, int subpel, int zero_phase, const int32_t* items, int64_t n, int32_t* out,
                           void* stream)
{
    lf_status st = search_args(w, h, bs, win, n);
    if (st != LF_OK || n == 0) return st;
    return launch_any(pred, ref, n_pred, n_ref, w, h, bs, win, subpel != 0, zero_phase != 0, items, n, out,
                      (hipStream_t)stream);
}
