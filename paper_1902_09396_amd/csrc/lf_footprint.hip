// Per-view footprint accounting (see lf_footprint_bytes in hmlfc.h): mark
// what one view reads, then weigh the marks.  Used for roofline figures, not
// on the render path.
#include <hip/hip_runtime.h>

#include <mutex>
#include <vector>

#include "lf_internal.h"

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
    if (lf_status cs = lf_require_full_chroma(h, "lf_footprint_bytes")) return cs;
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

// ---------------------------------------------------------------------------
// Allocation-free variant: the marks and partial sums live in a file-scope
// device array, per-view totals are written to a caller's device buffer.
// ---------------------------------------------------------------------------

namespace {

constexpr int64_t FP_PARTS = 1024;
constexpr int64_t FP_SCRATCH_BYTES = LF_FOOTPRINT_SCRATCH_MAX;

// Per GPU: the marks (2 * entries + root blocks bytes, from byte 0) and the
// workgroup partial sums (FP_PARTS doubles, at the end).
__device__ __align__(256) uint8_t scratch[FP_SCRATCH_BYTES];

constexpr int kMaxDevices = 64;
std::mutex g_scratch_mu;
uint8_t* g_scratch_ptr[kMaxDevices];  // device address of `scratch` on each GPU, set once

// view total = 12 bytes per ray + the partial sums in index order (fixed order: deterministic)
__global__ void k_fp_total(const double* __restrict__ partial, int nparts, double rays_bytes, double* __restrict__ out)
{
    if (threadIdx.x == 0 && blockIdx.x == 0) {
        double tot = rays_bytes;
        for (int k = 0; k < nparts; k++) tot += partial[k];
        *out = tot;
    }
}

lf_status scratch_address(uint8_t** out)
{
    int dev = -1;
    if (hipGetDevice(&dev) != hipSuccess || dev < 0 || dev >= kMaxDevices)
        return lf_fail(LF_EDEVICE, "no current device");
    std::lock_guard<std::mutex> lock(g_scratch_mu);
    if (!g_scratch_ptr[dev]) {
        void* ptr = nullptr;
        hipError_t e = hipGetSymbolAddress(&ptr, HIP_SYMBOL(scratch));
        if (e != hipSuccess || !ptr)
            return lf_fail(LF_EDEVICE, "hipGetSymbolAddress(scratch): %s", hipGetErrorString(e));
        g_scratch_ptr[dev] = (uint8_t*)ptr;
    }
    *out = g_scratch_ptr[dev];
    return LF_OK;
}

}  // namespace

extern "C" lf_status lf_footprint_bytes_noalloc(const lf_handle* h, const float* d_cams, int32_t n_views,
                                                int32_t width, int32_t height, double* d_out, void* stream)
{
    if (!h || n_views < 0 || width < 1 || height < 1) return lf_fail(LF_EINVAL, "bad argument");
    if (lf_status cs = lf_require_full_chroma(h, "lf_footprint_bytes_noalloc")) return cs;
    if (n_views == 0) return LF_OK;
    if (!d_cams || !d_out) return lf_fail(LF_EINVAL, "null buffer");
    const LfGeom& g = h->L.g;
    const int64_t n_ent = 3 * (int64_t)g.n_nodes * g.nblk;
    const int64_t n_root = 3 * (int64_t)g.root_na * g.root_nb * g.nblk;
    const int64_t marks = 2 * n_ent + n_root;
    const int64_t parts_off = FP_SCRATCH_BYTES - FP_PARTS * (int64_t)sizeof(double);
    if (marks > parts_off)
        return lf_fail(LF_EINVAL, "light field needs %lld bytes of footprint marks; the allocation-free call holds %lld",
                       (long long)marks, (long long)parts_off);
    uint8_t* buf = nullptr;
    lf_status st = scratch_address(&buf);
    if (st != LF_OK) return st;
    double* part = (double*)(buf + parts_off);
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
    hipStream_t s = (hipStream_t)stream;
    const int64_t rays = (int64_t)width * height;
    for (int v = 0; v < n_views; v++) {
        hipLaunchKernelGGL(k_fill_u8, dim3(1024), dim3(256), 0, s, buf, marks);
        hipLaunchKernelGGL(k_fp_mark, dim3((unsigned)((rays + 255) / 256)), dim3(256), 0, s, g, h->p, d_cams + 18 * v,
                           width, height, buf, buf + n_ent, buf + 2 * n_ent);
        hipLaunchKernelGGL(k_fp_sum, dim3((unsigned)FP_PARTS), dim3(256), 0, s, g, h->p, w, buf, buf + n_ent,
                           buf + 2 * n_ent, n_ent, n_root, part);
        hipLaunchKernelGGL(k_fp_total, dim3(1), dim3(64), 0, s, (const double*)part, (int)FP_PARTS, 12.0 * (double)rays,
                           d_out + v);
        st = lf_check_launch("footprint_noalloc");
        if (st != LF_OK) return st;
    }
    return LF_OK;
}
