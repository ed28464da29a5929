// HMLFC encoder (host, OpenMP): builds the compressed stream that the device
// kernels decode.  It follows the paper's pipeline (Fig. 1 caption):
//   1. reversible YCoCg per sample (Compressing HMLFC tree),
//   2. RLFC hierarchy: each level-(l+1) RKV is the rounded mean of a 2x2
//      grid-aligned cluster of level-l views, up to the tree height
//      (RLFC: Hierarchical Compression Scheme),
//   3. top-down closed loop: SRV = view - reconstructed parent RKV; the
//      (even, even) SRV of each cluster is the reference, every block of the
//      other SRVs is predicted from it by the phase-shifted search of Eq. 1-2
//      (Phase-shifted Motion Compensation), then the residual replaces the
//      block (replacement step),
//   4. uniform quantisation and the two block thresholds,
//   5. bounded-integer-sequence coding of blocks and motion vectors in BFS
//      node order (Bounded Integer Sequence Encoding; Compressed Stream
//      Structure).
// Search decisions: integer-pel full search over [-W, W]^2 for each phase,
// then a +-3 quarter-pel refinement around each phase's best; candidates rank
// by (cost, |mx| + |my|, my, mx) and phase -1 wins only on a strictly lower
// cost.  The search sums both phases in one pass and abandons a candidate as
// soon as its partial cost is strictly above the best, which never changes
// the result.
#include <omp.h>

#include <algorithm>
#include <atomic>
#include <climits>
#include <cstdio>
#include <cstdlib>
#include <cstring>
#include <vector>

#include "lf_internal.h"

namespace {

inline int floor_div(int p, int q) { return p >= 0 ? p / q : -((-p + q - 1) / q); }
inline int clampi(int v, int lo, int hi) { return v < lo ? lo : (v > hi ? hi : v); }
inline int iabs(int v) { return v < 0 ? -v : v; }

struct Key {
    int64_t cost;
    int mx, my;
};

inline bool key_less(int64_t c, int mx, int my, const Key& b)
{
    if (c != b.cost) return c < b.cost;
    int n = iabs(mx) + iabs(my), bn = iabs(b.mx) + iabs(b.my);
    if (n != bn) return n < bn;
    if (my != b.my) return my < b.my;
    return mx < b.mx;
}

// quarter-pel bilinear prediction (same rule as the decoder)
inline int qpel(const int16_t* R, int w, int h, int y, int x, int mx, int my)
{
    int X = 4 * x + mx, Y = 4 * y + my;
    int x0 = X >> 2, y0 = Y >> 2, fx = X & 3, fy = Y & 3;
    int xa = clampi(x0, 0, w - 1), xb = clampi(x0 + 1, 0, w - 1);
    int ya = clampi(y0, 0, h - 1), yb = clampi(y0 + 1, 0, h - 1);
    int acc = (4 - fx) * (4 - fy) * R[ya * w + xa] + fx * (4 - fy) * R[ya * w + xb] + (4 - fx) * fy * R[yb * w + xa] +
              fx * fy * R[yb * w + xb];
    return (acc + 8) >> 4;
}

struct MV {
    int mx, my, sg;
};

MV search_block(const int16_t* P, const int16_t* R, int w, int h, int by0, int bx0, int bs, int win, bool subpel,
                bool zero_phase)
{
    Key best[2] = {{INT64_MAX, 0, 0}, {INT64_MAX, 0, 0}};  // [0]: phase +1, [1]: phase -1
    // integer positions: both phases in one pass
    for (int dy = -win; dy <= win; dy++)
        for (int dx = -win; dx <= win; dx++) {
            int64_t cp = 0, cm = 0;
            bool interior = by0 + dy >= 0 && by0 + dy + bs <= h && bx0 + dx >= 0 && bx0 + dx + bs <= w;
            bool alive = true;
            for (int y = by0; y < by0 + bs && alive; y++) {
                const int16_t* prow = P + (int64_t)y * w;
                if (interior) {
                    const int16_t* rrow = R + (int64_t)(y + dy) * w + dx;
                    for (int x = bx0; x < bx0 + bs; x++) {
                        int pv = prow[x], rv = rrow[x];
                        cp += iabs(pv - rv);
                        cm += iabs(pv + rv);
                    }
                } else {
                    const int16_t* rrow = R + (int64_t)clampi(y + dy, 0, h - 1) * w;
                    for (int x = bx0; x < bx0 + bs; x++) {
                        int pv = prow[x], rv = rrow[clampi(x + dx, 0, w - 1)];
                        cp += iabs(pv - rv);
                        cm += iabs(pv + rv);
                    }
                }
                alive = cp <= best[0].cost || cm <= best[1].cost;
            }
            if (!alive) continue;
            if (key_less(cp, 4 * dx, 4 * dy, best[0])) best[0] = {cp, 4 * dx, 4 * dy};
            if (key_less(cm, 4 * dx, 4 * dy, best[1])) best[1] = {cm, 4 * dx, 4 * dy};
        }
    if (subpel) {
        const Key centre[2] = {best[0], best[1]};
        const int lim = 4 * win;
        for (int s = 0; s < 2; s++) {
            const int sgn = s == 0 ? 1 : -1;
            for (int ey = -3; ey <= 3; ey++)
                for (int ex = -3; ex <= 3; ex++) {
                    int qx = centre[s].mx + ex, qy = centre[s].my + ey;
                    if (qx < -lim || qx > lim || qy < -lim || qy > lim) continue;
                    if ((qx & 3) == 0 && (qy & 3) == 0) continue;
                    int64_t c = 0;
                    bool alive = true;
                    for (int y = 0; y < bs && alive; y++) {
                        for (int x = 0; x < bs; x++)
                            c += iabs(P[(int64_t)(by0 + y) * w + bx0 + x] - sgn * qpel(R, w, h, by0 + y, bx0 + x, qx, qy));
                        alive = c <= best[s].cost;
                    }
                    if (alive && key_less(c, qx, qy, best[s])) best[s] = {c, qx, qy};
                }
        }
    }
    MV r;
    int pick = best[1].cost < best[0].cost ? 1 : 0;
    r.mx = best[pick].mx;
    r.my = best[pick].my;
    r.sg = pick == 0 ? 1 : -1;
    if (zero_phase) {
        int64_t c0 = 0;
        for (int y = by0; y < by0 + bs; y++)
            for (int x = bx0; x < bx0 + bs; x++) c0 += iabs(P[(int64_t)y * w + x]);
        if (c0 < best[pick].cost) r = {0, 0, 0};
    }
    return r;
}

inline int quantise(int e, int step)
{
    int m = (iabs(e) + step / 2) / step;
    return e < 0 ? -m : m;
}

// quantise a block and apply the block threshold on sum |q * step|
void code_block(const int* e, int n, int step, int thr, int* q)
{
    int64_t energy = 0;
    for (int i = 0; i < n; i++) {
        q[i] = quantise(e[i], step);
        energy += (int64_t)iabs(q[i]) * step;
    }
    if (energy < thr)
        for (int i = 0; i < n; i++) q[i] = 0;
}

int64_t seq_bits(int mode, int64_t n)
{
    int fam = mode >> 5, b = mode & 31;
    if (fam == 0) return n * b;
    if (fam == 1) return (n + 4) / 5 * (8 + 5 * b);
    return (n + 2) / 3 * (7 + 3 * b);
}

// smallest coding of n values in [0, vmax]; ties keep the earlier family
int pick_mode(uint32_t vmax, int64_t n)
{
    int best = -1;
    int64_t bits = 0;
    const uint32_t mult[3] = {1, 3, 5};
    for (int fam = 0; fam < 3; fam++) {
        int b = 0;
        while (((uint64_t)mult[fam] << b) <= vmax) b++;
        if (b > 20) continue;
        int m = (fam << 5) | b;
        int64_t nb = seq_bits(m, n);
        if (best < 0 || nb < bits) {
            best = m;
            bits = nb;
        }
    }
    return best;
}

struct BitWriter {
    uint32_t* w;
    void put(int64_t pos, int n, uint32_t v)
    {
        for (int t = 0; t < n;) {
            int64_t p = pos + t;
            int room = 32 - (int)(p & 31), take = n - t < room ? n - t : room;
            uint32_t bits = (v >> t) & (take == 32 ? 0xFFFFFFFFu : ((1u << take) - 1u));
            w[p >> 5] |= bits << (p & 31);
            t += take;
        }
    }
};

void pack_seq(const uint32_t* v, int64_t n, int mode, uint32_t* words)
{
    BitWriter bw{words};
    const int fam = mode >> 5, b = mode & 31;
    if (fam == 0) {
        for (int64_t i = 0; i < n; i++) bw.put(i * b, b, v[i]);
        return;
    }
    const int gs = fam == 1 ? 5 : 3, hb = fam == 1 ? 8 : 7, radix = fam == 1 ? 3 : 5;
    const int64_t gbits = hb + (int64_t)gs * b;
    for (int64_t g0 = 0; g0 < n; g0 += gs) {
        int64_t base = (g0 / gs) * gbits;
        uint32_t hi = 0, scale = 1;
        for (int k = 0; k < gs; k++) {
            uint32_t val = g0 + k < n ? v[g0 + k] : 0u;
            hi += (val >> b) * scale;
            scale *= radix;
            bw.put(base + hb + (int64_t)k * b, b, val & ((1u << b) - 1u));
        }
        bw.put(base, hb, hi);
    }
}

struct Coded {
    std::vector<uint32_t> words;
    int mode = LF_MODE_ZERO;
    int16_t mn = 0;
};

void put32(uint8_t* p, uint32_t v) { memcpy(p, &v, 4); }
void put64(uint8_t* p, uint64_t v) { memcpy(p, &v, 8); }

// device workspace and stream for the motion search (null: search on the host)
struct DeviceSearch {
    void* work;
    int64_t bytes;
    void* stream;
};

lf_status encode_impl(const uint8_t* host_lf, int32_t nb, int32_t na, int32_t height, int32_t width,
                      const lf_encode_params* prm, int32_t threads, const DeviceSearch* dev, uint8_t** out_stream,
                      size_t* out_bytes)
{
    if (!host_lf || !prm || !out_stream || !out_bytes) return lf_fail(LF_EINVAL, "null argument");
    const int H = prm->levels, bs = prm->block, w = width, h = height;
    if (H < 1 || H > LF_MAX_LEVELS || bs < 1 || bs > 64 || w < 1 || h < 1 || w % bs || h % bs || na < 1 || nb < 1)
        return lf_fail(LF_EINVAL, "bad geometry");
    for (int l = 0; l < H; l++)
        if (prm->step[l] < 1 || prm->step[l] > 4096 || prm->win[l] < 0 || prm->win[l] > 255)
            return lf_fail(LF_EINVAL, "bad step/window");
    if (threads > 0) omp_set_num_threads(threads);
    // HMLFC_ENCODE_PROGRESS=1: a line on stderr after every tenth of a level's predictive blocks
    const char* pe = getenv("HMLFC_ENCODE_PROGRESS");
    const bool progress = pe && atoi(pe) != 0;
    int na_l[LF_MAX_LEVELS + 1], nb_l[LF_MAX_LEVELS + 1];
    na_l[0] = na;
    nb_l[0] = nb;
    for (int l = 0; l < H; l++) {
        na_l[l + 1] = (na_l[l] + 1) / 2;
        nb_l[l + 1] = (nb_l[l] + 1) / 2;
    }
    const int64_t plane = (int64_t)w * h;
    const int nbx = w / bs, nblk = nbx * (h / bs), n = bs * bs;
    auto views = [&](int l) { return (int64_t)na_l[l] * nb_l[l]; };

    // 1. colour: I[0] planes [3][views][h][w]
    std::vector<std::vector<int16_t>> I(H + 1);
    I[0].resize((size_t)(3 * views(0) * plane));
#pragma omp parallel for schedule(static)
    for (int64_t v = 0; v < views(0); v++)
        for (int64_t px = 0; px < plane; px++) {
            const uint8_t* s = host_lf + (v * plane + px) * 3;
            int co = (int)s[0] - (int)s[2];
            int t = s[2] + (co >> 1);
            int cg = (int)s[1] - t;
            int y = t + (cg >> 1);
            I[0][(0 * views(0) + v) * plane + px] = (int16_t)y;
            I[0][(1 * views(0) + v) * plane + px] = (int16_t)co;
            I[0][(2 * views(0) + v) * plane + px] = (int16_t)cg;
        }
    // 2. RKV pyramid: rounded mean of each 2x2 cluster (ragged at odd edges)
    for (int l = 0; l < H; l++) {
        I[l + 1].resize((size_t)(3 * views(l + 1) * plane));
#pragma omp parallel for collapse(2) schedule(static)
        for (int c = 0; c < 3; c++)
            for (int64_t pv = 0; pv < views(l + 1); pv++) {
                const int B = (int)(pv / na_l[l + 1]), A = (int)(pv % na_l[l + 1]);
                const int16_t* kid[4];
                int cnt = 0;
                for (int j = 0; j < 2; j++)
                    for (int i = 0; i < 2; i++)
                        if (2 * B + j < nb_l[l] && 2 * A + i < na_l[l])
                            kid[cnt++] = &I[l][(c * views(l) + (int64_t)(2 * B + j) * na_l[l] + 2 * A + i) * plane];
                int16_t* dst = &I[l + 1][(c * views(l + 1) + pv) * plane];
                for (int64_t px = 0; px < plane; px++) {
                    int sum = 0;
                    for (int k = 0; k < cnt; k++) sum += kid[k][px];
                    dst[px] = (int16_t)floor_div(sum + cnt / 2, cnt);
                }
            }
    }
    int node_base[LF_MAX_LEVELS];
    int64_t n_nodes = 0;
    for (int l = H - 1; l >= 0; l--) {
        node_base[l] = (int)n_nodes;
        n_nodes += views(l);
    }
    const int64_t nent = 3 * n_nodes * nblk;
    std::vector<Coded> coded((size_t)nent);
    std::vector<std::vector<MV>> mvs((size_t)(3 * H));
    int64_t npred[LF_MAX_LEVELS];
    for (int l = 0; l < H; l++) {
        npred[l] = ((int64_t)(nb_l[l] / 2) * na_l[l] + (int64_t)((nb_l[l] + 1) / 2) * (na_l[l] / 2)) * nblk;
        for (int c = 0; c < 3; c++) mvs[c * H + l].assign((size_t)npred[l], MV{0, 0, 0});
    }
    std::atomic<bool> overflow{false};
    auto code_and_store = [&](int c, int64_t node, int blk, const int* q) {
        Coded& cd = coded[(size_t)((c * n_nodes + node) * nblk + blk)];
        int qmin = q[0];
        bool nz = false;
        for (int i = 0; i < n; i++) {
            qmin = q[i] < qmin ? q[i] : qmin;
            nz |= q[i] != 0;
        }
        if (!nz) return;
        if (qmin < -32768 || qmin > 32767) overflow = true;
        uint32_t v[64 * 64], vmax = 0;
        for (int i = 0; i < n; i++) {
            v[i] = (uint32_t)(q[i] - qmin);
            vmax = v[i] > vmax ? v[i] : vmax;
        }
        int mode = pick_mode(vmax, n);
        if (mode < 0) {
            overflow = true;
            return;
        }
        cd.mode = mode;
        cd.mn = (int16_t)qmin;
        cd.words.assign((size_t)((seq_bits(mode, n) + 31) / 32), 0u);
        pack_seq(v, n, mode, cd.words.data());
    };

    // 3. closed-loop top-down coding
    std::vector<int16_t> up = I[H];
    for (int l = H - 1; l >= 0; l--) {
        const int nal = na_l[l], nbl = nb_l[l], nau = na_l[l + 1];
        const int64_t nv = views(l), nvu = views(l + 1);
        const int step = prm->step[l];
        std::vector<int16_t> S((size_t)(3 * nv * plane)), Shat((size_t)(3 * nv * plane));
#pragma omp parallel for collapse(2) schedule(static)
        for (int c = 0; c < 3; c++)
            for (int64_t v = 0; v < nv; v++) {
                const int B = (int)(v / nal), A = (int)(v % nal);
                const int16_t* src = &I[l][(c * nv + v) * plane];
                const int16_t* par = &up[(c * nvu + (int64_t)(B / 2) * nau + A / 2) * plane];
                int16_t* dst = &S[(c * nv + v) * plane];
                for (int64_t px = 0; px < plane; px++) dst[px] = (int16_t)(src[px] - par[px]);
            }
        // references
#pragma omp parallel for collapse(2) schedule(dynamic)
        for (int c = 0; c < 3; c++)
            for (int64_t pv = 0; pv < nvu; pv++) {
                const int B = 2 * (int)(pv / nau), A = 2 * (int)(pv % nau);
                const int64_t v = (int64_t)B * nal + A;
                int e[64 * 64], q[64 * 64];
                for (int k = 0; k < nblk; k++) {
                    const int by0 = (k / nbx) * bs, bx0 = (k % nbx) * bs;
                    for (int i = 0; i < n; i++) e[i] = S[(c * nv + v) * plane + (int64_t)(by0 + i / bs) * w + bx0 + i % bs];
                    code_block(e, n, step, prm->t_ref[l], q);
                    code_and_store(c, node_base[l] + v, k, q);
                    for (int i = 0; i < n; i++)
                        Shat[(c * nv + v) * plane + (int64_t)(by0 + i / bs) * w + bx0 + i % bs] = (int16_t)(q[i] * step);
                }
            }
        // predictive blocks: enumerate predictive nodes in raster order
        std::vector<int> pnodes;
        for (int B = 0; B < nbl; B++)
            for (int A = 0; A < nal; A++)
                if ((A | B) & 1) pnodes.push_back(B * nal + A);
        const int64_t items = 3 * npred[l];
        if (dev && !prm->no_mc && items > 0) {
            // every predictive block of the level in one device search
            std::vector<int32_t> work((size_t)(3 * items)), res((size_t)(4 * items));
            for (int64_t it = 0; it < items; it++) {
                const int c = (int)(it / npred[l]);
                const int64_t j = it % npred[l];
                const int v = pnodes[(size_t)(j / nblk)];
                const int B = v / nal, A = v % nal;
                work[(size_t)(3 * it)] = (int32_t)(c * nv + v);
                work[(size_t)(3 * it + 1)] = (int32_t)(c * nv + (int64_t)(B & ~1) * nal + (A & ~1));
                work[(size_t)(3 * it + 2)] = (int32_t)(j % nblk);
            }
            lf_status st = lf_search_level_device(S.data(), Shat.data(), 3 * nv, w, h, bs, prm->win[l],
                                                  prm->subpel != 0, prm->zero_phase != 0, work.data(), items,
                                                  res.data(), dev->work, dev->bytes, dev->stream);
            if (st != LF_OK) return st;
            for (int64_t it = 0; it < items; it++) {
                if (res[(size_t)(4 * it + 3)] < 0) return lf_fail(LF_EINVAL, "search input out of range");
                mvs[(size_t)((it / npred[l]) * H + l)][(size_t)(it % npred[l])] =
                    MV{res[(size_t)(4 * it)], res[(size_t)(4 * it + 1)], res[(size_t)(4 * it + 2)]};
            }
        }
        const bool searched = dev && !prm->no_mc;
        std::atomic<int64_t> done{0};
#pragma omp parallel for schedule(dynamic, 8)
        for (int64_t it = 0; it < items; it++) {
            if (progress && items >= 10) {
                const int64_t d = done.fetch_add(1) + 1;
                if (d % (items / 10) == 0)
                    fprintf(stderr, "encode: level %d, %lld of %lld predictive blocks\n", l, (long long)d, (long long)items);
            }
            const int c = (int)(it / npred[l]);
            const int64_t j = it % npred[l];
            const int v = pnodes[(size_t)(j / nblk)];
            const int k = (int)(j % nblk);
            const int B = v / nal, A = v % nal;
            const int64_t rv = (int64_t)(B & ~1) * nal + (A & ~1);
            const int16_t* P = &S[(c * nv + v) * plane];
            const int16_t* R = &Shat[(c * nv + rv) * plane];
            const int by0 = (k / nbx) * bs, bx0 = (k % nbx) * bs;
            MV m{0, 0, 0};
            if (searched)
                m = mvs[c * H + l][(size_t)j];
            else if (!prm->no_mc)
                m = search_block(P, R, w, h, by0, bx0, bs, prm->win[l], prm->subpel != 0, prm->zero_phase != 0);
            mvs[c * H + l][(size_t)j] = m;
            int e[64 * 64], q[64 * 64], pr[64 * 64];
            for (int i = 0; i < n; i++) {
                const int y = by0 + i / bs, x = bx0 + i % bs;
                pr[i] = m.sg * qpel(R, w, h, y, x, m.mx, m.my);
                e[i] = P[(int64_t)y * w + x] - pr[i];
            }
            code_block(e, n, step, prm->t_pred[l], q);
            code_and_store(c, node_base[l] + v, k, q);
            int16_t* dst = &Shat[(c * nv + v) * plane];
            for (int i = 0; i < n; i++) dst[(int64_t)(by0 + i / bs) * w + bx0 + i % bs] = (int16_t)(pr[i] + q[i] * step);
        }
        // reconstruction of level l
        std::vector<int16_t> rec((size_t)(3 * nv * plane));
#pragma omp parallel for collapse(2) schedule(static)
        for (int c = 0; c < 3; c++)
            for (int64_t v = 0; v < nv; v++) {
                const int B = (int)(v / nal), A = (int)(v % nal);
                const int16_t* par = &up[(c * nvu + (int64_t)(B / 2) * nau + A / 2) * plane];
                const int16_t* sh = &Shat[(c * nv + v) * plane];
                int16_t* dst = &rec[(c * nv + v) * plane];
                for (int64_t px = 0; px < plane; px++) dst[px] = (int16_t)(par[px] + sh[px]);
            }
        up.swap(rec);
        std::vector<int16_t>().swap(I[l]);
    }
    if (overflow) return lf_fail(LF_EINVAL, "values exceed the stream's integer ranges");

    // 4. assemble: payload word offsets in entry order
    std::vector<int64_t> woff((size_t)nent, 0);
    int64_t pw = 0;
    for (int64_t e = 0; e < nent; e++) {
        woff[(size_t)e] = pw;
        pw += (int64_t)coded[(size_t)e].words.size();
    }
    if (pw > 0xFFFFFFFFll) return lf_fail(LF_EINVAL, "payload exceeds 16 GiB");
    const int64_t payload_words = pw + 2;
    uint32_t mv_word[3][LF_MAX_LEVELS] = {}, sig_word[3][LF_MAX_LEVELS] = {};
    int mv_mode[3][LF_MAX_LEVELS] = {};
    int64_t mw = 0;
    for (int c = 0; c < 3; c++)
        for (int l = H - 1; l >= 0; l--) {
            mv_mode[c][l] = pick_mode((uint32_t)(8 * prm->win[l]), npred[l] > 0 ? 2 * npred[l] : 2);
            mv_word[c][l] = (uint32_t)mw;
            mw += (seq_bits(mv_mode[c][l], 2 * npred[l]) + 31) / 32;
            sig_word[c][l] = (uint32_t)mw;
            mw += (2 * npred[l] + 31) / 32;
        }
    const int64_t mv_words = mw + 2;
    const int64_t root_bytes = 3 * views(H) * plane * 2;
    const int64_t o_root = LF_HDR_BYTES, o_table = o_root + root_bytes, o_payload = o_table + nent * 8,
                  o_mv = o_payload + payload_words * 4, total = o_mv + mv_words * 4;
    uint8_t* s = (uint8_t*)calloc((size_t)total, 1);
    if (!s) return lf_fail(LF_EINVAL, "out of host memory");
    memcpy(s, "HMLFCv1", 8);
    put32(s + 8, LF_HDR_BYTES);
    put32(s + 12, 1);
    int32_t dims[8] = {na, nb, w, h, H, bs, 3, 4};
    memcpy(s + 16, dims, 32);
    for (int l = 0; l < H; l++) {
        put32(s + 48 + 4 * l, (uint32_t)prm->step[l]);
        put32(s + 80 + 4 * l, (uint32_t)prm->win[l]);
    }
    put64(s + 112, o_root);
    put64(s + 120, root_bytes);
    put64(s + 128, o_table);
    put64(s + 136, nent * 8);
    put64(s + 144, o_payload);
    put64(s + 152, payload_words * 4);
    put64(s + 160, o_mv);
    put64(s + 168, mv_words * 4);
    for (int c = 0; c < 3; c++)
        for (int l = 0; l < H; l++) {
            uint8_t* d = s + 176 + (c * LF_MAX_LEVELS + l) * 16;
            put32(d, mv_word[c][l]);
            put32(d + 4, sig_word[c][l]);
            put32(d + 8, (uint32_t)npred[l]);
            d[12] = (uint8_t)mv_mode[c][l];
        }
    memcpy(s + o_root, I[H].data(), (size_t)root_bytes);
    uint32_t* payload = (uint32_t*)(s + o_payload);
    for (int64_t e = 0; e < nent; e++) {
        const Coded& cd = coded[(size_t)e];
        uint8_t* t = s + o_table + 8 * e;
        if (cd.mode == LF_MODE_ZERO) {
            t[6] = LF_MODE_ZERO;
            continue;
        }
        put32(t, (uint32_t)woff[(size_t)e]);
        memcpy(t + 4, &cd.mn, 2);
        t[6] = (uint8_t)cd.mode;
        memcpy(payload + woff[(size_t)e], cd.words.data(), cd.words.size() * 4);
    }
    uint32_t* mvsec = (uint32_t*)(s + o_mv);
    for (int c = 0; c < 3; c++)
        for (int l = 0; l < H; l++) {
            if (npred[l] == 0) continue;
            const std::vector<MV>& m = mvs[c * H + l];
            std::vector<uint32_t> vals((size_t)(2 * npred[l]));
            BitWriter sw{mvsec + sig_word[c][l]};
            for (int64_t j = 0; j < npred[l]; j++) {
                vals[(size_t)(2 * j)] = (uint32_t)(m[(size_t)j].mx + 4 * prm->win[l]);
                vals[(size_t)(2 * j + 1)] = (uint32_t)(m[(size_t)j].my + 4 * prm->win[l]);
                sw.put(2 * j, 2, m[(size_t)j].sg == 1 ? 0u : (m[(size_t)j].sg == -1 ? 1u : 2u));
            }
            pack_seq(vals.data(), 2 * npred[l], mv_mode[c][l], mvsec + mv_word[c][l]);
        }
    *out_stream = s;
    *out_bytes = (size_t)total;
    return LF_OK;
}

}  // namespace

extern "C" lf_status lf_encode(const uint8_t* host_lf, int32_t nb, int32_t na, int32_t height, int32_t width,
                               const lf_encode_params* prm, int32_t threads, uint8_t** out_stream, size_t* out_bytes)
{
    return encode_impl(host_lf, nb, na, height, width, prm, threads, nullptr, out_stream, out_bytes);
}

extern "C" lf_status lf_encode_workspace_bytes(int32_t nb, int32_t na, int32_t height, int32_t width,
                                               const lf_encode_params* prm, int64_t* bytes)
{
    if (!prm || !bytes) return lf_fail(LF_EINVAL, "null argument");
    const int H = prm->levels, bs = prm->block;
    if (H < 1 || H > LF_MAX_LEVELS || bs < 1 || width < 1 || height < 1 || width % bs || height % bs || na < 1 ||
        nb < 1)
        return lf_fail(LF_EINVAL, "bad geometry");
    int64_t need = 0;
    if (!prm->no_mc) {
        int nal = na, nbl = nb;
        for (int l = 0; l < H; l++) {
            const int64_t nblk = (int64_t)(width / bs) * (height / bs);
            const int64_t npred = ((int64_t)(nbl / 2) * nal + (int64_t)((nbl + 1) / 2) * (nal / 2)) * nblk;
            need = std::max(need, lf_search_work_bytes(3 * (int64_t)nal * nbl, width, height, 3 * npred));
            nal = (nal + 1) / 2;
            nbl = (nbl + 1) / 2;
        }
    }
    *bytes = need;
    return LF_OK;
}

extern "C" lf_status lf_encode_device(const uint8_t* host_lf, int32_t nb, int32_t na, int32_t height, int32_t width,
                                      const lf_encode_params* prm, int32_t threads, void* d_work, int64_t work_bytes,
                                      void* stream, uint8_t** out_stream, size_t* out_bytes)
{
    int64_t need = 0;
    lf_status st = lf_encode_workspace_bytes(nb, na, height, width, prm, &need);
    if (st != LF_OK) return st;
    if (need > work_bytes || (need > 0 && !d_work)) return lf_fail(LF_ENOMEM, "workspace too small");
    const int bs = prm->block;
    if (!prm->no_mc) {
        if (bs != 2 && bs != 4 && bs != 8 && bs != 16 && bs != 32 && bs != 64)
            return lf_fail(LF_EINVAL, "device search needs a block size of 2, 4, 8, 16, 32 or 64");
        for (int l = 0; l < prm->levels; l++)
            if (prm->win[l] < 0 || bs + 2 * prm->win[l] + 1 > 96)
                return lf_fail(LF_EINVAL, "device search window too large at level %d", l);
    }
    const DeviceSearch dev{d_work, work_bytes, stream};
    return encode_impl(host_lf, nb, na, height, width, prm, threads, &dev, out_stream, out_bytes);
}

extern "C" void lf_encode_free(uint8_t* p) { free(p); }
