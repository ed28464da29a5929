/*
 * HMLFC CPU oracle: colour transform, hierarchy, motion compensation, block
 * coding, stream writer/reader and the two decoders.  TEST INFRASTRUCTURE ONLY.
 */
#include <stdlib.h>
#include <string.h>

#include "internal.h"

/* ------------------------------------------------------------------ */
/* integer helpers                                                     */
/* ------------------------------------------------------------------ */

int orc_asr(int x, int s)
{
    int d = 1 << s;
    return x >= 0 ? x / d : -((-x + d - 1) / d);
}

int orc_fdiv(int p, int q)
{
    return p >= 0 ? p / q : -((-p + q - 1) / q);
}

int orc_clampi(int v, int lo, int hi)
{
    return v < lo ? lo : (v > hi ? hi : v);
}

static int iabs(int v) { return v < 0 ? -v : v; }

/* ------------------------------------------------------------------ */
/* Colour: reversible YCoCg lifting (Compressing HMLFC tree).          */
/* ------------------------------------------------------------------ */

void orc_ycocg_fwd(int r, int g, int b, int* y, int* co, int* cg)
{
    int t;
    *co = r - b;
    t = b + orc_asr(*co, 1);
    *cg = g - t;
    *y = t + orc_asr(*cg, 1);
}

void orc_ycocg_inv(int y, int co, int cg, int* r, int* g, int* b)
{
    int t = y - orc_asr(cg, 1);
    *g = cg + t;
    *b = t - orc_asr(co, 1);
    *r = *b + co;
}

void orc_ycocg_fwd_n(const int32_t* rgb, int64_t n, int32_t* ycc)
{
    for (int64_t i = 0; i < n; i++) orc_ycocg_fwd(rgb[3 * i], rgb[3 * i + 1], rgb[3 * i + 2], &ycc[3 * i], &ycc[3 * i + 1], &ycc[3 * i + 2]);
}

void orc_ycocg_inv_n(const int32_t* ycc, int64_t n, int32_t* rgb)
{
    for (int64_t i = 0; i < n; i++) orc_ycocg_inv(ycc[3 * i], ycc[3 * i + 1], ycc[3 * i + 2], &rgb[3 * i], &rgb[3 * i + 1], &rgb[3 * i + 2]);
}

/* ------------------------------------------------------------------ */
/* Hierarchy geometry (RLFC: Hierarchical Compression Scheme).         */
/* Level l+1 clusters the 2x2 grid-aligned views of level l.           */
/* ------------------------------------------------------------------ */

void orc_level_grid(int na, int nb, int H, int* na_l, int* nb_l)
{
    na_l[0] = na;
    nb_l[0] = nb;
    for (int l = 0; l < H; l++) {
        na_l[l + 1] = (na_l[l] + 1) / 2;
        nb_l[l + 1] = (nb_l[l] + 1) / 2;
    }
}

/* A node (B, A) of a level is predictive when it is not the (even, even)
 * member of its 2x2 cluster.  Its ordinal among the predictive nodes of the
 * level, counted in raster order. */
int64_t orc_pred_ordinal(int na_l, int B, int A)
{
    int64_t odd_rows = B / 2, even_rows = (B + 1) / 2;
    int64_t n = odd_rows * na_l + even_rows * (na_l / 2);
    return n + ((B & 1) ? A : A / 2);
}

int64_t orc_pred_nodes(int na_l, int nb_l)
{
    return (int64_t)(nb_l / 2) * na_l + (int64_t)((nb_l + 1) / 2) * (na_l / 2);
}

/* ------------------------------------------------------------------ */
/* Quarter-pel bilinear prediction (sub-pel motion compensation is     */
/* named in Future Work; integer shifts are the fx = fy = 0 case).     */
/* ------------------------------------------------------------------ */

int32_t orc_qpel(const int32_t* plane, int w, int h, int y, int x, int mx, int my)
{
    int X = 4 * x + mx, Y = 4 * y + my;
    int x0 = orc_asr(X, 2), y0 = orc_asr(Y, 2);
    int fx = X - 4 * x0, fy = Y - 4 * y0;
    int xa = orc_clampi(x0, 0, w - 1), xb = orc_clampi(x0 + 1, 0, w - 1);
    int ya = orc_clampi(y0, 0, h - 1), yb = orc_clampi(y0 + 1, 0, h - 1);
    int32_t acc = (4 - fx) * (4 - fy) * plane[(int64_t)ya * w + xa]
                + fx * (4 - fy) * plane[(int64_t)ya * w + xb]
                + (4 - fx) * fy * plane[(int64_t)yb * w + xa]
                + fx * fy * plane[(int64_t)yb * w + xb];
    return orc_asr(acc + 8, 4);
}

/* ------------------------------------------------------------------ */
/* Phase-shifted motion search (Phase-shifted Motion Compensation,     */
/* Eq. 1 and 2).  sigma = +1 is the subtractive error (prediction +R), */
/* sigma = -1 the additive one (prediction -R).  Candidates are ranked */
/* by (cost, |mx|+|my|, my, mx); equal costs across the two phases     */
/* keep sigma = +1, the case the paper lists first.                    */
/* ------------------------------------------------------------------ */

static int better(int64_t c, int mx, int my, int64_t bc, int bmx, int bmy)
{
    if (c != bc) return c < bc;
    int n = iabs(mx) + iabs(my), bn = iabs(bmx) + iabs(bmy);
    if (n != bn) return n < bn;
    if (my != bmy) return my < bmy;
    return mx < bmx;
}

/* Eq. 1 (sigma = +1) and Eq. 2 (sigma = -1) cost of one candidate: the sum
 * over the block of |P - sigma * Q(R; mx, my)|. */
static int64_t block_cost(const int32_t* p, const int32_t* r, int w, int h, int by0, int bx0, int bs,
                          int mx, int my, int sigma)
{
    int64_t s = 0;
    for (int y = by0; y < by0 + bs; y++)
        for (int x = bx0; x < bx0 + bs; x++) {
            int32_t pred = sigma * orc_qpel(r, w, h, y, x, mx, my);
            s += iabs(p[(int64_t)y * w + x] - pred);
        }
    return s;
}

int64_t orc_mc_search(const int32_t* p, const int32_t* r, int w, int h, int by0, int bx0, int bs,
                      int win, int subpel, int zero_phase, int* mx, int* my, int* sigma)
{
    /* index 0: sigma = +1 (Eq. 1, subtractive error), index 1: sigma = -1 (Eq. 2, additive error) */
    int64_t best_cost[2];
    int best_mx[2], best_my[2];
    const int sig[2] = {+1, -1};
    for (int si = 0; si < 2; si++) {
        /* every whole-pixel shift in [-W, W]^2 */
        int64_t bc = INT64_MAX;
        int bmx = 0, bmy = 0;
        for (int dy = -win; dy <= win; dy++)
            for (int dx = -win; dx <= win; dx++) {
                int64_t c = block_cost(p, r, w, h, by0, bx0, bs, 4 * dx, 4 * dy, sig[si]);
                if (bc == INT64_MAX || better(c, 4 * dx, 4 * dy, bc, bmx, bmy)) {
                    bc = c;
                    bmx = 4 * dx;
                    bmy = 4 * dy;
                }
            }
        /* then the quarter-pel positions within +-3 of that phase's whole-pixel best */
        if (subpel) {
            const int cmx = bmx, cmy = bmy;
            for (int ey = -3; ey <= 3; ey++)
                for (int ex = -3; ex <= 3; ex++) {
                    int qx = cmx + ex, qy = cmy + ey;
                    if (qx < -4 * win || qx > 4 * win || qy < -4 * win || qy > 4 * win) continue;
                    if ((qx & 3) == 0 && (qy & 3) == 0) continue; /* whole-pixel positions already ranked */
                    int64_t c = block_cost(p, r, w, h, by0, bx0, bs, qx, qy, sig[si]);
                    if (better(c, qx, qy, bc, bmx, bmy)) {
                        bc = c;
                        bmx = qx;
                        bmy = qy;
                    }
                }
        }
        best_cost[si] = bc;
        best_mx[si] = bmx;
        best_my[si] = bmy;
    }
    int pick = best_cost[1] < best_cost[0] ? 1 : 0;
    *mx = best_mx[pick];
    *my = best_my[pick];
    *sigma = sig[pick];
    int64_t cost = best_cost[pick];
    if (zero_phase) {
        int64_t c0 = 0;
        for (int y = by0; y < by0 + bs; y++)
            for (int x = bx0; x < bx0 + bs; x++) c0 += iabs(p[(int64_t)y * w + x]);
        if (c0 < cost) {
            *mx = 0;
            *my = 0;
            *sigma = 0;
            cost = c0;
        }
    }
    return cost;
}

/* ------------------------------------------------------------------ */
/* Bounded integer sequence coding (Bounded Integer Sequence Encoding).*/
/* Mode byte: family in bits 7..5 (0 plain bits, 1 trits, 2 quints),   */
/* b in bits 4..0.  Trit groups hold 5 values: an 8-bit base-3 field   */
/* then five b-bit low parts; quint groups hold 3 values: a 7-bit      */
/* base-5 field then three b-bit low parts.  LSB-first bit order.      */
/* ------------------------------------------------------------------ */

static uint32_t read_bits(const uint32_t* words, int64_t pos, int n)
{
    uint32_t v = 0;
    for (int t = 0; t < n; t++) {
        int64_t p = pos + t;
        uint32_t bit = (words[p >> 5] >> (p & 31)) & 1u;
        v |= bit << t;
    }
    return v;
}

static void write_bits(uint32_t* words, int64_t pos, int n, uint32_t v)
{
    for (int t = 0; t < n; t++) {
        int64_t p = pos + t;
        if ((v >> t) & 1u) words[p >> 5] |= 1u << (p & 31);
    }
}

int64_t orc_bise_bits(int mode, int n)
{
    int fam = mode >> 5, b = mode & 31;
    if (mode == ORC_INSIGNIFICANT) return 0;
    if (fam == 0) return (int64_t)n * b;
    if (fam == 1) return (int64_t)((n + 4) / 5) * (8 + 5 * b);
    return (int64_t)((n + 2) / 3) * (7 + 3 * b);
}

/* Smallest coding of n values in [0, vmax]; ties keep the earlier family. */
static int choose_mode(uint32_t vmax, int n)
{
    int best = -1;
    int64_t best_bits = 0;
    for (int fam = 0; fam < 3; fam++) {
        uint32_t mult = fam == 0 ? 1 : (fam == 1 ? 3 : 5);
        int b = 0;
        while ((uint64_t)mult << b <= vmax) b++;
        if (b > 20) continue;
        int mode = (fam << 5) | b;
        int64_t bits = orc_bise_bits(mode, n);
        if (best < 0 || bits < best_bits) {
            best = mode;
            best_bits = bits;
        }
    }
    return best;
}

int orc_bise_choose(const uint32_t* v, int n)
{
    uint32_t vmax = 0;
    for (int i = 0; i < n; i++)
        if (v[i] > vmax) vmax = v[i];
    return choose_mode(vmax, n);
}

void orc_bise_pack(const uint32_t* v, int n, int mode, uint32_t* words)
{
    int fam = mode >> 5, b = mode & 31;
    if (fam == 0) {
        for (int i = 0; i < n; i++) write_bits(words, (int64_t)i * b, b, v[i]);
        return;
    }
    int gsz = fam == 1 ? 5 : 3, hb = fam == 1 ? 8 : 7, radix = fam == 1 ? 3 : 5;
    int ngroups = (n + gsz - 1) / gsz;
    for (int g = 0; g < ngroups; g++) {
        int64_t base = (int64_t)g * (hb + gsz * b);
        uint32_t field = 0, scale = 1;
        for (int k = 0; k < gsz; k++) {
            int i = g * gsz + k;
            uint32_t val = i < n ? v[i] : 0;
            field += (val >> b) * scale;
            scale *= radix;
            write_bits(words, base + hb + (int64_t)k * b, b, val & ((1u << b) - 1u));
        }
        write_bits(words, base, hb, field);
    }
}

uint32_t orc_bise_get(const uint32_t* words, int mode, int i)
{
    int fam = mode >> 5, b = mode & 31;
    if (fam == 0) return read_bits(words, (int64_t)i * b, b);
    int gsz = fam == 1 ? 5 : 3, hb = fam == 1 ? 8 : 7, radix = fam == 1 ? 3 : 5;
    int g = i / gsz, k = i % gsz;
    int64_t base = (int64_t)g * (hb + gsz * b);
    uint32_t field = read_bits(words, base, hb);
    for (int t = 0; t < k; t++) field /= radix;
    uint32_t hi = field % radix;
    uint32_t lo = read_bits(words, base + hb + (int64_t)k * b, b);
    return (hi << b) | lo;
}

/* Sequential decode with a running bit cursor (the full decoder's path). */
void orc_bise_unpack(const uint32_t* words, int mode, int n, uint32_t* v)
{
    int fam = mode >> 5, b = mode & 31;
    int64_t pos = 0;
    if (fam == 0) {
        for (int i = 0; i < n; i++, pos += b) v[i] = read_bits(words, pos, b);
        return;
    }
    int gsz = fam == 1 ? 5 : 3, hb = fam == 1 ? 8 : 7, radix = fam == 1 ? 3 : 5;
    for (int i0 = 0; i0 < n; i0 += gsz) {
        uint32_t field = read_bits(words, pos, hb);
        pos += hb;
        for (int k = 0; k < gsz; k++, pos += b) {
            uint32_t lo = read_bits(words, pos, b);
            uint32_t hi = field % radix;
            field /= radix;
            if (i0 + k < n) v[i0 + k] = (hi << b) | lo;
        }
    }
}

/* ------------------------------------------------------------------ */
/* Quantisation and block thresholding (Compressing HMLFC tree).       */
/* q = sgn(e) * floor((|e| + floor(step/2)) / step); a block whose     */
/* dequantised energy sum |q*step| is below the threshold is zeroed.   */
/* ------------------------------------------------------------------ */

static int quant(int e, int step)
{
    int m = (iabs(e) + step / 2) / step;
    return e < 0 ? -m : m;
}

static void code_block(const int32_t* e, int n, int step, int thr, int32_t* q)
{
    int64_t energy = 0;
    for (int i = 0; i < n; i++) {
        q[i] = quant(e[i], step);
        energy += (int64_t)iabs(q[i]) * step;
    }
    if (energy < thr)
        for (int i = 0; i < n; i++) q[i] = 0;
}

/* ------------------------------------------------------------------ */
/* Encoder                                                             */
/* ------------------------------------------------------------------ */

typedef struct {
    int mx, my, sigma;
} mvrec;

static void put32(uint8_t* p, uint32_t v) { memcpy(p, &v, 4); }
static void put64(uint8_t* p, uint64_t v) { memcpy(p, &v, 8); }
static uint32_t get32(const uint8_t* p) { uint32_t v; memcpy(&v, p, 4); return v; }
static uint64_t get64(const uint8_t* p) { uint64_t v; memcpy(&v, p, 8); return v; }

void orc_free(void* p) { free(p); }

/* Channel geometry: luma at full resolution; with 4:2:0 chroma (Compressing
 * HMLFC tree: the chroma channels are sub-sampled) Co and Cg are coded at
 * half the width and height. */
static void channel_dims(int w, int h, int chroma420, int c, int* wc, int* hc)
{
    *wc = (chroma420 && c > 0) ? w / 2 : w;
    *hc = (chroma420 && c > 0) ? h / 2 : h;
}

/* 2x2 rounded mean of a full-resolution chroma plane: the half-resolution
 * sample (Y, X) covers full-resolution rows 2Y, 2Y+1 and columns 2X, 2X+1;
 * floor((sum + 2) / 4), the RKV rule for four members. */
void orc_chroma_down(const int32_t* full, int w, int h, int32_t* half)
{
    for (int Y = 0; Y < h / 2; Y++)
        for (int X = 0; X < w / 2; X++) {
            int sum = full[(int64_t)(2 * Y) * w + 2 * X] + full[(int64_t)(2 * Y) * w + 2 * X + 1] +
                      full[(int64_t)(2 * Y + 1) * w + 2 * X] + full[(int64_t)(2 * Y + 1) * w + 2 * X + 1];
            half[(int64_t)Y * (w / 2) + X] = orc_fdiv(sum + 2, 4);
        }
}

/* Per-channel coding state of one encode. */
typedef struct {
    int w, h, nbx, nblk, n;
    int64_t plane;
    int32_t* I[ORC_MAX_LEVELS + 1]; /* original planes per level [views][h][w] */
    int32_t* q;                     /* quantised values [n_nodes][nblk][n] */
    mvrec* mvs[ORC_MAX_LEVELS];
    int64_t npred[ORC_MAX_LEVELS];
} chan_state;

/* The tree of one channel (RLFC hierarchy, then the top-down closed loop
 * with phase-shifted motion compensation), given its level-0 planes. */
static int code_channel(chan_state* S, const orc_params* p, const int* na_l, const int* nb_l,
                        const int64_t* node_base, int64_t n_nodes)
{
    const int H = p->levels, bs = p->block, w = S->w, h = S->h, nbx = S->nbx, nblk = S->nblk, n = S->n;
    const int64_t plane = S->plane;
    /* representative key views: rounded mean over each 2x2 cluster */
    for (int l = 0; l < H; l++) {
        S->I[l + 1] = (int32_t*)malloc(sizeof(int32_t) * na_l[l + 1] * nb_l[l + 1] * plane);
#pragma omp parallel for collapse(2) schedule(static)
        for (int B = 0; B < nb_l[l + 1]; B++)
            for (int A = 0; A < na_l[l + 1]; A++) {
                int32_t* dst = S->I[l + 1] + ((int64_t)B * na_l[l + 1] + A) * plane;
                for (int64_t px = 0; px < plane; px++) {
                    int sum = 0, cnt = 0;
                    for (int j = 0; j < 2; j++)
                        for (int i = 0; i < 2; i++) {
                            int bb = 2 * B + j, aa = 2 * A + i;
                            if (bb >= nb_l[l] || aa >= na_l[l]) continue;
                            sum += S->I[l][((int64_t)bb * na_l[l] + aa) * plane + px];
                            cnt++;
                        }
                    dst[px] = orc_fdiv(sum + cnt / 2, cnt);
                }
            }
    }
    S->q = (int32_t*)calloc((size_t)n_nodes * nblk * n, sizeof(int32_t));
    for (int l = 0; l < H; l++) {
        S->npred[l] = orc_pred_nodes(na_l[l], nb_l[l]) * nblk;
        S->mvs[l] = (mvrec*)calloc((size_t)(S->npred[l] > 0 ? S->npred[l] : 1), sizeof(mvrec));
    }
    /* closed loop from the lossless root */
    int32_t* Irec_up = (int32_t*)malloc(sizeof(int32_t) * na_l[H] * nb_l[H] * plane);
    memcpy(Irec_up, S->I[H], sizeof(int32_t) * na_l[H] * nb_l[H] * plane);
    for (int l = H - 1; l >= 0; l--) {
        const int nal = na_l[l], nbl = nb_l[l], nau = na_l[l + 1], nbu = nb_l[l + 1];
        const int64_t nv = (int64_t)nal * nbl, nvu = (int64_t)nau * nbu;
        int32_t* Sv = (int32_t*)malloc(sizeof(int32_t) * nv * plane);   /* SRVs          */
        int32_t* Shat = (int32_t*)malloc(sizeof(int32_t) * nv * plane); /* decoded SRVs  */
        /* SRV = view - reconstructed parent RKV */
        for (int B = 0; B < nbl; B++)
            for (int A = 0; A < nal; A++) {
                const int32_t* src = S->I[l] + ((int64_t)B * nal + A) * plane;
                const int32_t* par = Irec_up + ((int64_t)(B / 2) * nau + A / 2) * plane;
                int32_t* dst = Sv + ((int64_t)B * nal + A) * plane;
                for (int64_t px = 0; px < plane; px++) dst[px] = src[px] - par[px];
            }
        /* reference SRVs: the (even, even) member of each cluster */
#pragma omp parallel for schedule(dynamic)
        for (int64_t ci = 0; ci < nvu; ci++) {
            int B = 2 * (int)(ci / nau), A = 2 * (int)(ci % nau);
            int64_t vi = (int64_t)B * nal + A;
            int32_t e[4096], q[4096];
            for (int k = 0; k < nblk; k++) {
                int by0 = (k / nbx) * bs, bx0 = (k % nbx) * bs;
                for (int i = 0; i < n; i++) e[i] = Sv[vi * plane + (int64_t)(by0 + i / bs) * w + bx0 + i % bs];
                code_block(e, n, p->step[l], p->t_ref[l], q);
                int64_t node = node_base[l] + vi;
                memcpy(S->q + (node * nblk + k) * n, q, sizeof(int32_t) * n);
                for (int i = 0; i < n; i++)
                    Shat[vi * plane + (int64_t)(by0 + i / bs) * w + bx0 + i % bs] = q[i] * p->step[l];
            }
        }
        /* predictive SRVs: phase-shifted motion compensation against the
         * decoded reference of the same cluster, then the residual is coded */
#pragma omp parallel for schedule(dynamic, 16)
        for (int64_t j = 0; j < S->npred[l]; j++) {
            int64_t pord = j / nblk;
            int k = (int)(j % nblk);
            /* invert the predictive ordinal by scanning (plain, not fast) */
            int B = -1, A = -1;
            for (int bb = 0; bb < nbl && B < 0; bb++)
                for (int aa = 0; aa < nal; aa++)
                    if (((aa | bb) & 1) && orc_pred_ordinal(nal, bb, aa) == pord) {
                        B = bb;
                        A = aa;
                        break;
                    }
            int64_t vi = (int64_t)B * nal + A;
            int64_t ri = (int64_t)(B & ~1) * nal + (A & ~1);
            const int32_t* P = Sv + vi * plane;
            const int32_t* R = Shat + ri * plane;
            int by0 = (k / nbx) * bs, bx0 = (k % nbx) * bs;
            int mx = 0, my = 0, sg = 0;
            if (!p->no_mc)
                orc_mc_search(P, R, w, h, by0, bx0, bs, p->win[l], p->subpel, p->zero_phase, &mx, &my, &sg);
            S->mvs[l][j].mx = mx;
            S->mvs[l][j].my = my;
            S->mvs[l][j].sigma = sg;
            int32_t e[4096], q[4096], pred[4096];
            for (int i = 0; i < n; i++) {
                int y = by0 + i / bs, x = bx0 + i % bs;
                pred[i] = sg * orc_qpel(R, w, h, y, x, mx, my);
                e[i] = P[(int64_t)y * w + x] - pred[i];
            }
            code_block(e, n, p->step[l], p->t_pred[l], q);
            int64_t node = node_base[l] + vi;
            memcpy(S->q + (node * nblk + k) * n, q, sizeof(int32_t) * n);
            int32_t* dst = Shat + vi * plane;
            for (int i = 0; i < n; i++) dst[(int64_t)(by0 + i / bs) * w + bx0 + i % bs] = pred[i] + q[i] * p->step[l];
        }
        /* reconstruction of this level: parent RKV + decoded SRV */
        int32_t* Irec = (int32_t*)malloc(sizeof(int32_t) * nv * plane);
        for (int B = 0; B < nbl; B++)
            for (int A = 0; A < nal; A++) {
                const int32_t* par = Irec_up + ((int64_t)(B / 2) * nau + A / 2) * plane;
                const int32_t* sh = Shat + ((int64_t)B * nal + A) * plane;
                int32_t* dst = Irec + ((int64_t)B * nal + A) * plane;
                for (int64_t px = 0; px < plane; px++) dst[px] = par[px] + sh[px];
            }
        free(Irec_up);
        Irec_up = Irec;
        free(Sv);
        free(Shat);
    }
    free(Irec_up);
    return 0;
}

int orc_encode(const uint8_t* lf, int nb, int na, int h, int w, const orc_params* p,
               int nthreads, uint8_t** out, size_t* out_len)
{
    (void)nthreads;
    const int H = p->levels, bs = p->block, c420 = p->chroma420 != 0;
    if (H < 1 || H > ORC_MAX_LEVELS || bs < 1 || bs > 64 || w % bs || h % bs || na < 1 || nb < 1) return -1;
    if (c420 && (w % (2 * bs) || h % (2 * bs))) return -1; /* chroma planes must hold whole blocks */
    for (int l = 0; l < H; l++)
        if (p->step[l] < 1 || p->win[l] < 0) return -1;
    int na_l[ORC_MAX_LEVELS + 1], nb_l[ORC_MAX_LEVELS + 1];
    orc_level_grid(na, nb, H, na_l, nb_l);
    const int64_t nv0 = (int64_t)na * nb;
    int64_t node_base[ORC_MAX_LEVELS];
    int64_t n_nodes = 0;
    for (int l = H - 1; l >= 0; l--) {
        node_base[l] = n_nodes;
        n_nodes += (int64_t)na_l[l] * nb_l[l];
    }
    chan_state S[3];
    memset(S, 0, sizeof S);
    for (int c = 0; c < 3; c++) {
        channel_dims(w, h, c420, c, &S[c].w, &S[c].h);
        S[c].nbx = S[c].w / bs;
        S[c].nblk = S[c].nbx * (S[c].h / bs);
        S[c].n = bs * bs;
        S[c].plane = (int64_t)S[c].w * S[c].h;
        S[c].I[0] = (int32_t*)malloc(sizeof(int32_t) * nv0 * S[c].plane);
    }
    /* 1. colour transform (and chroma sub-sampling) */
    const int64_t fplane = (int64_t)w * h;
    int32_t* tmp = c420 ? (int32_t*)malloc(sizeof(int32_t) * fplane * 2) : NULL;
    for (int64_t v = 0; v < nv0; v++) {
        for (int64_t px = 0; px < fplane; px++) {
            const uint8_t* s = lf + (v * fplane + px) * 3;
            int Y, Co, Cg;
            orc_ycocg_fwd(s[0], s[1], s[2], &Y, &Co, &Cg);
            S[0].I[0][v * fplane + px] = Y;
            if (c420) {
                tmp[px] = Co;
                tmp[fplane + px] = Cg;
            } else {
                S[1].I[0][v * fplane + px] = Co;
                S[2].I[0][v * fplane + px] = Cg;
            }
        }
        if (c420) {
            orc_chroma_down(tmp, w, h, S[1].I[0] + v * S[1].plane);
            orc_chroma_down(tmp + fplane, w, h, S[2].I[0] + v * S[2].plane);
        }
    }
    free(tmp);
    /* 2-3. hierarchy and closed-loop coding, channel by channel */
    for (int c = 0; c < 3; c++) code_channel(&S[c], p, na_l, nb_l, node_base, n_nodes);

    /* 4. block payloads (channel, BFS node, block order), table entries */
    int64_t tbase[3], nent = 0;
    for (int c = 0; c < 3; c++) {
        tbase[c] = nent;
        nent += n_nodes * S[c].nblk;
    }
    uint8_t* table = (uint8_t*)calloc((size_t)nent, 8);
    int* modes = (int*)malloc(sizeof(int) * nent);
    int16_t* mins = (int16_t*)malloc(sizeof(int16_t) * nent);
    int64_t* woff = (int64_t*)malloc(sizeof(int64_t) * nent);
    int64_t pw = 0;
    int status = 0;
    for (int c = 0; c < 3; c++)
        for (int64_t e0 = 0; e0 < n_nodes * S[c].nblk; e0++) {
            const int n = S[c].n;
            const int64_t e = tbase[c] + e0;
            const int32_t* q = S[c].q + e0 * n;
            int32_t qmin = q[0], nz = 0;
            for (int i = 0; i < n; i++) {
                if (q[i] < qmin) qmin = q[i];
                if (q[i]) nz = 1;
            }
            if (!nz) {
                modes[e] = ORC_INSIGNIFICANT;
                mins[e] = 0;
                woff[e] = 0;
                continue;
            }
            if (qmin < -32768 || qmin > 32767) status = -2;
            uint32_t v[4096];
            for (int i = 0; i < n; i++) v[i] = (uint32_t)(q[i] - qmin);
            int mode = orc_bise_choose(v, n);
            if (mode < 0) status = -2;
            modes[e] = mode;
            mins[e] = (int16_t)qmin;
            woff[e] = pw;
            pw += (orc_bise_bits(mode, n) + 31) / 32;
        }
    if (pw > 0xFFFFFFFFll) status = -2;
    int64_t payload_words = pw + 2; /* >= 8 bytes of trailing slack */
    uint32_t* payload = (uint32_t*)calloc((size_t)payload_words, 4);
    for (int c = 0; c < 3 && status == 0; c++)
        for (int64_t e0 = 0; e0 < n_nodes * S[c].nblk; e0++) {
            const int n = S[c].n;
            const int64_t e = tbase[c] + e0;
            if (modes[e] == ORC_INSIGNIFICANT) continue;
            const int32_t* q = S[c].q + e0 * n;
            uint32_t v[4096];
            for (int i = 0; i < n; i++) v[i] = (uint32_t)(q[i] - mins[e]);
            orc_bise_pack(v, n, modes[e], payload + woff[e]);
            put32(table + e * 8, (uint32_t)woff[e]);
            memcpy(table + e * 8 + 4, &mins[e], 2);
            table[e * 8 + 6] = (uint8_t)modes[e];
        }
    for (int64_t e = 0; e < nent; e++)
        if (modes[e] == ORC_INSIGNIFICANT) table[e * 8 + 6] = ORC_INSIGNIFICANT;

    /* 5. motion vectors: per (channel, level) a BISE sequence of
     *    (mx + 4W, my + 4W) pairs, then 2-bit phase codes (0: +1, 1: -1, 2: none) */
    uint32_t mv_word[3][ORC_MAX_LEVELS] = {{0}}, sig_word[3][ORC_MAX_LEVELS] = {{0}};
    int mv_mode[3][ORC_MAX_LEVELS] = {{0}};
    int64_t mw = 0;
    for (int c = 0; c < 3; c++)
        for (int l = H - 1; l >= 0; l--) {
            const int64_t np = S[c].npred[l];
            mv_mode[c][l] = choose_mode((uint32_t)(8 * p->win[l]), (int)(np > 0 ? 2 * np : 2));
            mv_word[c][l] = (uint32_t)mw;
            mw += (orc_bise_bits(mv_mode[c][l], (int)(2 * np)) + 31) / 32;
            sig_word[c][l] = (uint32_t)mw;
            mw += (2 * np + 31) / 32;
        }
    int64_t mv_words = mw + 2;
    uint32_t* mvsec = (uint32_t*)calloc((size_t)mv_words, 4);
    for (int c = 0; c < 3; c++)
        for (int l = 0; l < H; l++) {
            const int64_t np = S[c].npred[l];
            if (np == 0) continue;
            uint32_t* vals = (uint32_t*)malloc(sizeof(uint32_t) * 2 * np);
            for (int64_t j = 0; j < np; j++) {
                const mvrec* m = &S[c].mvs[l][j];
                int mxv = m->mx + 4 * p->win[l], myv = m->my + 4 * p->win[l];
                if (mxv < 0 || myv < 0 || mxv > 8 * p->win[l] || myv > 8 * p->win[l]) status = -3;
                vals[2 * j] = (uint32_t)mxv;
                vals[2 * j + 1] = (uint32_t)myv;
                uint32_t code = m->sigma == 1 ? 0u : (m->sigma == -1 ? 1u : 2u);
                write_bits(mvsec + sig_word[c][l], 2 * j, 2, code);
            }
            orc_bise_pack(vals, (int)(2 * np), mv_mode[c][l], mvsec + mv_word[c][l]);
            free(vals);
        }

    /* 6. assemble: header, root, table, payload, mv */
    int64_t root_bytes = 0;
    for (int c = 0; c < 3; c++) root_bytes += (int64_t)na_l[H] * nb_l[H] * S[c].plane * 2;
    int64_t off_root = ORC_HDR_BYTES;
    int64_t off_table = off_root + root_bytes;
    int64_t off_payload = off_table + nent * 8;
    int64_t off_mv = off_payload + payload_words * 4;
    int64_t total_len = off_mv + mv_words * 4;
    uint8_t* s = (uint8_t*)calloc((size_t)total_len, 1);
    memcpy(s, "HMLFCv1", 8);
    put32(s + 8, ORC_HDR_BYTES);
    put32(s + 12, 1);
    int32_t dims[8] = {na, nb, w, h, H, bs, 3, 4};
    memcpy(s + 16, dims, 32);
    for (int l = 0; l < H; l++) {
        put32(s + 48 + 4 * l, (uint32_t)p->step[l]);
        put32(s + 80 + 4 * l, (uint32_t)p->win[l]);
    }
    put64(s + 112, off_root);
    put64(s + 120, root_bytes);
    put64(s + 128, off_table);
    put64(s + 136, nent * 8);
    put64(s + 144, off_payload);
    put64(s + 152, payload_words * 4);
    put64(s + 160, off_mv);
    put64(s + 168, mv_words * 4);
    for (int c = 0; c < 3; c++)
        for (int l = 0; l < H; l++) {
            uint8_t* d = s + 176 + (c * ORC_MAX_LEVELS + l) * 16;
            put32(d, mv_word[c][l]);
            put32(d + 4, sig_word[c][l]);
            put32(d + 8, (uint32_t)S[c].npred[l]);
            d[12] = (uint8_t)mv_mode[c][l];
        }
    put32(s + ORC_HDR_CHROMA, (uint32_t)c420);
    /* root: the level-H representative key views of each channel, stored losslessly */
    int16_t* root = (int16_t*)(s + off_root);
    for (int c = 0; c < 3; c++) {
        const int64_t cnt = (int64_t)na_l[H] * nb_l[H] * S[c].plane;
        for (int64_t i = 0; i < cnt; i++) {
            if (S[c].I[H][i] < -32768 || S[c].I[H][i] > 32767) status = -2;
            *root++ = (int16_t)S[c].I[H][i];
        }
    }
    memcpy(s + off_table, table, (size_t)nent * 8);
    memcpy(s + off_payload, payload, (size_t)payload_words * 4);
    memcpy(s + off_mv, mvsec, (size_t)mv_words * 4);

    for (int c = 0; c < 3; c++) {
        for (int l = 0; l <= H; l++) free(S[c].I[l]);
        for (int l = 0; l < H; l++) free(S[c].mvs[l]);
        free(S[c].q);
    }
    free(table);
    free(modes);
    free(mins);
    free(woff);
    free(payload);
    free(mvsec);
    if (status) {
        free(s);
        return status;
    }
    *out = s;
    *out_len = (size_t)total_len;
    return 0;
}

/* ------------------------------------------------------------------ */
/* Stream reader                                                       */
/* ------------------------------------------------------------------ */

int orc_open(const uint8_t* st, size_t len, orc_lf** out)
{
    if (len < ORC_HDR_BYTES || memcmp(st, "HMLFCv1", 8) != 0) return -3;
    if (get32(st + 8) != ORC_HDR_BYTES || get32(st + 12) != 1) return -3;
    orc_lf* lf = (orc_lf*)calloc(1, sizeof(orc_lf));
    int32_t dims[8];
    memcpy(dims, st + 16, 32);
    lf->base = st;
    lf->len = len;
    lf->na = dims[0];
    lf->nb = dims[1];
    lf->w = dims[2];
    lf->h = dims[3];
    lf->H = dims[4];
    lf->bs = dims[5];
    if (lf->H < 1 || lf->H > ORC_MAX_LEVELS || lf->bs < 1 || lf->bs > 64 || lf->w < 1 || lf->h < 1 || lf->w % lf->bs ||
        lf->h % lf->bs || lf->na < 1 || lf->nb < 1 || dims[6] != 3 || dims[7] != 4) {
        free(lf);
        return -3;
    }
    for (int l = 0; l < lf->H; l++) {
        memcpy(&lf->step[l], st + 48 + 4 * l, 4);
        memcpy(&lf->win[l], st + 80 + 4 * l, 4);
    }
    orc_level_grid(lf->na, lf->nb, lf->H, lf->na_l, lf->nb_l);
    lf->n_nodes = 0;
    for (int l = lf->H - 1; l >= 0; l--) {
        lf->node_base[l] = lf->n_nodes;
        lf->n_nodes += (int64_t)lf->na_l[l] * lf->nb_l[l];
    }
    lf->nbx = lf->w / lf->bs;
    lf->nby = lf->h / lf->bs;
    lf->nblk = lf->nbx * lf->nby;
    lf->chroma420 = (int)get32(st + ORC_HDR_CHROMA);
    if (lf->chroma420 > 1 || (lf->chroma420 && (lf->w % (2 * lf->bs) || lf->h % (2 * lf->bs)))) {
        free(lf);
        return -3;
    }
    int64_t tb_expect = 0, rb_expect = 0;
    for (int c = 0; c < 3; c++) {
        channel_dims(lf->w, lf->h, lf->chroma420, c, &lf->cw[c], &lf->ch[c]);
        lf->cnbx[c] = lf->cw[c] / lf->bs;
        lf->cnblk[c] = lf->cnbx[c] * (lf->ch[c] / lf->bs);
        lf->tbase[c] = tb_expect;
        lf->rbase[c] = rb_expect;
        tb_expect += lf->n_nodes * lf->cnblk[c];
        rb_expect += (int64_t)lf->na_l[lf->H] * lf->nb_l[lf->H] * lf->cw[c] * lf->ch[c];
    }
    uint64_t ro = get64(st + 112), rb = get64(st + 120), to = get64(st + 128), tb = get64(st + 136);
    uint64_t po = get64(st + 144), pb = get64(st + 152), mo = get64(st + 160), mb = get64(st + 168);
    int64_t plane = (int64_t)lf->w * lf->h;
    (void)plane;
    if (rb != (uint64_t)rb_expect * 2 || tb != (uint64_t)tb_expect * 8 || ro + rb > len || to + tb > len || po + pb > len ||
        mo + mb > len || pb < 8 || mb < 8 || (po & 3) || (mo & 3) || (ro & 1)) {
        free(lf);
        return -3;
    }
    lf->root = (const int16_t*)(st + ro);
    lf->table = st + to;
    lf->payload = (const uint32_t*)(st + po);
    lf->payload_words = (int64_t)(pb / 4);
    lf->mv = (const uint32_t*)(st + mo);
    lf->mv_words = (int64_t)(mb / 4);
    int64_t sb = 0;
    for (int c = 0; c < 3; c++)
        for (int l = lf->H - 1; l >= 0; l--) {
            const uint8_t* d = st + 176 + (c * ORC_MAX_LEVELS + l) * 16;
            lf->mv_word[c][l] = get32(d);
            lf->sig_word[c][l] = get32(d + 4);
            lf->mv_count[c][l] = get32(d + 8);
            lf->mv_mode[c][l] = d[12];
            int64_t expect = orc_pred_nodes(lf->na_l[l], lf->nb_l[l]) * lf->cnblk[c];
            if ((int64_t)lf->mv_count[c][l] != expect) {
                free(lf);
                return -3;
            }
            if (expect > 0 && ((lf->mv_mode[c][l] >> 5) > 2 || (lf->mv_mode[c][l] & 31) > 20 ||
                               (int64_t)lf->mv_word[c][l] + (orc_bise_bits(lf->mv_mode[c][l], (int)(2 * expect)) + 31) / 32 >
                                   lf->mv_words ||
                               (int64_t)lf->sig_word[c][l] + (2 * expect + 31) / 32 > lf->mv_words)) {
                free(lf);
                return -3;
            }
            lf->shift_base[c][l] = sb;
            sb += expect;
        }
    lf->n_pred_total = sb;
    /* every block payload must lie inside the payload section */
    for (int64_t e = 0; e < tb_expect; e++) {
        const uint8_t* t = lf->table + e * 8;
        int mode = t[6];
        if (mode == ORC_INSIGNIFICANT) continue;
        if ((mode >> 5) > 2 || (mode & 31) > 20) {
            free(lf);
            return -3;
        }
        int64_t words = (orc_bise_bits(mode, lf->bs * lf->bs) + 31) / 32;
        if ((int64_t)get32(t) + words > lf->payload_words) {
            free(lf);
            return -3;
        }
    }
    *out = lf;
    return 0;
}

void orc_close(orc_lf* lf) { free(lf); }

void orc_info(const orc_lf* lf, int64_t* o)
{
    o[0] = lf->na;
    o[1] = lf->nb;
    o[2] = lf->w;
    o[3] = lf->h;
    o[4] = lf->H;
    o[5] = lf->bs;
    o[6] = lf->n_nodes;
    o[7] = lf->n_pred_total;
    o[8] = lf->na_l[lf->H];
    o[9] = lf->nb_l[lf->H];
    o[10] = lf->chroma420;
}

/* ------------------------------------------------------------------ */
/* Random-access decoding (Decoding Procedure): the value of one SRV   */
/* pixel is fetched from its block's bounded-integer sequence.         */
/* ------------------------------------------------------------------ */

int32_t orc_srv_value(const orc_lf* lf, int c, int l, int B, int A, int y, int x)
{
    int64_t node = lf->node_base[l] + (int64_t)B * lf->na_l[l] + A;
    int blk = (y / lf->bs) * lf->cnbx[c] + x / lf->bs;
    int i = (y % lf->bs) * lf->bs + x % lf->bs;
    const uint8_t* t = lf->table + (lf->tbase[c] + node * lf->cnblk[c] + blk) * 8;
    int mode = t[6];
    if (mode == ORC_INSIGNIFICANT) return 0;
    int16_t mn;
    memcpy(&mn, t + 4, 2);
    uint32_t v = orc_bise_get(lf->payload + get32(t), mode, i);
    return ((int32_t)mn + (int32_t)v) * lf->step[l];
}

void orc_mv_record(const orc_lf* lf, int c, int l, int B, int A, int blk, int* mx, int* my, int* sigma)
{
    int64_t j = orc_pred_ordinal(lf->na_l[l], B, A) * lf->cnblk[c] + blk;
    int mode = lf->mv_mode[c][l];
    *mx = (int)orc_bise_get(lf->mv + lf->mv_word[c][l], mode, (int)(2 * j)) - 4 * lf->win[l];
    *my = (int)orc_bise_get(lf->mv + lf->mv_word[c][l], mode, (int)(2 * j + 1)) - 4 * lf->win[l];
    uint32_t code = read_bits(lf->mv + lf->sig_word[c][l], 2 * j, 2);
    *sigma = code == 0 ? 1 : (code == 1 ? -1 : 0);
}

int32_t orc_root_value(const orc_lf* lf, int c, int b, int a, int y, int x)
{
    int Bh = b >> lf->H, Ah = a >> lf->H;
    int64_t idx = lf->rbase[c] + ((int64_t)Bh * lf->na_l[lf->H] + Ah) * lf->cw[c] * lf->ch[c] +
                  (int64_t)y * lf->cw[c] + x;
    return lf->root[idx];
}

/* Reference-plane value with clamped coordinates, for re-compensation. */
static int32_t ref_tap(const orc_lf* lf, int c, int l, int Br, int Ar, int y, int x)
{
    y = orc_clampi(y, 0, lf->ch[c] - 1);
    x = orc_clampi(x, 0, lf->cw[c] - 1);
    return orc_srv_value(lf, c, l, Br, Ar, y, x);
}

static int32_t qpel_stream(const orc_lf* lf, int c, int l, int Br, int Ar, int y, int x, int mx, int my)
{
    int X = 4 * x + mx, Y = 4 * y + my;
    int x0 = orc_asr(X, 2), y0 = orc_asr(Y, 2);
    int fx = X - 4 * x0, fy = Y - 4 * y0;
    int32_t acc = (4 - fx) * (4 - fy) * ref_tap(lf, c, l, Br, Ar, y0, x0)
                + fx * (4 - fy) * ref_tap(lf, c, l, Br, Ar, y0, x0 + 1)
                + (4 - fx) * fy * ref_tap(lf, c, l, Br, Ar, y0 + 1, x0)
                + fx * fy * ref_tap(lf, c, l, Br, Ar, y0 + 1, x0 + 1);
    return orc_asr(acc + 8, 4);
}

/* One channel of one sample: root RKV plus the decoded SRVs of the levels
 * lod .. H-1 on the path from the leaf view (b, a) to the root (Decoding
 * Procedure).  lod = 0 gives the leaf view itself; lod = l > 0 stops the
 * walk at the level-l ancestor (B, A) = (b >> l, a >> l) and gives that
 * node's reconstructed RKV, the progressive decode of the hierarchy. */
static int32_t decode_channel_lod(const orc_lf* lf, int c, int b, int a, int y, int x, int lod)
{
    int32_t v = orc_root_value(lf, c, b, a, y, x);
    for (int l = lod; l < lf->H; l++) {
        int B = b >> l, A = a >> l;
        int32_t r = orc_srv_value(lf, c, l, B, A, y, x);
        if ((A | B) & 1) {
            int mx, my, sg;
            int blk = (y / lf->bs) * lf->cnbx[c] + x / lf->bs;
            orc_mv_record(lf, c, l, B, A, blk, &mx, &my, &sg);
            if (sg) r += sg * qpel_stream(lf, c, l, B & ~1, A & ~1, y, x, mx, my);
        }
        v += r;
    }
    return v;
}

/* Channel c of full-resolution sample (y, x): luma, and chroma of a 4:4:4
 * stream, directly; 4:2:0 chroma by the centred bilinear up-sampling of the
 * four half-resolution samples around it (weights 9, 3, 3, 1 / 16). */
static int32_t sample_channel(const orc_lf* lf, int c, int b, int a, int y, int x, int lod)
{
    if (c == 0 || !lf->chroma420) return decode_channel_lod(lf, c, b, a, y, x, lod);
    const int hy = y >> 1, hx = x >> 1;
    const int ry[2] = {(y & 1) ? hy : hy - 1, (y & 1) ? hy + 1 : hy};
    const int rx[2] = {(x & 1) ? hx : hx - 1, (x & 1) ? hx + 1 : hx};
    const int wy[2] = {(y & 1) ? 3 : 1, (y & 1) ? 1 : 3};
    const int wx[2] = {(x & 1) ? 3 : 1, (x & 1) ? 1 : 3};
    int32_t acc = 0;
    for (int j = 0; j < 2; j++)
        for (int i = 0; i < 2; i++) {
            const int yy = orc_clampi(ry[j], 0, lf->ch[c] - 1), xx = orc_clampi(rx[i], 0, lf->cw[c] - 1);
            acc += wy[j] * wx[i] * decode_channel_lod(lf, c, b, a, yy, xx, lod);
        }
    return orc_asr(acc + 8, 4);
}

static int32_t decode_channel(const orc_lf* lf, int c, int b, int a, int y, int x)
{
    return sample_channel(lf, c, b, a, y, x, 0);
}

void orc_chroma_up(const int32_t* half, int w, int h, int32_t* full)
{
    const int hw = w / 2, hh = h / 2;
    for (int y = 0; y < h; y++)
        for (int x = 0; x < w; x++) {
            const int hy = y >> 1, hx = x >> 1;
            const int ry[2] = {(y & 1) ? hy : hy - 1, (y & 1) ? hy + 1 : hy};
            const int rx[2] = {(x & 1) ? hx : hx - 1, (x & 1) ? hx + 1 : hx};
            const int wy[2] = {(y & 1) ? 3 : 1, (y & 1) ? 1 : 3};
            const int wx[2] = {(x & 1) ? 3 : 1, (x & 1) ? 1 : 3};
            int32_t acc = 0;
            for (int j = 0; j < 2; j++)
                for (int i = 0; i < 2; i++)
                    acc += wy[j] * wx[i] *
                           half[(int64_t)orc_clampi(ry[j], 0, hh - 1) * hw + orc_clampi(rx[i], 0, hw - 1)];
            full[(int64_t)y * w + x] = orc_asr(acc + 8, 4);
        }
}

int orc_decode_channel_at(const orc_lf* lf, int c, int lod, const int32_t* coords, int64_t n, int32_t* out)
{
    if (c < 0 || c > 2 || lod < 0 || lod > lf->H) return -1;
    for (int64_t k = 0; k < n; k++) {
        const int32_t* q = coords + 4 * k;
        if (q[0] < 0 || q[0] >= lf->nb || q[1] < 0 || q[1] >= lf->na || q[2] < 0 || q[2] >= lf->ch[c] || q[3] < 0 ||
            q[3] >= lf->cw[c])
            return -1;
        out[k] = decode_channel_lod(lf, c, q[0], q[1], q[2], q[3], lod);
    }
    return 0;
}

/* Node images at level `level` (0 .. H): coords[k] = (B, A, y, x) with B, A
 * node indices of that level; RGB of the node's reconstructed RKV. */
int orc_decode_node(const orc_lf* lf, int level, const int32_t* coords, int64_t n, uint8_t* rgb)
{
    if (level < 0 || level > lf->H) return -1;
    int status = 0;
    for (int64_t k = 0; k < n; k++) {
        const int32_t* q = coords + 4 * k;
        const int b = q[0] << level, a = q[1] << level;
        if (q[0] < 0 || q[1] < 0 || b >= lf->nb || a >= lf->na || q[2] < 0 || q[2] >= lf->h || q[3] < 0 ||
            q[3] >= lf->w) {
            status = -1;
            continue;
        }
        int ch[3];
        for (int c = 0; c < 3; c++) ch[c] = sample_channel(lf, c, b, a, q[2], q[3], level);
        int r, g, bl;
        orc_ycocg_inv(ch[0], ch[1], ch[2], &r, &g, &bl);
        rgb[3 * k] = (uint8_t)(r < 0 ? 0 : (r > 255 ? 255 : r));
        rgb[3 * k + 1] = (uint8_t)(g < 0 ? 0 : (g > 255 ? 255 : g));
        rgb[3 * k + 2] = (uint8_t)(bl < 0 ? 0 : (bl > 255 ? 255 : bl));
    }
    return status;
}

static int valid_coord(const orc_lf* lf, const int32_t* q)
{
    return q[0] >= 0 && q[0] < lf->nb && q[1] >= 0 && q[1] < lf->na && q[2] >= 0 && q[2] < lf->h && q[3] >= 0 &&
           q[3] < lf->w;
}

int orc_decode_at_ycocg(const orc_lf* lf, const int32_t* coords, int64_t n, int32_t* ycc)
{
    for (int64_t k = 0; k < n; k++) {
        const int32_t* q = coords + 4 * k;
        if (!valid_coord(lf, q)) return -1;
        for (int c = 0; c < 3; c++) ycc[3 * k + c] = decode_channel(lf, c, q[0], q[1], q[2], q[3]);
    }
    return 0;
}

static uint8_t clamp8(int v) { return (uint8_t)(v < 0 ? 0 : (v > 255 ? 255 : v)); }

int orc_decode_at(const orc_lf* lf, const int32_t* coords, int64_t n, uint8_t* rgb)
{
    int status = 0;
#pragma omp parallel for schedule(static)
    for (int64_t k = 0; k < n; k++) {
        const int32_t* q = coords + 4 * k;
        if (!valid_coord(lf, q)) {
            status = -1;
            continue;
        }
        int Y = decode_channel(lf, 0, q[0], q[1], q[2], q[3]);
        int Co = decode_channel(lf, 1, q[0], q[1], q[2], q[3]);
        int Cg = decode_channel(lf, 2, q[0], q[1], q[2], q[3]);
        int r, g, b;
        orc_ycocg_inv(Y, Co, Cg, &r, &g, &b);
        rgb[3 * k] = clamp8(r);
        rgb[3 * k + 1] = clamp8(g);
        rgb[3 * k + 2] = clamp8(b);
    }
    return status;
}

/* ------------------------------------------------------------------ */
/* Full-tree decoding: every block of every SRV is unpacked            */
/* sequentially, predictive blocks are re-compensated from the decoded */
/* reference planes, and each view is the root plus the path sum.      */
/* ------------------------------------------------------------------ */

/* Decoded SRV planes of every node, channel by channel at the channel's
 * resolution: channel c starts at sum over c' < c of n_nodes * w_c' * h_c'
 * (for a 4:4:4 stream, [3][n_nodes][h][w]). */
static int64_t srv_base(const orc_lf* lf, int c)
{
    int64_t b = 0;
    for (int k = 0; k < c; k++) b += lf->n_nodes * (int64_t)lf->cw[k] * lf->ch[k];
    return b;
}

int orc_decode_srv(const orc_lf* lf, int32_t* out)
{
    const int bs = lf->bs, n = bs * bs;
    uint32_t v[4096];
    /* pass 1: dequantised residual planes of every node */
    for (int c = 0; c < 3; c++) {
        const int w = lf->cw[c];
        const int64_t plane = (int64_t)w * lf->ch[c];
        for (int64_t node = 0; node < lf->n_nodes; node++) {
            int32_t* dst = out + srv_base(lf, c) + node * plane;
            int l = 0;
            while (l + 1 < lf->H && node < lf->node_base[l]) l++;
            for (int k = 0; k < lf->cnblk[c]; k++) {
                const uint8_t* t = lf->table + (lf->tbase[c] + node * lf->cnblk[c] + k) * 8;
                int mode = t[6];
                int16_t mn;
                memcpy(&mn, t + 4, 2);
                if (mode != ORC_INSIGNIFICANT) orc_bise_unpack(lf->payload + get32(t), mode, n, v);
                int by0 = (k / lf->cnbx[c]) * bs, bx0 = (k % lf->cnbx[c]) * bs;
                for (int i = 0; i < n; i++)
                    dst[(int64_t)(by0 + i / bs) * w + bx0 + i % bs] =
                        mode == ORC_INSIGNIFICANT ? 0 : ((int32_t)mn + (int32_t)v[i]) * lf->step[l];
            }
        }
    }
    /* pass 2: add the phase-signed prediction to predictive blocks */
    for (int c = 0; c < 3; c++) {
        const int w = lf->cw[c], h = lf->ch[c];
        const int64_t plane = (int64_t)w * h;
        for (int l = 0; l < lf->H; l++)
            for (int B = 0; B < lf->nb_l[l]; B++)
                for (int A = 0; A < lf->na_l[l]; A++) {
                    if (!((A | B) & 1)) continue;
                    int64_t node = lf->node_base[l] + (int64_t)B * lf->na_l[l] + A;
                    int64_t rnode = lf->node_base[l] + (int64_t)(B & ~1) * lf->na_l[l] + (A & ~1);
                    int32_t* dst = out + srv_base(lf, c) + node * plane;
                    const int32_t* ref = out + srv_base(lf, c) + rnode * plane;
                    for (int k = 0; k < lf->cnblk[c]; k++) {
                        int mx, my, sg;
                        orc_mv_record(lf, c, l, B, A, k, &mx, &my, &sg);
                        if (!sg) continue;
                        int by0 = (k / lf->cnbx[c]) * bs, bx0 = (k % lf->cnbx[c]) * bs;
                        for (int y = by0; y < by0 + bs; y++)
                            for (int x = bx0; x < bx0 + bs; x++)
                                dst[(int64_t)y * w + x] += sg * orc_qpel(ref, w, h, y, x, mx, my);
                    }
                }
    }
    return 0;
}

/* Full decode, [3][nb][na][h][w] at full resolution: each channel's views
 * at its own resolution (root + path sum of the SRV planes), 4:2:0 chroma
 * then up-sampled. */
int orc_decode_full_ycocg(const orc_lf* lf, int32_t* out)
{
    const int64_t fplane = (int64_t)lf->w * lf->h;
    int32_t* srv = (int32_t*)malloc(sizeof(int32_t) * srv_base(lf, 3));
    int32_t* view = (int32_t*)malloc(sizeof(int32_t) * fplane);
    if (!srv || !view) {
        free(srv);
        free(view);
        return -2;
    }
    orc_decode_srv(lf, srv);
    for (int c = 0; c < 3; c++) {
        const int w = lf->cw[c];
        const int64_t plane = (int64_t)w * lf->ch[c];
        for (int b = 0; b < lf->nb; b++)
            for (int a = 0; a < lf->na; a++) {
                int32_t* dst = out + (((int64_t)c * lf->nb + b) * lf->na + a) * fplane;
                int32_t* cv = (plane == fplane) ? dst : view;
                for (int64_t px = 0; px < plane; px++)
                    cv[px] = orc_root_value(lf, c, b, a, (int)(px / w), (int)(px % w));
                for (int l = 0; l < lf->H; l++) {
                    int64_t node = lf->node_base[l] + (int64_t)(b >> l) * lf->na_l[l] + (a >> l);
                    const int32_t* sv = srv + srv_base(lf, c) + node * plane;
                    for (int64_t px = 0; px < plane; px++) cv[px] += sv[px];
                }
                if (cv != dst) orc_chroma_up(cv, lf->w, lf->h, dst);
            }
    }
    free(view);
    free(srv);
    return 0;
}

int orc_decode_full(const orc_lf* lf, uint8_t* out)
{
    const int64_t plane = (int64_t)lf->w * lf->h, nv = (int64_t)lf->na * lf->nb;
    int32_t* ycc = (int32_t*)malloc(sizeof(int32_t) * 3 * nv * plane);
    if (!ycc) return -2;
    orc_decode_full_ycocg(lf, ycc);
    for (int64_t v = 0; v < nv; v++)
        for (int64_t px = 0; px < plane; px++) {
            int r, g, b;
            orc_ycocg_inv(ycc[(0 * nv + v) * plane + px], ycc[(1 * nv + v) * plane + px],
                          ycc[(2 * nv + v) * plane + px], &r, &g, &b);
            uint8_t* d = out + (v * plane + px) * 3;
            d[0] = clamp8(r);
            d[1] = clamp8(g);
            d[2] = clamp8(b);
        }
    free(ycc);
    return 0;
}
