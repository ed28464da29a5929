/*
 * HMLFC CPU oracle: two-plane light-field rendering, per-view footprint
 * accounting and the relaxed (real-valued) model with its derivatives.
 * TEST INFRASTRUCTURE ONLY.
 *
 * Rendering (Prior Work / Light Field Rendering; the paper's renderer is a
 * ray-based interpolation of captured rays): output pixel (i, j) of a camera
 * is sent through two homographies at its centre, giving (u, v) on the view
 * grid and (s, t) on the image plane.  Each coordinate is clamped to the
 * grid, and the 16 neighbouring samples are blended quadrilinearly: in s,
 * then t within each view, then u, then v.  Ray coordinates are evaluated in
 * binary32 with every product and sum rounded separately; the blend is
 * binary64.
 */
#include <math.h>
#include <omp.h>
#include <stdlib.h>
#include <string.h>

#include "internal.h"

/* ------------------------------------------------------------------ */
/* ray coordinates                                                     */
/* ------------------------------------------------------------------ */

static float apply_h(const float* hm, float px, float py, int row)
{
    volatile float a = hm[3 * row + 0] * px;
    volatile float b = hm[3 * row + 1] * py;
    volatile float s = a + b;
    return s + hm[3 * row + 2];
}

int orc_ray_coords(const float* cam, int wo, int ho, int i, int j, float* uvst)
{
    (void)wo;
    (void)ho;
    float px = (float)i + 0.5f, py = (float)j + 0.5f;
    const float* huv = cam;
    const float* hst = cam + 9;
    float xu = apply_h(huv, px, py, 0), yu = apply_h(huv, px, py, 1), wu = apply_h(huv, px, py, 2);
    float xs = apply_h(hst, px, py, 0), ys = apply_h(hst, px, py, 1), ws = apply_h(hst, px, py, 2);
    uvst[0] = xu / wu;
    uvst[1] = yu / wu;
    uvst[2] = xs / ws;
    uvst[3] = ys / ws;
    return 0;
}

/* clamp to [0, n-1], lower neighbour, upper neighbour and fraction */
static void axis(float c, int n, int* i0, int* i1, float* f)
{
    float hi = (float)(n - 1);
    c = fminf(fmaxf(c, 0.0f), hi);
    int k = (int)floorf(c);
    if (k > n - 2) k = n - 2;
    if (k < 0) k = 0;
    *i0 = k;
    *i1 = k + 1 < n ? k + 1 : n - 1;
    *f = c - (float)k;
}

typedef struct {
    int b[2], a[2], y[2], x[2];
    float fv, fu, ft, fs;
} footprint;

static void ray_footprint(const float* cam, int wo, int ho, int i, int j, int na, int nb, int w, int h,
                          footprint* fp)
{
    float q[4];
    orc_ray_coords(cam, wo, ho, i, j, q);
    axis(q[0], na, &fp->a[0], &fp->a[1], &fp->fu);
    axis(q[1], nb, &fp->b[0], &fp->b[1], &fp->fv);
    axis(q[2], w, &fp->x[0], &fp->x[1], &fp->fs);
    axis(q[3], h, &fp->y[0], &fp->y[1], &fp->ft);
}

static double lerp(double p, double q, double f) { return p + f * (q - p); }

/* blend of 16 samples s[jb][ia][jy][ix] */
static double blend16(const double s[2][2][2][2], const footprint* fp)
{
    double view[2][2];
    for (int jb = 0; jb < 2; jb++)
        for (int ia = 0; ia < 2; ia++) {
            double top = lerp(s[jb][ia][0][0], s[jb][ia][0][1], fp->fs);
            double bot = lerp(s[jb][ia][1][0], s[jb][ia][1][1], fp->fs);
            view[jb][ia] = lerp(top, bot, fp->ft);
        }
    double r0 = lerp(view[0][0], view[0][1], fp->fu);
    double r1 = lerp(view[1][0], view[1][1], fp->fu);
    return lerp(r0, r1, fp->fv);
}

/* Threads of every OpenMP loop that follows (n <= 0: one per processor);
 * returns the count now in effect.  For timing the oracle on n cores. */
int orc_set_threads(int n)
{
    omp_set_num_threads(n > 0 ? n : omp_get_num_procs());
    return omp_get_max_threads();
}

int orc_render(const orc_lf* lf, const float* cams, int nv, int wo, int ho, int nthreads, double* out)
{
    (void)nthreads;
    int status = 0;
    const int64_t npix = (int64_t)wo * ho;
#pragma omp parallel for schedule(dynamic, 64)
    for (int64_t r = 0; r < (int64_t)nv * npix; r++) {
        int v = (int)(r / npix);
        int j = (int)((r % npix) / wo), i = (int)(r % wo);
        footprint fp;
        ray_footprint(cams + 18 * v, wo, ho, i, j, lf->na, lf->nb, lf->w, lf->h, &fp);
        int32_t coords[16 * 4];
        uint8_t rgb[16 * 3];
        int k = 0;
        for (int jb = 0; jb < 2; jb++)
            for (int ia = 0; ia < 2; ia++)
                for (int jy = 0; jy < 2; jy++)
                    for (int ix = 0; ix < 2; ix++, k++) {
                        coords[4 * k] = fp.b[jb];
                        coords[4 * k + 1] = fp.a[ia];
                        coords[4 * k + 2] = fp.y[jy];
                        coords[4 * k + 3] = fp.x[ix];
                    }
        if (orc_decode_at(lf, coords, 16, rgb)) status = -1;
        for (int c = 0; c < 3; c++) {
            double s[2][2][2][2];
            for (k = 0; k < 16; k++) s[k >> 3][(k >> 2) & 1][(k >> 1) & 1][k & 1] = rgb[3 * k + c] / 255.0;
            out[((int64_t)v * 3 + c) * npix + (int64_t)j * wo + i] = blend16(s, &fp);
        }
    }
    return status;
}

/* The same rendering with every sample replaced by its level-lod ancestor's
 * reconstructed RKV: the view (b, a) of a sample reads node (b >> lod,
 * a >> lod) of level lod (progressive decode, lod = 0: orc_render). */
int orc_render_lod(const orc_lf* lf, int lod, const float* cams, int nv, int wo, int ho, double* out)
{
    if (lod < 0 || lod > lf->H) return -1;
    int status = 0;
    const int64_t npix = (int64_t)wo * ho;
#pragma omp parallel for schedule(dynamic, 64)
    for (int64_t r = 0; r < (int64_t)nv * npix; r++) {
        int v = (int)(r / npix);
        int j = (int)((r % npix) / wo), i = (int)(r % wo);
        footprint fp;
        ray_footprint(cams + 18 * v, wo, ho, i, j, lf->na, lf->nb, lf->w, lf->h, &fp);
        int32_t coords[16 * 4];
        uint8_t rgb[16 * 3];
        int k = 0;
        for (int jb = 0; jb < 2; jb++)
            for (int ia = 0; ia < 2; ia++)
                for (int jy = 0; jy < 2; jy++)
                    for (int ix = 0; ix < 2; ix++, k++) {
                        coords[4 * k] = fp.b[jb] >> lod;
                        coords[4 * k + 1] = fp.a[ia] >> lod;
                        coords[4 * k + 2] = fp.y[jy];
                        coords[4 * k + 3] = fp.x[ix];
                    }
        if (orc_decode_node(lf, lod, coords, 16, rgb)) status = -1;
        for (int c = 0; c < 3; c++) {
            double s[2][2][2][2];
            for (k = 0; k < 16; k++) s[k >> 3][(k >> 2) & 1][(k >> 1) & 1][k & 1] = rgb[3 * k + c] / 255.0;
            out[((int64_t)v * 3 + c) * npix + (int64_t)j * wo + i] = blend16(s, &fp);
        }
    }
    return status;
}

/* Selected rays only: rays[k] = (view, i, j); out[k][3]. */
int orc_render_rays(const orc_lf* lf, const float* cams, int wo, int ho, const int32_t* rays, int64_t n,
                    double* out)
{
    int status = 0;
#pragma omp parallel for schedule(dynamic, 16)
    for (int64_t r = 0; r < n; r++) {
        int v = rays[3 * r], i = rays[3 * r + 1], j = rays[3 * r + 2];
        if (i < 0 || i >= wo || j < 0 || j >= ho || v < 0) {
            status = -1;
            continue;
        }
        footprint fp;
        ray_footprint(cams + 18 * v, wo, ho, i, j, lf->na, lf->nb, lf->w, lf->h, &fp);
        int32_t coords[16 * 4];
        uint8_t rgb[16 * 3];
        for (int k = 0; k < 16; k++) {
            coords[4 * k] = fp.b[k >> 3];
            coords[4 * k + 1] = fp.a[(k >> 2) & 1];
            coords[4 * k + 2] = fp.y[(k >> 1) & 1];
            coords[4 * k + 3] = fp.x[k & 1];
        }
        if (orc_decode_at(lf, coords, 16, rgb)) status = -1;
        for (int c = 0; c < 3; c++) {
            double s[2][2][2][2];
            for (int k = 0; k < 16; k++) s[k >> 3][(k >> 2) & 1][(k >> 1) & 1][k & 1] = rgb[3 * k + c] / 255.0;
            out[3 * r + c] = blend16(s, &fp);
        }
    }
    return status;
}

int orc_render_dense(const uint8_t* L, int nb, int na, int h, int w, const float* cams, int nv, int wo, int ho,
                     double* out)
{
    const int64_t npix = (int64_t)wo * ho;
    for (int v = 0; v < nv; v++)
        for (int j = 0; j < ho; j++)
            for (int i = 0; i < wo; i++) {
                footprint fp;
                ray_footprint(cams + 18 * v, wo, ho, i, j, na, nb, w, h, &fp);
                for (int c = 0; c < 3; c++) {
                    double s[2][2][2][2];
                    for (int k = 0; k < 16; k++) {
                        int b = fp.b[k >> 3], a = fp.a[(k >> 2) & 1], y = fp.y[(k >> 1) & 1], x = fp.x[k & 1];
                        s[k >> 3][(k >> 2) & 1][(k >> 1) & 1][k & 1] =
                            L[((((int64_t)b * na + a) * h + y) * w + x) * 3 + c] / 255.0;
                    }
                    out[((int64_t)v * 3 + c) * npix + (int64_t)j * wo + i] = blend16(s, &fp);
                }
            }
    return 0;
}

/* ------------------------------------------------------------------ */
/* Footprint bytes of one view: the output plus every distinct piece   */
/* of compressed or resident data the view's samples need.  Per        */
/* predictive block: its 8-byte table entry, its payload words and its */
/* share of the motion-vector stream.  Per reference-SRV block read    */
/* (directly, or through a non-zero-weight prediction tap) and per     */
/* root block: 2 bytes per pixel.  Reuse across views is not credited. */
/* ------------------------------------------------------------------ */

int orc_footprint_bytes(const orc_lf* lf, const float* cams, int nv, int wo, int ho, double* out)
{
    if (lf->chroma420) return -4; /* full-size chroma planes only */
    const int64_t nent = 3 * lf->n_nodes * lf->nblk;
    const int64_t nroot = (int64_t)3 * lf->na_l[lf->H] * lf->nb_l[lf->H] * lf->nblk;
    uint8_t* pred = (uint8_t*)malloc((size_t)nent);
    uint8_t* ref = (uint8_t*)malloc((size_t)nent);
    uint8_t* root = (uint8_t*)malloc((size_t)nroot);
    double mvbytes[3][ORC_MAX_LEVELS];
    for (int c = 0; c < 3; c++)
        for (int l = 0; l < lf->H; l++) {
            double cnt = (double)lf->mv_count[c][l];
            mvbytes[c][l] = cnt > 0 ? ((double)orc_bise_bits(lf->mv_mode[c][l], (int)(2 * cnt)) + 2.0 * cnt) / (8.0 * cnt)
                                    : 0.0;
        }
    for (int v = 0; v < nv; v++) {
        memset(pred, 0, (size_t)nent);
        memset(ref, 0, (size_t)nent);
        memset(root, 0, (size_t)nroot);
        for (int j = 0; j < ho; j++)
            for (int i = 0; i < wo; i++) {
                footprint fp;
                ray_footprint(cams + 18 * v, wo, ho, i, j, lf->na, lf->nb, lf->w, lf->h, &fp);
                for (int k = 0; k < 16; k++) {
                    int b = fp.b[k >> 3], a = fp.a[(k >> 2) & 1], y = fp.y[(k >> 1) & 1], x = fp.x[k & 1];
                    int blk = (y / lf->bs) * lf->nbx + x / lf->bs;
                    for (int c = 0; c < 3; c++) {
                        int64_t rn = ((int64_t)(b >> lf->H) * lf->na_l[lf->H] + (a >> lf->H));
                        root[((int64_t)c * lf->na_l[lf->H] * lf->nb_l[lf->H] + rn) * lf->nblk + blk] = 1;
                        for (int l = 0; l < lf->H; l++) {
                            int B = b >> l, A = a >> l;
                            int64_t node = lf->node_base[l] + (int64_t)B * lf->na_l[l] + A;
                            if (!((A | B) & 1)) {
                                ref[((int64_t)c * lf->n_nodes + node) * lf->nblk + blk] = 1;
                                continue;
                            }
                            pred[((int64_t)c * lf->n_nodes + node) * lf->nblk + blk] = 1;
                            int mx, my, sg;
                            orc_mv_record(lf, c, l, B, A, blk, &mx, &my, &sg);
                            if (!sg) continue;
                            int64_t rnode = lf->node_base[l] + (int64_t)(B & ~1) * lf->na_l[l] + (A & ~1);
                            int X = 4 * x + mx, Y = 4 * y + my;
                            int x0 = orc_asr(X, 2), y0 = orc_asr(Y, 2), fx = X - 4 * x0, fy = Y - 4 * y0;
                            for (int ty = 0; ty < 2; ty++)
                                for (int tx = 0; tx < 2; tx++) {
                                    int wgt = (tx ? fx : 4 - fx) * (ty ? fy : 4 - fy);
                                    if (!wgt) continue;
                                    int yy = orc_clampi(y0 + ty, 0, lf->h - 1), xx = orc_clampi(x0 + tx, 0, lf->w - 1);
                                    int tb = (yy / lf->bs) * lf->nbx + xx / lf->bs;
                                    ref[((int64_t)c * lf->n_nodes + rnode) * lf->nblk + tb] = 1;
                                }
                        }
                    }
                }
            }
        double bytes = 12.0 * wo * ho;
        for (int c = 0; c < 3; c++)
            for (int64_t node = 0; node < lf->n_nodes; node++) {
                int l = 0;
                while (node < lf->node_base[l]) l++;
                for (int k = 0; k < lf->nblk; k++) {
                    int64_t e = ((int64_t)c * lf->n_nodes + node) * lf->nblk + k;
                    if (ref[e]) bytes += 2.0 * lf->bs * lf->bs;
                    if (pred[e]) {
                        const uint8_t* t = lf->table + e * 8;
                        bytes += 8.0 + mvbytes[c][l];
                        if (t[6] != ORC_INSIGNIFICANT)
                            bytes += 4.0 * (double)((orc_bise_bits(t[6], lf->bs * lf->bs) + 31) / 32);
                    }
                }
            }
        for (int64_t e = 0; e < nroot; e++)
            if (root[e]) bytes += 2.0 * lf->bs * lf->bs;
        out[v] = bytes;
    }
    free(pred);
    free(ref);
    free(root);
    return 0;
}

/* ------------------------------------------------------------------ */
/* Relaxed model.  Parameters: real dequantised residual planes for    */
/* every SRV node ([3][n_nodes][h][w]) and real per-block shifts in    */
/* pixels ([n_pred_total][2] = (dx, dy)).  A reference SRV equals its  */
/* residual; a predictive SRV is sigma * bilinear(reference, shifted)  */
/* plus its residual, with no rounding; the colour inverse is linear   */
/* (R = Y + Co/2 - Cg/2, G = Y + Cg/2, B = Y - Co/2 - Cg/2) and nothing */
/* is clamped.  Derivatives use dual numbers (forward mode) for single */
/* parameters and an explicit transpose for the full adjoint.          */
/* ------------------------------------------------------------------ */

typedef struct {
    double v, d;
} dual;

static dual dc(double v) { dual r = {v, 0.0}; return r; }
static dual dadd(dual a, dual b) { dual r = {a.v + b.v, a.d + b.d}; return r; }
static dual dsub(dual a, dual b) { dual r = {a.v - b.v, a.d - b.d}; return r; }
static dual dmul(dual a, dual b) { dual r = {a.v * b.v, a.v * b.d + a.d * b.v}; return r; }
static dual dscale(dual a, double s) { dual r = {a.v * s, a.d * s}; return r; }
static dual dlerp(dual p, dual q, dual f) { return dadd(p, dmul(f, dsub(q, p))); }

typedef struct {
    const orc_lf* lf;
    const float* res;
    const float* shift;
    int seed_kind;        /* -1 none, 0 residual, 1 shift */
    int64_t seed_index;
    double delta;         /* added to the seeded parameter's value */
} relax_ctx;

static dual res_get(const relax_ctx* x, int c, int64_t node, int y, int X)
{
    const orc_lf* lf = x->lf;
    int64_t idx = (((int64_t)c * lf->n_nodes + node) * lf->h + y) * lf->w + X;
    dual r = dc(x->res[idx]);
    if (x->seed_kind == 0 && x->seed_index == idx) {
        r.v += x->delta;
        r.d = 1.0;
    }
    return r;
}

static dual shift_get(const relax_ctx* x, int64_t rec, int comp)
{
    int64_t idx = 2 * rec + comp;
    dual r = dc(x->shift[idx]);
    if (x->seed_kind == 1 && x->seed_index == idx) {
        r.v += x->delta;
        r.d = 1.0;
    }
    return r;
}

static int sigma_of(const orc_lf* lf, int c, int l, int B, int A, int blk)
{
    int mx, my, sg;
    orc_mv_record(lf, c, l, B, A, blk, &mx, &my, &sg);
    return sg;
}

static dual relaxed_channel(const relax_ctx* x, int c, int b, int a, int y, int X)
{
    const orc_lf* lf = x->lf;
    dual v = dc(orc_root_value(lf, c, b, a, y, X));
    for (int l = 0; l < lf->H; l++) {
        int B = b >> l, A = a >> l;
        int64_t node = lf->node_base[l] + (int64_t)B * lf->na_l[l] + A;
        dual r = res_get(x, c, node, y, X);
        if ((A | B) & 1) {
            int blk = (y / lf->bs) * lf->nbx + X / lf->bs;
            int sg = sigma_of(lf, c, l, B, A, blk);
            if (sg) {
                int64_t rec = lf->shift_base[c][l] + orc_pred_ordinal(lf->na_l[l], B, A) * lf->nblk + blk;
                int64_t rnode = lf->node_base[l] + (int64_t)(B & ~1) * lf->na_l[l] + (A & ~1);
                dual px = dadd(dc(X), shift_get(x, rec, 0));
                dual py = dadd(dc(y), shift_get(x, rec, 1));
                double x0 = floor(px.v), y0 = floor(py.v);
                dual fx = dsub(px, dc(x0)), fy = dsub(py, dc(y0));
                int xa = orc_clampi((int)x0, 0, lf->w - 1), xb = orc_clampi((int)x0 + 1, 0, lf->w - 1);
                int ya = orc_clampi((int)y0, 0, lf->h - 1), yb = orc_clampi((int)y0 + 1, 0, lf->h - 1);
                dual t00 = res_get(x, c, rnode, ya, xa), t01 = res_get(x, c, rnode, ya, xb);
                dual t10 = res_get(x, c, rnode, yb, xa), t11 = res_get(x, c, rnode, yb, xb);
                dual bil = dlerp(dlerp(t00, t01, fx), dlerp(t10, t11, fx), fy);
                r = dadd(r, dscale(bil, (double)sg));
            }
        }
        v = dadd(v, r);
    }
    return v;
}

static void relaxed_rgb(const relax_ctx* x, int b, int a, int y, int X, dual* rgb)
{
    dual Y = relaxed_channel(x, 0, b, a, y, X);
    dual Co = relaxed_channel(x, 1, b, a, y, X);
    dual Cg = relaxed_channel(x, 2, b, a, y, X);
    dual hco = dscale(Co, 0.5), hcg = dscale(Cg, 0.5);
    rgb[0] = dsub(dadd(Y, hco), hcg);
    rgb[1] = dadd(Y, hcg);
    rgb[2] = dsub(dsub(Y, hco), hcg);
}

static void relaxed_ray(const relax_ctx* x, const float* cam, int wo, int ho, int i, int j, dual* out3)
{
    const orc_lf* lf = x->lf;
    footprint fp;
    ray_footprint(cam, wo, ho, i, j, lf->na, lf->nb, lf->w, lf->h, &fp);
    dual s[16][3];
    for (int k = 0; k < 16; k++)
        relaxed_rgb(x, fp.b[k >> 3], fp.a[(k >> 2) & 1], fp.y[(k >> 1) & 1], fp.x[k & 1], s[k]);
    dual fs = dc(fp.fs), ft = dc(fp.ft), fu = dc(fp.fu), fv = dc(fp.fv);
    for (int c = 0; c < 3; c++) {
        dual view[4];
        for (int q = 0; q < 4; q++) {
            dual top = dlerp(dscale(s[4 * q + 0][c], 1.0 / 255.0), dscale(s[4 * q + 1][c], 1.0 / 255.0), fs);
            dual bot = dlerp(dscale(s[4 * q + 2][c], 1.0 / 255.0), dscale(s[4 * q + 3][c], 1.0 / 255.0), fs);
            view[q] = dlerp(top, bot, ft);
        }
        dual r0 = dlerp(view[0], view[1], fu), r1 = dlerp(view[2], view[3], fu);
        out3[c] = dlerp(r0, r1, fv);
    }
}

int orc_export_params(const orc_lf* lf, float* residual, float* shift)
{
    if (lf->chroma420) return -4; /* full-size chroma planes only */
    const int64_t plane = (int64_t)lf->w * lf->h;
    for (int c = 0; c < 3; c++)
        for (int l = 0; l < lf->H; l++)
            for (int B = 0; B < lf->nb_l[l]; B++)
                for (int A = 0; A < lf->na_l[l]; A++) {
                    int64_t node = lf->node_base[l] + (int64_t)B * lf->na_l[l] + A;
                    float* dst = residual + ((int64_t)c * lf->n_nodes + node) * plane;
                    for (int y = 0; y < lf->h; y++)
                        for (int x = 0; x < lf->w; x++)
                            dst[(int64_t)y * lf->w + x] = (float)orc_srv_value(lf, c, l, B, A, y, x);
                    if (!((A | B) & 1)) continue;
                    for (int k = 0; k < lf->nblk; k++) {
                        int mx, my, sg;
                        orc_mv_record(lf, c, l, B, A, k, &mx, &my, &sg);
                        int64_t rec = lf->shift_base[c][l] + orc_pred_ordinal(lf->na_l[l], B, A) * lf->nblk + k;
                        shift[2 * rec] = (float)(mx / 4.0);
                        shift[2 * rec + 1] = (float)(my / 4.0);
                    }
                }
    return 0;
}

int orc_render_relaxed(const orc_lf* lf, const float* residual, const float* shift, const float* cams, int nv,
                       int wo, int ho, int nthreads, double* out)
{
    if (lf->chroma420) return -4; /* full-size chroma planes only */
    (void)nthreads;
    relax_ctx x = {lf, residual, shift, -1, 0, 0.0};
    const int64_t npix = (int64_t)wo * ho;
#pragma omp parallel for schedule(dynamic, 64)
    for (int64_t r = 0; r < (int64_t)nv * npix; r++) {
        int v = (int)(r / npix), j = (int)((r % npix) / wo), i = (int)(r % wo);
        dual o[3];
        relaxed_ray(&x, cams + 18 * v, wo, ho, i, j, o);
        for (int c = 0; c < 3; c++) out[((int64_t)v * 3 + c) * npix + (int64_t)j * wo + i] = o[c].v;
    }
    return 0;
}

double orc_relaxed_loss(const orc_lf* lf, const float* residual, const float* shift, const float* cams, int nv,
                        int wo, int ho, const float* target, int nthreads)
{
    if (lf->chroma420) return NAN; /* full-size chroma planes only */
    (void)nthreads;
    relax_ctx x = {lf, residual, shift, -1, 0, 0.0};
    const int64_t npix = (int64_t)wo * ho;
    double loss = 0.0;
    for (int64_t r = 0; r < (int64_t)nv * npix; r++) {
        int v = (int)(r / npix), j = (int)((r % npix) / wo), i = (int)(r % wo);
        dual o[3];
        relaxed_ray(&x, cams + 18 * v, wo, ho, i, j, o);
        for (int c = 0; c < 3; c++) {
            double d = o[c].v - target[((int64_t)v * 3 + c) * npix + (int64_t)j * wo + i];
            loss += d * d;
        }
    }
    return loss;
}

/* Does LF sample (b, a, y, x) depend on the given parameter? */
static int sample_depends(const orc_lf* lf, int kind, int c, int l, int B, int A, int py, int px, int blk,
                          int b, int a, int y, int x)
{
    int Bs = b >> l, As = a >> l;
    if (kind == 1) return Bs == B && As == A && (y / lf->bs) * lf->nbx + x / lf->bs == blk;
    if (Bs == B && As == A && y == py && x == px) return 1;
    /* a reference residual also feeds the predictive siblings' prediction taps */
    if ((A | B) & 1) return 0;
    if ((Bs & ~1) != B || (As & ~1) != A || !((As | Bs) & 1)) return 0;
    int sblk = (y / lf->bs) * lf->nbx + x / lf->bs;
    if (!sigma_of(lf, c, l, Bs, As, sblk)) return 0;
    return -1; /* needs the shift value: resolved by the caller */
}

int64_t orc_param_check(const orc_lf* lf, const float* residual, const float* shift, const float* cams, int nv,
                        int wo, int ho, const float* target, int kind, int64_t index, double eps, double* fd,
                        double* fwd)
{
    if (lf->chroma420) return -4; /* full-size chroma planes only */
    const int64_t plane = (int64_t)lf->w * lf->h, npix = (int64_t)wo * ho;
    int c, l = 0, B, A, py = 0, px = 0, blk = 0;
    if (kind == 0) {
        c = (int)(index / (lf->n_nodes * plane));
        int64_t node = (index / plane) % lf->n_nodes;
        while (node < lf->node_base[l]) l++;
        int64_t local = node - lf->node_base[l];
        B = (int)(local / lf->na_l[l]);
        A = (int)(local % lf->na_l[l]);
        py = (int)((index % plane) / lf->w);
        px = (int)(index % lf->w);
    } else {
        int64_t rec = index / 2;
        c = 0;
        while (c < 2 && rec >= lf->shift_base[c + 1][lf->H - 1]) c++;
        l = lf->H - 1;
        while (l > 0 && rec >= lf->shift_base[c][l - 1]) l--;
        int64_t j = rec - lf->shift_base[c][l];
        int64_t pord = j / lf->nblk;
        blk = (int)(j % lf->nblk);
        B = A = -1;
        for (int bb = 0; bb < lf->nb_l[l] && B < 0; bb++)
            for (int aa = 0; aa < lf->na_l[l]; aa++)
                if (((aa | bb) & 1) && orc_pred_ordinal(lf->na_l[l], bb, aa) == pord) {
                    B = bb;
                    A = aa;
                    break;
                }
    }
    relax_ctx plus = {lf, residual, shift, kind, index, eps};
    relax_ctx minus = {lf, residual, shift, kind, index, -eps};
    relax_ctx base = {lf, residual, shift, kind, index, 0.0};
    double sum_fd = 0.0, sum_fwd = 0.0;
    int64_t hits = 0;
    for (int v = 0; v < nv; v++)
        for (int j = 0; j < ho; j++)
            for (int i = 0; i < wo; i++) {
                footprint fp;
                ray_footprint(cams + 18 * v, wo, ho, i, j, lf->na, lf->nb, lf->w, lf->h, &fp);
                int hit = 0;
                for (int k = 0; k < 16 && !hit; k++) {
                    int b = fp.b[k >> 3], a = fp.a[(k >> 2) & 1], y = fp.y[(k >> 1) & 1], x = fp.x[k & 1];
                    int dep = sample_depends(lf, kind, c, l, B, A, py, px, blk, b, a, y, x);
                    if (dep == -1) {
                        /* predictive sibling: does any tap (at +-eps shift values too) touch (py, px)? */
                        int Bs = b >> l, As = a >> l;
                        int sblk = (y / lf->bs) * lf->nbx + x / lf->bs;
                        int64_t rec = lf->shift_base[c][l] + orc_pred_ordinal(lf->na_l[l], Bs, As) * lf->nblk + sblk;
                        double X = x + shift[2 * rec], Y = y + shift[2 * rec + 1];
                        int x0 = (int)floor(X), y0 = (int)floor(Y);
                        int xa = orc_clampi(x0, 0, lf->w - 1), xb = orc_clampi(x0 + 1, 0, lf->w - 1);
                        int ya = orc_clampi(y0, 0, lf->h - 1), yb = orc_clampi(y0 + 1, 0, lf->h - 1);
                        dep = (ya == py || yb == py) && (xa == px || xb == px);
                    }
                    hit = dep != 0;
                }
                if (!hit) continue;
                hits++;
                dual op[3], om[3], ob[3];
                relaxed_ray(&plus, cams + 18 * v, wo, ho, i, j, op);
                relaxed_ray(&minus, cams + 18 * v, wo, ho, i, j, om);
                relaxed_ray(&base, cams + 18 * v, wo, ho, i, j, ob);
                for (int cc = 0; cc < 3; cc++) {
                    double t = target[((int64_t)v * 3 + cc) * npix + (int64_t)j * wo + i];
                    double dp = op[cc].v - t, dm = om[cc].v - t, db = ob[cc].v - t;
                    sum_fd += dp * dp - dm * dm;
                    sum_fwd += 2.0 * db * ob[cc].d;
                }
            }
    *fd = sum_fd / (2.0 * eps);
    *fwd = sum_fwd;
    return hits;
}

/* Full reverse-mode adjoint, written as explicit transposes of each step:
 * blend weights -> sample gradient, colour transpose, sum over each node's
 * descendants, then the bilinear transpose into the reference residual and
 * the per-block shift derivatives. */
int orc_relaxed_grad(const orc_lf* lf, const float* residual, const float* shift, const float* cams, int nv, int wo,
                     int ho, const double* grad_out, double* g_res, double* g_shift)
{
    if (lf->chroma420) return -4; /* full-size chroma planes only */
    const int64_t plane = (int64_t)lf->w * lf->h, npix = (int64_t)wo * ho;
    const int64_t nviews = (int64_t)lf->na * lf->nb;
    double* gs = (double*)calloc((size_t)(nviews * plane * 3), sizeof(double)); /* [b][a][y][x][rgb] */
    if (!gs) return -2;
    for (int v = 0; v < nv; v++)
        for (int j = 0; j < ho; j++)
            for (int i = 0; i < wo; i++) {
                footprint fp;
                ray_footprint(cams + 18 * v, wo, ho, i, j, lf->na, lf->nb, lf->w, lf->h, &fp);
                for (int k = 0; k < 16; k++) {
                    int jb = k >> 3, ia = (k >> 2) & 1, jy = (k >> 1) & 1, ix = k & 1;
                    double wgt = (jb ? fp.fv : 1.0 - fp.fv) * (ia ? fp.fu : 1.0 - fp.fu) *
                                 (jy ? fp.ft : 1.0 - fp.ft) * (ix ? fp.fs : 1.0 - fp.fs) / 255.0;
                    int64_t s = (((int64_t)fp.b[jb] * lf->na + fp.a[ia]) * lf->h + fp.y[jy]) * lf->w + fp.x[ix];
                    for (int c = 0; c < 3; c++)
                        gs[3 * s + c] += wgt * grad_out[((int64_t)v * 3 + c) * npix + (int64_t)j * wo + i];
                }
            }
    /* colour transpose and path sums: dL/dS(node) = sum over the node's descendant views */
    memset(g_res, 0, sizeof(double) * 3 * lf->n_nodes * plane);
    memset(g_shift, 0, sizeof(double) * 2 * lf->n_pred_total);
    double* gS = (double*)calloc((size_t)(3 * lf->n_nodes * plane), sizeof(double));
    for (int b = 0; b < lf->nb; b++)
        for (int a = 0; a < lf->na; a++)
            for (int64_t px = 0; px < plane; px++) {
                const double* g = gs + (((int64_t)b * lf->na + a) * plane + px) * 3;
                double gy = g[0] + g[1] + g[2];
                double gco = 0.5 * g[0] - 0.5 * g[2];
                double gcg = -0.5 * g[0] + 0.5 * g[1] - 0.5 * g[2];
                for (int l = 0; l < lf->H; l++) {
                    int64_t node = lf->node_base[l] + (int64_t)(b >> l) * lf->na_l[l] + (a >> l);
                    gS[(0 * lf->n_nodes + node) * plane + px] += gy;
                    gS[(1 * lf->n_nodes + node) * plane + px] += gco;
                    gS[(2 * lf->n_nodes + node) * plane + px] += gcg;
                }
            }
    /* residuals receive their SRV's gradient; predictive SRVs push sigma *
     * bilinear-transpose into the reference residual and reduce shift grads */
    memcpy(g_res, gS, sizeof(double) * 3 * lf->n_nodes * plane);
    for (int c = 0; c < 3; c++)
        for (int l = 0; l < lf->H; l++)
            for (int B = 0; B < lf->nb_l[l]; B++)
                for (int A = 0; A < lf->na_l[l]; A++) {
                    if (!((A | B) & 1)) continue;
                    int64_t node = lf->node_base[l] + (int64_t)B * lf->na_l[l] + A;
                    int64_t rnode = lf->node_base[l] + (int64_t)(B & ~1) * lf->na_l[l] + (A & ~1);
                    const double* gp = gS + ((int64_t)c * lf->n_nodes + node) * plane;
                    double* gr = g_res + ((int64_t)c * lf->n_nodes + rnode) * plane;
                    const float* R = residual + ((int64_t)c * lf->n_nodes + rnode) * plane;
                    for (int k = 0; k < lf->nblk; k++) {
                        int sg = sigma_of(lf, c, l, B, A, k);
                        if (!sg) continue;
                        int64_t rec = lf->shift_base[c][l] + orc_pred_ordinal(lf->na_l[l], B, A) * lf->nblk + k;
                        double dx = shift[2 * rec], dy = shift[2 * rec + 1];
                        int by0 = (k / lf->nbx) * lf->bs, bx0 = (k % lf->nbx) * lf->bs;
                        for (int y = by0; y < by0 + lf->bs; y++)
                            for (int x = bx0; x < bx0 + lf->bs; x++) {
                                double g = gp[(int64_t)y * lf->w + x] * sg;
                                double X = x + dx, Y = y + dy;
                                double x0 = floor(X), y0 = floor(Y), fx = X - x0, fy = Y - y0;
                                int xa = orc_clampi((int)x0, 0, lf->w - 1), xb = orc_clampi((int)x0 + 1, 0, lf->w - 1);
                                int ya = orc_clampi((int)y0, 0, lf->h - 1), yb = orc_clampi((int)y0 + 1, 0, lf->h - 1);
                                gr[(int64_t)ya * lf->w + xa] += g * (1 - fx) * (1 - fy);
                                gr[(int64_t)ya * lf->w + xb] += g * fx * (1 - fy);
                                gr[(int64_t)yb * lf->w + xa] += g * (1 - fx) * fy;
                                gr[(int64_t)yb * lf->w + xb] += g * fx * fy;
                                double t00 = R[(int64_t)ya * lf->w + xa], t01 = R[(int64_t)ya * lf->w + xb];
                                double t10 = R[(int64_t)yb * lf->w + xa], t11 = R[(int64_t)yb * lf->w + xb];
                                g_shift[2 * rec] += g * ((1 - fy) * (t01 - t00) + fy * (t11 - t10));
                                g_shift[2 * rec + 1] += g * ((1 - fx) * (t10 - t00) + fx * (t11 - t01));
                            }
                    }
                }
    free(gS);
    free(gs);
    return 0;
}
