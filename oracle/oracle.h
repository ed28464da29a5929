/*
 * HMLFC CPU oracle -- TEST INFRASTRUCTURE ONLY.
 *
 * A plain, slow, single-purpose C implementation of the HMLFC codec
 * (Pratapa & Manocha, "HMLFC: Hierarchical Motion-Compensated Light Field
 * Compression for Interactive Rendering"): an encoder, a full-tree decoder, a
 * random-access decoder, a two-plane light-field renderer and the relaxed
 * (real-valued) forward model with its adjoint.  It exists to check the GPU
 * library against.  Only the test-suite, the smoke check and the benchmark's
 * CPU-baseline leg may load it; the GPU library never links, includes or
 * calls it, and it shares no source with that library.
 *
 * Paper sections followed (cited by title):
 *   RLFC: Hierarchical Compression Scheme        -> clusters, RKV, SRV, tree height
 *   Phase-shifted Motion Compensation (Eq. 1-2)  -> search, phase sign, replacement
 *   Compressing HMLFC tree                       -> YCoCg, per-channel trees, block thresholds
 *   Bounded Integer Sequence Encoding            -> block payloads
 *   Compressed Stream Structure                  -> BFS order, BISE motion vectors
 *   Decompression / Decoding Procedure           -> tree traversal + re-compensation + root
 *   Decompression Memory Overhead                -> reference SRVs decoded up front
 *   Future Work (sub-pel motion compensation)    -> quarter-pel bilinear prediction
 *   Prior Work / Light Field Rendering           -> two-plane (u,v,s,t) interpolation
 *
 * Conventions: a light field is uint8 L[b][a][y][x][3] (b = view row (v),
 * a = view column (u), y = t, x = s).  Integer division and right shifts of
 * signed values are floors.  All integer arithmetic is int32/int64; the
 * renderer evaluates ray coordinates in IEEE binary32 without contraction
 * and blends in binary64.
 *
 * Every function is pinned by CPU tests against properties the paper and
 * the mathematics fix.  Parity unpinned: the cluster shape and RKV weights
 * (the paper defers them to RLFC, whose text is not available), taken here
 * as grid-aligned 2x2 clusters with an equal-weight rounded mean.
 */
#ifndef HMLFC_ORACLE_H
#define HMLFC_ORACLE_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

#define ORC_MAX_LEVELS 8

typedef struct {
    int32_t levels;                   /* tree height H: number of SRV levels           */
    int32_t block;                    /* block size Bs                                 */
    int32_t step[ORC_MAX_LEVELS];     /* quantisation step per level (1 = lossless)    */
    int32_t t_ref[ORC_MAX_LEVELS];    /* block threshold, reference SRVs               */
    int32_t t_pred[ORC_MAX_LEVELS];   /* block threshold, motion-compensated residuals */
    int32_t win[ORC_MAX_LEVELS];      /* search window W in whole pixels               */
    int32_t subpel;                   /* 1: quarter-pel refinement after integer search */
    int32_t zero_phase;               /* 1: also allow "no prediction" (sigma = 0)     */
    int32_t no_mc;                    /* 1: disable motion compensation (plain RLFC)   */
    int32_t chroma420;                /* 1: Co and Cg coded at half width and height   */
} orc_params;

typedef struct orc_lf orc_lf;

/* ---- building blocks (exposed for the pins) ---- */
void orc_ycocg_fwd(int r, int g, int b, int* y, int* co, int* cg);
void orc_ycocg_inv(int y, int co, int cg, int* r, int* g, int* b);
void orc_ycocg_fwd_n(const int32_t* rgb, int64_t n, int32_t* ycc);
void orc_ycocg_inv_n(const int32_t* ycc, int64_t n, int32_t* rgb);
/* quarter-pel bilinear prediction of pixel (y, x) of a w x h plane shifted by
 * (mx, my) quarter pixels, before the phase sign is applied */
int32_t orc_qpel(const int32_t* plane, int w, int h, int y, int x, int mx, int my);
/* phase-shifted search of one block (origin (by0, bx0), size bs) of the
 * predictive plane p against the reference plane r; returns the cost */
int64_t orc_mc_search(const int32_t* p, const int32_t* r, int w, int h, int by0, int bx0, int bs,
                      int win, int subpel, int zero_phase, int* mx, int* my, int* sigma);
/* bounded-integer-sequence coding of n values in [0, ...]; mode byte as in the stream */
int orc_bise_choose(const uint32_t* v, int n);                 /* returns the mode byte */
int64_t orc_bise_bits(int mode, int n);                          /* size in bits          */
void orc_bise_pack(const uint32_t* v, int n, int mode, uint32_t* words); /* words zeroed by caller */
uint32_t orc_bise_get(const uint32_t* words, int mode, int i);   /* random access         */
void orc_bise_unpack(const uint32_t* words, int mode, int n, uint32_t* v); /* sequential */

/* 4:2:0 chroma (Compressing HMLFC tree: chroma channels are sub-sampled):
 * the half-resolution plane is the 2x2 rounded mean, floor((sum + 2) / 4);
 * decoding brings it back to full resolution with centred bilinear weights
 * (sample (Y, X) sits at full-resolution position (2Y + 1/2, 2X + 1/2)):
 * full-resolution row y reads half-resolution rows (y/2 - 1, y/2) with
 * weights (1, 3) when y is even and (y/2, y/2 + 1) with (3, 1) when odd,
 * clamped to the plane, columns likewise, (sum of w * v + 8) >> 4. */
void orc_chroma_down(const int32_t* full, int w, int h, int32_t* half);
void orc_chroma_up(const int32_t* half, int w, int h, int32_t* full);  /* w, h: full size */

/* ---- encoder ---- */
int orc_encode(const uint8_t* lf, int nb, int na, int h, int w, const orc_params* p,
               int nthreads, uint8_t** out, size_t* out_len);
void orc_free(void* p);

/* ---- stream ---- */
int orc_open(const uint8_t* stream, size_t len, orc_lf** out);  /* borrows stream */
void orc_close(orc_lf* lf);
/* na, nb, w, h, levels, block, n_nodes, n_pred_total, root_na, root_nb, chroma420 */
void orc_info(const orc_lf* lf, int64_t* out11);
/* decoded value of channel c at its own resolution (half size for 4:2:0
 * chroma): coords[k] = (b, a, y, x) in that channel's plane; lod as in
 * orc_decode_node (0: leaf views) */
int orc_decode_channel_at(const orc_lf* lf, int c, int lod, const int32_t* coords, int64_t n, int32_t* out);

/* ---- decoders ---- */
int orc_decode_at(const orc_lf* lf, const int32_t* coords, int64_t n, uint8_t* rgb);
int orc_decode_node(const orc_lf* lf, int level, const int32_t* coords, int64_t n, uint8_t* rgb); /* (B,A,y,x) */
int orc_decode_at_ycocg(const orc_lf* lf, const int32_t* coords, int64_t n, int32_t* ycc);
int orc_decode_full(const orc_lf* lf, uint8_t* out);           /* [nb][na][h][w][3]        */
int orc_decode_full_ycocg(const orc_lf* lf, int32_t* out);     /* [3][nb][na][h][w]        */
/* per-level decoded SRV planes S_hat: [3][n_nodes][h][w] (BFS node order) */
int orc_decode_srv(const orc_lf* lf, int32_t* out);

/* ---- threads of the OpenMP loops (n <= 0: all processors); returns the count in effect ---- */
int orc_set_threads(int n);

/* ---- renderer ---- */
int orc_ray_coords(const float* cam, int wo, int ho, int i, int j, float* uvst4);
int orc_render(const orc_lf* lf, const float* cams, int nv, int wo, int ho, int nthreads, double* out);
/* rendering with every sample's walk stopped at level lod (progressive decode) */
int orc_render_lod(const orc_lf* lf, int lod, const float* cams, int nv, int wo, int ho, double* out);
int orc_render_rays(const orc_lf* lf, const float* cams, int wo, int ho, const int32_t* rays, int64_t n,
                    double* out);
int orc_render_dense(const uint8_t* lf, int nb, int na, int h, int w, const float* cams, int nv,
                     int wo, int ho, double* out);
int orc_footprint_bytes(const orc_lf* lf, const float* cams, int nv, int wo, int ho, double* out);

/* ---- relaxed model (real residuals, real per-block shifts) ---- */
int orc_export_params(const orc_lf* lf, float* residual, float* shift);
int orc_render_relaxed(const orc_lf* lf, const float* residual, const float* shift,
                       const float* cams, int nv, int wo, int ho, int nthreads, double* out);
int orc_relaxed_grad(const orc_lf* lf, const float* residual, const float* shift,
                     const float* cams, int nv, int wo, int ho, const double* grad_out,
                     double* g_res, double* g_shift);
/* For one parameter (kind 0: residual flat index, kind 1: shift flat index =
 * 2*record + component), over the rays it affects: central difference of the
 * loss sum((render - target)^2) with step eps, and the exact derivative by
 * forward-mode propagation.  Returns the number of affected rays. */
int64_t orc_param_check(const orc_lf* lf, const float* residual, const float* shift,
                        const float* cams, int nv, int wo, int ho, const float* target,
                        int kind, int64_t index, double eps, double* fd, double* fwd);
/* Relaxed loss sum((render - target)^2) over all rays. */
double orc_relaxed_loss(const orc_lf* lf, const float* residual, const float* shift,
                        const float* cams, int nv, int wo, int ho, const float* target, int nthreads);

#ifdef __cplusplus
}
#endif
#endif
