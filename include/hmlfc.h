/*
 * hmlfc.h -- C ABI of the MI355X (gfx950) HMLFC light-field decode + render library.
 *
 * HMLFC (Pratapa & Manocha, "HMLFC: Hierarchical Motion-Compensated Light
 * Field Compression for Interactive Rendering") stores a two-plane light
 * field as a tree of residual views (RLFC hierarchy) whose non-reference
 * views are phase-shifted motion-compensated against a reference view of
 * the same cluster, block-coded with bounded integer sequences.  This
 * library loads such a stream into device memory and serves random-access
 * sample decoding and novel-view rendering with hand-written HIP kernels.
 *
 * Conventions shared by every call:
 *  - Light-field samples are addressed (b, a, y, x): b = view row (v),
 *    a = view column (u), y = image row (t), x = image column (s).
 *  - A camera is float[18]: a row-major 3x3 homography h_uv followed by
 *    h_st.  Output pixel (i, j) (column, row) is mapped at its centre
 *    (i + 0.5, j + 0.5, 1); dividing by the third component gives the ray's
 *    (u, v) in view-grid units and (s, t) in image pixels.
 *  - "Device" pointers are HIP device allocations owned by the caller.  The
 *    render and decode calls allocate nothing; lf_footprint_bytes allocates
 *    a temporary buffer and the serving loop its small tables.
 *    "Host" pointers are ordinary process memory.
 *  - `stream` is a hipStream_t passed as void* (NULL = the default stream).
 *    Every call that takes a stream only enqueues work on it; outputs are
 *    ready when the stream is synchronised.  The exceptions say so: loading
 *    (lf_load_compressed, lf_load_compressed_ex) and the encoder
 *    (lf_encode_device) wait for their work before returning.
 *    Argument checks happen on the host before anything is enqueued.
 *  - Return value: LF_OK, or a negative lf_status; lf_last_error() gives a
 *    thread-local message for the last failure.
 *  - A handle is immutable after loading; calls that only read it may run
 *    concurrently on different streams.
 *
 * Stream format (little-endian; the encoder writes it, the loader checks
 * it): a 1024-byte header (magic "HMLFCv1", grid sizes, tree height H,
 * block size Bs, per-level quantisation steps and search windows, section
 * offsets, and a per-(channel, level) motion-vector directory), then
 *   root     int16 [3][nb_H][na_H][height][width]   level-H RKVs (YCoCg)
 *   table    8-byte entries [3][n_nodes][n_blocks]: u32 payload word,
 *            i16 minimum, u8 mode (0xFF = insignificant block), u8 0
 *   payload  u32 words of bounded-integer-sequence block payloads
 *   mv       u32 words: per (channel, level) BISE (mx + 4W, my + 4W)
 *            pairs, then 2-bit phase codes (0: +1, 1: -1, 2: none)
 * Nodes are numbered breadth-first from the top level (H-1) down to the
 * leaf views (level 0), raster order within a level (Compressed Stream
 * Structure).
 */
#ifndef HMLFC_H
#define HMLFC_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef struct lf_handle lf_handle;

typedef enum {
    LF_OK = 0,
    LF_EINVAL = -1,  /* bad argument: null pointer, size, range           */
    LF_ENOMEM = -2,  /* caller-provided buffer too small                  */
    LF_EFORMAT = -3, /* stream is malformed or inconsistent               */
    LF_EDEVICE = -4  /* a HIP call or kernel launch failed                */
} lf_status;

typedef struct {
    int32_t na, nb;          /* view grid: columns (u), rows (v)              */
    int32_t width, height;   /* view image size                               */
    int32_t levels;          /* tree height H                                 */
    int32_t block;           /* block size Bs                                 */
    int32_t root_na, root_nb;/* level-H grid                                  */
    int64_t n_nodes;         /* SRV nodes (levels 0..H-1)                     */
    int64_t n_pred_records;  /* motion-compensated blocks over all channels   */
    int64_t n_refs;          /* reference SRV views per channel               */
    int64_t arena_bytes;     /* device bytes the handle occupies              */
    int64_t stream_bytes;    /* compressed stream size                        */
    int64_t payload_bytes;   /* block payload section size                    */
    int64_t ref_bytes;       /* device bytes of the resident reference SRVs   */
    int32_t sparse_refs;     /* 0 dense planes, 1 LF_LOAD_SPARSE_REFS tiles,
                                2 LF_LOAD_CSR_REFS sparse rows                */
    int64_t clamped_coords;  /* decode requests (lf_decode_pixels, _lod) with
                                a coordinate outside the grid, clamped to it,
                                since load (Random Access for Interactive
                                Rendering: requests are grid positions)       */
    int32_t chroma420;       /* 1: Co and Cg coded at half width and height   */
} lf_info;

/* Load flag: keep the reference SRVs block-sparse (only significant blocks,
 * as int16 tiles, plus a tile index per block) instead of dense planes — the
 * reduced-memory reference storage of the Decompression Analysis.  Every
 * result is unchanged.  A sparse handle serves lf_decode_pixels(_lod),
 * lf_render_views(_per_ray, _lod) (one thread per ray) and the relaxed
 * render and adjoint; the serving loop rejects it. */
#define LF_LOAD_SPARSE_REFS 1

/* Load flag: keep the reference SRVs as a per-pixel sparse matrix in
 * compressed sparse rows (the paper's reference storage, Decompression
 * Analysis): per reference row, the columns (uint16) and values (int16) of
 * its nonzero pixels in increasing column order, and the row starts (uint32
 * [3][n_refs][height] + 1).  A tap binary-searches its row.  Same results
 * and same calls as LF_LOAD_SPARSE_REFS (not combinable with it); the arena
 * reserves values and columns for every pixel of the significant reference
 * blocks, lf_info.ref_bytes reports what the nonzeros use. */
#define LF_LOAD_CSR_REFS 2

/* ---------------------------------------------------------------------- */
/* Loading (Decompression Memory Overhead: the top-level RKVs and every    */
/* reference SRV are decoded once, before any sample is requested).        */
/* ---------------------------------------------------------------------- */

/* Parse a stream's header on the host and report the device arena size
 * lf_load_compressed needs.  host_stream: nbytes of stream.  Errors:
 * LF_EINVAL (null), LF_EFORMAT (malformed). */
lf_status lf_query_arena(const void* host_stream, size_t nbytes, int64_t* arena_bytes);

/* Validate the stream completely on the host, copy it into the caller's
 * device arena (d_arena, 256-byte aligned, arena_bytes >= lf_query_arena),
 * decode every reference SRV into resident int16 planes and expand every
 * block's table entry and motion vector into a 16-byte descriptor (Decoding
 * Procedure; Decompression Memory Overhead).  Arena sections, 256-byte
 * aligned: root, block table, payload, motion vectors, reference planes,
 * descriptors, 256-byte status.  The handle borrows d_arena until lf_free;
 * host_stream may be released when the call returns (the copy is complete
 * on return).  Errors: LF_EINVAL, LF_EFORMAT (any header field, section
 * size or block offset out of range, or a decoded reference SRV beyond
 * +-2047, which no stream of 8-bit content produces), LF_ENOMEM (arena too
 * small), LF_EDEVICE. */
lf_status lf_load_compressed(const void* host_stream, size_t nbytes, void* d_arena, int64_t arena_bytes,
                             void* stream, lf_handle** out);

/* lf_query_arena / lf_load_compressed with load flags (0, LF_LOAD_SPARSE_REFS
 * or LF_LOAD_CSR_REFS; other bits or both: LF_EINVAL; either with a 4:2:0
 * stream: LF_EINVAL).  Sparse arena sections:
 * root, block table, payload, motion vectors, reference tiles (int16
 * [n_tiles][Bs][Bs], significant reference blocks in (channel, reference
 * node, block) order), tile index (int32 [3][n_refs][n_blocks], -1 for a
 * zero block), status; no descriptors. */
lf_status lf_query_arena_ex(const void* host_stream, size_t nbytes, int32_t flags, int64_t* arena_bytes);
lf_status lf_load_compressed_ex(const void* host_stream, size_t nbytes, int32_t flags, void* d_arena,
                                int64_t arena_bytes, void* stream, lf_handle** out);

/* Release the host-side handle (the arena stays the caller's). */
lf_status lf_free(lf_handle* h);

/* Fills *out.  Reads the clamp counter with a synchronous copy on the null
 * stream: decode calls still running on other streams may not be counted
 * yet (synchronise their stream first).  Errors: LF_EINVAL, LF_EDEVICE. */
lf_status lf_get_info(const lf_handle* h, lf_info* out);

/* ---------------------------------------------------------------------- */
/* Random-access decoding (Decoding Procedure; Random Access for           */
/* Interactive Rendering): each requested sample walks its tree path from  */
/* the leaf view to the root, re-compensates motion-compensated blocks     */
/* from the resident reference, adds the root RKV and inverts the colour   */
/* transform.                                                              */
/* ---------------------------------------------------------------------- */

/* d_coords: device int32 [n][4] = (b, a, y, x), 16-byte aligned (else
 * LF_EINVAL); coordinates outside the grid are clamped to it, and each
 * clamped request adds one to lf_info.clamped_coords.  d_rgb: device uint8
 * [n][3].  n = 0 is a no-op. */
lf_status lf_decode_pixels(const lf_handle* h, const int32_t* d_coords, int64_t n, uint8_t* d_rgb, void* stream);

/* Progressive decoding (claimed in the Introduction's contributions and the
 * HMLFC Overview; the hierarchy of the RLFC scheme): the walk stops at tree
 * level `level`, giving samples of the reconstructed level-`level` node
 * images (the root RKV plus the SRVs of levels level .. H-1).  level = 0 is
 * lf_decode_pixels; level = H is the root RKV alone.  d_coords: device int32
 * [n][4] = (B, A, y, x) with (B, A) a node of that level (0 <= B <
 * ceil(nb / 2^level), likewise A); coordinates outside are clamped (and
 * counted in lf_info.clamped_coords).  Must be 16-byte aligned.  d_rgb: device uint8 [n][3].  LF_EINVAL for level outside
 * 0 .. H. */
lf_status lf_decode_pixels_lod(const lf_handle* h, int32_t level, const int32_t* d_coords, int64_t n,
                               uint8_t* d_rgb, void* stream);

/* ---------------------------------------------------------------------- */
/* Novel-view rendering fused with decoding (Random Access for             */
/* Interactive Rendering; two-plane interpolation of Light Field           */
/* Rendering).  Each ray's (u, v, s, t) is clamped to the grid; the 16     */
/* neighbouring samples are decoded and blended quadrilinearly in FP32:    */
/* per neighbouring view the (s, t) bilinear sum, then the (u, v) bilinear */
/* sum of the four, scaled to [0, 1] at the end.                           */
/* ---------------------------------------------------------------------- */

/* d_cams: device float [n_views][18].  d_out: device float
 * [n_views][3][height][width] (planar RGB).  width, height >= 1.  Runs the
 * staged tile kernel (on a 4:2:0 handle each leaf sample from the luma and
 * the up-sampled chroma decodes); fields with blocks smaller than 4x4 and
 * handles loaded with LF_LOAD_SPARSE_REFS or LF_LOAD_CSR_REFS run the
 * one-thread-per-ray kernel (same results). */
lf_status lf_render_views(const lf_handle* h, const float* d_cams, int32_t n_views, int32_t width,
                          int32_t height, float* d_out, void* stream);

/* Launch configuration lf_render_views uses for n_views views of
 * width x height: views decoded together per group, and views per workgroup
 * chunk (decoded samples are kept in LDS between the groups of a chunk).
 * The group size is HMLFC_VIEWS_PER_GROUP (1..64, default 12); the chunk is
 * HMLFC_VIEWS_PER_CHUNK (1..64) if set, else as long as the launch keeps
 * about 2048 workgroups of 32x8-pixel tiles (at most 64 views, balanced).
 * Both variables are read once, at first use.  Either pointer may be NULL;
 * LF_EINVAL for sizes below 1. */
lf_status lf_get_render_config(int32_t n_views, int32_t width, int32_t height, int32_t* views_per_group,
                               int32_t* views_per_chunk);

/* The same rendering with one thread per ray and no staging (every ray walks
 * its 16 samples' tree paths itself).  Same arguments and results as
 * lf_render_views, bit for bit; kept as the simple reference path. */
lf_status lf_render_views_per_ray(const lf_handle* h, const float* d_cams, int32_t n_views, int32_t width,
                                  int32_t height, float* d_out, void* stream);

/* Level-of-detail rendering from the progressive decode: the same rays and
 * blend as lf_render_views over the full-resolution view grid, but sample
 * (b, a, y, x) is read from the level-`level` node image of (b >> level,
 * a >> level), i.e. every view of a 2^level x 2^level cluster shows its
 * reconstructed RKV.  One thread per ray (the walk is short).  level = 0
 * equals lf_render_views_per_ray.  LF_EINVAL for level outside 0 .. H. */
lf_status lf_render_views_lod(const lf_handle* h, int32_t level, const float* d_cams, int32_t n_views,
                              int32_t width, int32_t height, float* d_out, void* stream);

/* Ray coordinates as the renderer computes them (binary32, no contraction):
 * d_uvst: device float [n_views][height][width][4] = (u, v, s, t) before
 * clamping.  For checking the renderer's arithmetic. */
lf_status lf_ray_coords(const float* d_cams, int32_t n_views, int32_t width, int32_t height, float* d_uvst,
                        void* stream);

/* Per-view footprint bytes: the output (12 bytes per ray) plus every
 * distinct predictive block's table entry, payload words and share of the
 * motion-vector stream, and 2 bytes per pixel of every distinct reference
 * or root block the view's samples read (through non-zero-weight prediction
 * taps for references).  Reuse across views is not credited.  host_out:
 * double [n_views].  Uses a temporary device buffer of about
 * 3 * (2 * n_nodes + root views) * n_blocks bytes per call (the library
 * allocates and frees it; this call synchronises `stream`). */
lf_status lf_footprint_bytes(const lf_handle* h, const float* d_cams, int32_t n_views, int32_t width,
                             int32_t height, double* host_out, void* stream);

/* For callers that cannot allocate device memory (code under HIP graph
 * capture, serving loops that must not call hipMalloc): the per-view
 * footprint bytes of lf_footprint_bytes, equal to its figures bit for bit,
 * written to d_out (device double [n_views]) and only enqueued on `stream`
 * (no synchronisation, no allocation).  Its scratch is a static device array
 * of LF_FOOTPRINT_SCRATCH_MAX bytes in the library (one per GPU, held until
 * the process ends), located with hipGetSymbolAddress on the first call on
 * each device: the marks take 2 * 3 * n_nodes * n_blocks + 3 * root views *
 * n_blocks bytes and the partial sums the last 8 KiB; a light field whose
 * marks do not fit is rejected with LF_EINVAL.  Every call on a GPU shares
 * that array, so calls that overlap on one GPU (other streams or threads)
 * race: serialise them.  Errors: LF_EINVAL, LF_EDEVICE. */
#define LF_FOOTPRINT_SCRATCH_MAX (64ll << 20)
lf_status lf_footprint_bytes_noalloc(const lf_handle* h, const float* d_cams, int32_t n_views, int32_t width,
                                     int32_t height, double* d_out, void* stream);

/* ---------------------------------------------------------------------- */
/* Relaxed model and adjoint (encoder-side refinement).  Parameters: a     */
/* real residual for every SRV value, float [3][n_nodes][height][width]    */
/* in breadth-first node order, and a real shift per motion-compensated    */
/* block, float [n_pred_records][2] = (dx, dy) in pixels, records ordered  */
/* by channel, then level from H-1 down to 0, then predictive node (raster */
/* order), then block.  A reference SRV equals its residual plane; a       */
/* predictive SRV is phase * bilinear(reference, shifted by (dx, dy)) plus */
/* its residual (the motion re-compensation of the Decoding Procedure with */
/* real values and no rounding); the colour inverse is linear, nothing is  */
/* clamped, and rays blend as in lf_render_views.                          */
/* ---------------------------------------------------------------------- */

/* Dequantised residuals and motion vectors / 4 of the loaded stream. */
lf_status lf_export_params(const lf_handle* h, float* d_residual, float* d_shift, void* stream);

/* Relaxed forward render; same camera and output layout as lf_render_views. */
lf_status lf_render_relaxed(const lf_handle* h, const float* d_residual, const float* d_shift, const float* d_cams,
                            int32_t n_views, int32_t width, int32_t height, float* d_out, void* stream);

/* Device workspace bytes lf_render_backward needs for this view batch.
 * Host-only.  LF_EINVAL for batches above 2^29 - 1 rays (n_views * width *
 * height; each ray contributes 4 records to a sort whose count is an int). */
lf_status lf_backward_workspace(const lf_handle* h, int32_t n_views, int32_t width, int32_t height, int64_t* bytes);

/* Adjoint of lf_render_relaxed: given d_grad_out = dL/d(out) (same layout
 * as the output), writes dL/d(residual) and dL/d(shift) (overwritten, not
 * accumulated).  Deterministic and free of atomics: the forward's ray
 * geometry is recomputed, never stored.  d_workspace: caller-owned,
 * 256-byte aligned, >= lf_backward_workspace bytes.  Errors: LF_EINVAL,
 * LF_ENOMEM (workspace too small), LF_EDEVICE. */
lf_status lf_render_backward(const lf_handle* h, const float* d_residual, const float* d_shift, const float* d_cams,
                             int32_t n_views, int32_t width, int32_t height, const float* d_grad_out,
                             float* d_grad_residual, float* d_grad_shift, void* d_workspace, int64_t workspace_bytes,
                             void* stream);

/* ---------------------------------------------------------------------- */
/* Serving: several loaded light fields stay resident; view requests of    */
/* mixed resolution are admitted by output memory and request slots and   */
/* continuously batched (32x8 tiles, round robin between requests) into    */
/* launches of a persistent kernel, each launch a replay of a graph        */
/* captured once per stream, with up to n_streams launches in flight.      */
/* A request's pixels are the same as lf_render_views' for its camera.     */
/* The server allocates only its small tables (geometry, slots, work       */
/* lists); outputs live in the caller's pool.                              */
/* ---------------------------------------------------------------------- */

typedef struct lf_server lf_server;

typedef struct {
    int32_t max_slots;   /* requests resident on the device at once (>= 1)            */
    int32_t max_tiles;   /* 32x8 tiles per launch (>= 1)                               */
    int32_t chunk_tiles; /* tiles one request adds to a launch per round (>= 1)        */
    int32_t n_streams;   /* launches in flight, 1..4                                   */
    int32_t use_graphs;  /* 1: each launch replays a captured graph                    */
    int32_t grid;        /* persistent workgroups per launch (0: 3 per compute unit)   */
} lf_server_config;

typedef struct {
    int64_t submitted, admitted, completed, launches, tiles;
    int64_t graph_launches; /* launches that replayed the captured graph (the rest: direct, one workgroup per tile) */
    double queue_ms;        /* summed over completed requests: submission to the first launch of their tiles */
    double flight_ms;       /* summed over completed requests: that launch to the completion seen */
} lf_server_stats;

/* fields: n_fields loaded handles (block size >= 4), borrowed for the
 * server's lifetime.  d_pool: caller-owned device memory of pool_bytes that
 * holds request outputs (float [3][height][width] each, 256-byte aligned). */
lf_status lf_server_create(lf_handle* const* fields, int32_t n_fields, void* d_pool, int64_t pool_bytes,
                           const lf_server_config* cfg, lf_server** out);
/* Queue a request (host camera float[18]).  auto_release = 1 frees its
 * output memory as soon as it completes (for load tests that do not read
 * it).  LF_ENOMEM if its output can never fit the pool. */
lf_status lf_server_submit(lf_server* s, int32_t field, const float* host_cam, int32_t width, int32_t height,
                           int32_t auto_release, int64_t* id);
/* Block until request id completes; its output starts at d_pool + *out_offset;
 * latency is from submission to the completion of its last launch. */
lf_status lf_server_wait(lf_server* s, int64_t id, double timeout_s, int64_t* out_offset, double* latency_ms);
/* Forget a completed request and return its output memory to the pool. */
lf_status lf_server_release(lf_server* s, int64_t id);
lf_status lf_server_get_stats(lf_server* s, lf_server_stats* out);
lf_status lf_server_destroy(lf_server* s);

/* Open-loop replay: request k (field[k], cams[k][18], wh[k] = width, height)
 * is submitted arrival_s[k] seconds after the call starts; latency_ms[k] is
 * measured from submission to completion; *makespan_s ends at the last
 * completion. */
lf_status lf_server_replay(lf_server* s, int64_t n, const int32_t* field, const float* cams, const int32_t* wh,
                           const double* arrival_s, double* latency_ms, double* makespan_s);
/* The same schedule served by one lf_render_views launch per request, in
 * arrival order on one stream (d_out holds the largest output). */
lf_status lf_serve_baseline(lf_handle* const* fields, int32_t n_fields, int64_t n, const int32_t* field,
                            const float* cams, const int32_t* wh, const double* arrival_s, void* d_out,
                            int64_t out_bytes, double* latency_ms, double* makespan_s);

/* ---------------------------------------------------------------------- */
/* Encoding on the GPU (not on the render path).  Follows the paper's      */
/* pipeline (Fig. 1): reversible YCoCg, the RLFC hierarchy of 2x2-cluster  */
/* rounded-mean RKVs, a top-down closed loop with phase-shifted quarter-pel */
/* motion compensation of the non-reference SRVs of every cluster (Eq.     */
/* 1-2), uniform quantisation with the two block thresholds (Compressing   */
/* HMLFC tree), and bounded-integer-sequence coding in breadth-first node  */
/* order (Compressed Stream Structure).                                    */
/* ---------------------------------------------------------------------- */

typedef struct {
    int32_t levels;      /* tree height H (1..8)                                   */
    int32_t block;       /* block size Bs (1..64, a power of two dividing width
                            and height; at least 2 unless no_mc)                   */
    int32_t step[8];     /* quantisation step per level (1..4096; 1 = lossless)    */
    int32_t t_ref[8];    /* block threshold for reference SRVs                     */
    int32_t t_pred[8];   /* block threshold for motion-compensated residuals       */
    int32_t win[8];      /* search window W per level, whole pixels (0..255,
                            block + 2W + 1 <= 96 unless no_mc)                     */
    int32_t subpel;      /* 1: quarter-pel refinement around the integer best      */
    int32_t zero_phase;  /* 1: allow "no prediction" when it is strictly cheaper   */
    int32_t no_mc;       /* 1: no motion compensation (plain hierarchy)            */
    int32_t chroma420;   /* 1: Co and Cg sub-sampled 4:2:0 (2x2 rounded mean) and
                            coded at half width and height; the image sides must
                            be multiples of twice the block size                   */
} lf_encode_params;

/* Device workspace lf_encode_device needs, in bytes: 256-byte aligned
 * sections for the uploaded light field (3 bytes per sample), the int16
 * YCoCg planes of every tree level (2 bytes per sample and channel, levels
 * 0..H), the coded SRV planes of level 0, the quantised values of every
 * block (2 bytes per value), per-block extremes, word counts, payload
 * offsets and table entries (28 bytes per block), the motion records (16
 * bytes each), the level-0 search items (12 bytes each), a payload bound of
 * 16 bits per value, and the motion-vector section.  LF_EINVAL for
 * parameters lf_encode_device rejects. */
lf_status lf_encode_workspace_bytes(int32_t nb, int32_t na, int32_t height, int32_t width,
                                    const lf_encode_params* params, int64_t* bytes);

/* host_lf: host uint8 [nb][na][height][width][3] RGB.  Every stage runs on
 * the GPU in d_work (caller-owned, 256-byte aligned, at least
 * lf_encode_workspace_bytes bytes; its contents are scratch): colour
 * transform, hierarchy, per level the SRVs, the reference blocks, the
 * motion search of every predictive block (lf_mc_search's kernel and
 * decisions), the predictive residuals and the reconstruction, then the
 * block modes, payload offsets (device prefix sum), table, payload and
 * motion-vector packing.  On success *out_stream is a malloc'ed stream of
 * *out_bytes bytes (header written on the host, sections copied back),
 * released with lf_encode_free.  Synchronous: waits for its work on
 * `stream`.  Errors: LF_EINVAL (geometry, parameters, or a quantised value,
 * coded SRV or reconstruction outside int16, which 8-bit input never
 * produces), LF_ENOMEM (workspace too small, or no host memory for the
 * stream), LF_EDEVICE. */
lf_status lf_encode_device(const uint8_t* host_lf, int32_t nb, int32_t na, int32_t height, int32_t width,
                           const lf_encode_params* params, void* d_work, int64_t work_bytes, void* stream,
                           uint8_t** out_stream, size_t* out_bytes);
void lf_encode_free(uint8_t* stream);

/* Phase-shifted motion search (Phase-shifted Motion Compensation, Eq. 1 and
 * 2) of n blocks on the GPU.  d_pred: device int16 [n_pred][height][width]
 * SRV planes to predict; d_ref: device int16 [n_ref][height][width]
 * reconstructed reference SRV planes.  d_items: device int32 [n][3] =
 * (pred plane, ref plane, block index k; block k covers rows
 * (k / (width / block)) * block and columns (k % (width / block)) * block).
 * For each item: the integer displacement (dx, dy) in [-win, win]^2 and phase
 * sigma in {+1, -1} minimising sum |p - sigma * R(x + dx, y + dy)| (clamped
 * reference coordinates), then, if subpel, the +-3 quarter-pel
 * neighbourhood of each phase's best (bilinear prediction
 * (sum w * tap + 8) >> 4, within +-4 win); candidates rank by (cost,
 * |mx| + |my|, my, mx), phase -1 wins only on a strictly lower cost; with
 * zero_phase, "no prediction" (sigma = 0) wins when strictly cheaper.
 * d_out: device int32 [n][4] = (mx, my, sigma, cost), mx/my in quarter
 * pixels, 16-byte aligned.  Per-item errors: cost -1 when the block to
 * predict holds the value -32768 (reference values may span the whole int16
 * range), cost -2 for an item whose indices are out of range.  block: 2, 4, 8, 16, 32 or 64,
 * dividing width and height; block + 2 win + 1 <= 96; else LF_EINVAL. */
lf_status lf_mc_search(const int16_t* d_pred, int64_t n_pred, const int16_t* d_ref, int64_t n_ref, int32_t width,
                       int32_t height, int32_t block, int32_t win, int32_t subpel, int32_t zero_phase,
                       const int32_t* d_items, int64_t n, int32_t* d_out, void* stream);

/* Message for the calling thread's last non-OK status. */
const char* lf_last_error(void);

#ifdef __cplusplus
}
#endif
#endif
