// Host-side internals shared by the library's translation units.
#pragma once

#include <cstdarg>
#include <cstdint>

#include "../../include/hmlfc.h"
#include "lf_geom.h"

struct LfLayout {
    LfGeom g;
    uint64_t root_off, root_bytes, table_off, table_bytes, payload_off, payload_bytes, mv_off, mv_bytes;
    int64_t n_rec;        // motion records over all channels and levels
    int64_t stream_bytes;
    // arena offsets
    int64_t a_root, a_table, a_payload, a_mv, a_refs, a_desc, a_status, arena;
    // sparse reference residency (LF_LOAD_SPARSE_REFS): a_refs holds n_tiles
    // block tiles, a_slots the tile of every reference block; no descriptors
    int32_t sparse;  // reference residency: LF_RES_DENSE, LF_RES_TILES or LF_RES_CSR
    int64_t n_tiles, a_slots;
    // CSR residency: values (int16, at a_refs) and columns of at most
    // nnz_bound nonzero reference pixels, and row starts; nnz is the count
    // found at load
    int64_t nnz_bound, nnz, a_cols, a_rowptr;
    // 4:2:0 chroma (Co and Cg at half width and height): g is the luma
    // geometry (one channel) and gc the chroma geometry (two channels), each
    // with its own root, table, reference planes (at a_refs and a_refs_c)
    // and motion directories; no descriptors
    int32_t chroma420;
    LfGeom gc;
    int64_t a_refs_c;
};

struct lf_handle {
    LfLayout L;
    uint8_t* arena;
    LfPtrs p;   // every channel, or luma for 4:2:0
    LfPtrs pc;  // 4:2:0 chroma (Co, Cg)
};

// LF_EINVAL unless the handle's chroma planes are full size (calls built on
// one uniform plane geometry: the tile renderer, the relaxed model and its
// adjoint, footprint accounting, serving)
lf_status lf_require_full_chroma(const lf_handle* h, const char* what);

lf_status lf_fail(lf_status s, const char* fmt, ...);
lf_status lf_check_launch(const char* what);
lf_status lf_parse(const uint8_t* s, size_t n, LfLayout* L);

// Phase-shifted motion search (lf_search.hip) on device planes, for the
// device encoder: checks the sizes, enqueues k_mc_search on `stream`.
lf_status lf_search_launch(const int16_t* pred, const int16_t* ref, int64_t n_pred, int64_t n_ref, int w, int h,
                           int bs, int win, int subpel, int zero_phase, const int32_t* items, int64_t n, int32_t* out,
                           void* stream);
