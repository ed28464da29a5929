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
    int32_t sparse;
    int64_t n_tiles, a_slots;
};

struct lf_handle {
    LfLayout L;
    uint8_t* arena;
    LfPtrs p;
};

lf_status lf_fail(lf_status s, const char* fmt, ...);
lf_status lf_check_launch(const char* what);
lf_status lf_parse(const uint8_t* s, size_t n, LfLayout* L);

// Phase-shifted motion search (lf_search.hip) on device planes, for the
// device encoder: checks the sizes, enqueues k_mc_search on `stream`.
lf_status lf_search_launch(const int16_t* pred, const int16_t* ref, int64_t n_pred, int64_t n_ref, int w, int h,
                           int bs, int win, int subpel, int zero_phase, const int32_t* items, int64_t n, int32_t* out,
                           void* stream);
