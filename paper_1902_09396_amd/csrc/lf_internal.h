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

// Device motion search for the encoder (lf_search.hip): uploads one level's
// SRV planes S and reconstructed planes Shat (n_planes each, [plane][h][w]),
// searches every item (pred plane, ref plane, block) and copies the results
// (mx, my, sigma, cost) to the host buffer out; synchronous on stream.
int64_t lf_search_work_bytes(int64_t n_planes, int w, int h, int64_t n_items);
lf_status lf_search_level_device(const int16_t* S, const int16_t* Shat, int64_t n_planes, int w, int h, int bs,
                                 int win, int subpel, int zero_phase, const int32_t* items, int64_t n_items,
                                 int32_t* out, void* d_work, int64_t work_bytes, void* stream);
