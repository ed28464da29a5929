/* HMLFC CPU oracle: private declarations.  TEST INFRASTRUCTURE ONLY. */
#ifndef HMLFC_ORACLE_INTERNAL_H
#define HMLFC_ORACLE_INTERNAL_H

#include "oracle.h"

/* Stream layout (little-endian).  The header is 1024 bytes:
 *    0  magic "HMLFCv1\0"        8  u32 header bytes (1024)   12 u32 version (1)
 *   16  i32 na  20 nb  24 width  28 height  32 levels  36 block  40 channels (3)  44 mv_prec (4)
 *   48  i32 step[8]             80  i32 win[8]
 *  112  u64 root_off, root_bytes, table_off, table_bytes, payload_off, payload_bytes, mv_off, mv_bytes
 *  176  mv directory [3][8] x 16 bytes: u32 mv_word, u32 sigma_word, u32 records, u8 mode, u8 pad[3]
 *  560  u32 chroma format: 0 = every channel at full size, 1 = 4:2:0 (Co, Cg at width/2 x height/2)
 * Sections (w_c x h_c and n_blocks_c: channel c's plane and block grid):
 *   root    int16, per channel c: [nb_H][na_H][h_c][w_c]
 *   table   8-byte entries, per channel c: [n_nodes][n_blocks_c]: u32 payload word, i16 min, u8 mode, u8 0
 *   payload u32 words (block payloads start on word boundaries), then >= 8 zero bytes
 *   mv      u32 words; per (channel, level): BISE motion vectors, then 2-bit phase codes
 */
#define ORC_HDR_BYTES 1024
#define ORC_HDR_CHROMA 560
#define ORC_INSIGNIFICANT 0xFF

struct orc_lf {
    const uint8_t* base;
    size_t len;
    int na, nb, w, h, H, bs;
    int step[ORC_MAX_LEVELS], win[ORC_MAX_LEVELS];
    int na_l[ORC_MAX_LEVELS + 1], nb_l[ORC_MAX_LEVELS + 1];
    int64_t node_base[ORC_MAX_LEVELS];
    int64_t n_nodes;
    int nbx, nby, nblk;          /* luma (channel 0) block grid */
    int chroma420;
    int cw[3], ch[3], cnbx[3], cnblk[3]; /* per-channel plane and block grid */
    int64_t tbase[3];            /* first table entry of each channel */
    int64_t rbase[3];            /* first root sample of each channel */
    const int16_t* root;
    const uint8_t* table;
    const uint32_t* payload;
    int64_t payload_words;
    const uint32_t* mv;
    int64_t mv_words;
    uint32_t mv_word[3][ORC_MAX_LEVELS], sig_word[3][ORC_MAX_LEVELS], mv_count[3][ORC_MAX_LEVELS];
    int mv_mode[3][ORC_MAX_LEVELS];
    int64_t shift_base[3][ORC_MAX_LEVELS];   /* relaxed-shift record base per (c, level) */
    int64_t n_pred_total;
};

/* geometry helpers */
int orc_asr(int x, int s);                 /* floor(x / 2^s) */
int orc_fdiv(int p, int q);                /* floor(p / q), q > 0 */
int orc_clampi(int v, int lo, int hi);
int64_t orc_pred_ordinal(int na_l, int B, int A);
int64_t orc_pred_nodes(int na_l, int nb_l);
void orc_level_grid(int na, int nb, int H, int* na_l, int* nb_l);

/* stream access */
int32_t orc_srv_value(const orc_lf* lf, int c, int l, int B, int A, int y, int x);
void orc_mv_record(const orc_lf* lf, int c, int l, int B, int A, int blk, int* mx, int* my, int* sigma);
int32_t orc_root_value(const orc_lf* lf, int c, int b, int a, int y, int x);

#endif
