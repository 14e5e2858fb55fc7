// Internal structures shared by the fpt host library and its HIP kernels.
#pragma once

#include <stdint.h>

#include "fpt.h"

namespace fpt {

constexpr int kMaxNP = FPT_MAX_GRAD_PARAMS;
constexpr int kMedWords = 20;  // words per medium record in the table image
constexpr int kDyeWords = 4;   // words per dye record

// Medium record (32-bit words) in the table image:
//   0 sigma_s  1 sigma_s + sigma_a_bg  2 n_dyes (int)  3 1/sigma_s
//   4..7 dye index per slot (int)  8..11 1/conc per slot
//   12 gradient index of sigma_s (int)  13..16 gradient index of conc per slot (int)
// Dye record: 0 qy  1 1/qy  2 1/(1-qy)  3 gradient index of qy (int)
enum { MW_SS = 0, MW_THR_BG = 1, MW_NDYES = 2, MW_INV_SS = 3, MW_DYE = 4, MW_INV_C = 8,
       MW_PSS = 12, MW_PC = 13 };
enum { DW_QY = 0, DW_INV_QY = 1, DW_INV_1MQY = 2, DW_PQ = 3 };

struct KSphere {
    float c[3];
    float r2;
    int medium;
    int st_row;  // word offset of the medium's (sigma_t, 1/sigma_t) row in the table image
    int pad[2];
};

// Everything a launch needs that is uniform across the grid (kernel argument).
struct KParams {
    // table image (32-bit word offsets); staged into LDS by every block
    int N;
    int table_words;
    int off_med, off_dye;
    int off_st;     // float2 [n_media][N]: sigma_t, 1/sigma_t (+inf where sigma_t = 0)
    int off_cum;    // float [n_media][cum_stride][N]: absolute thresholds of dye slots 0..n-2
    int cum_stride;
    int off_cdf;    // float [n_dyes][N]: emission CDF, last entry exactly 1
    int off_rho;    // float [6][N]
    int off_kap;    // float [n_media][kap_stride][N]: d sigma_a / d conc per slot
    int kap_stride;
    int n_media, n_dyes, n_spheres, n_lines;
    KSphere spheres[FPT_MAX_SPHERES];
    float line_cum[FPT_MAX_LINES];
    int line_bin[FPT_MAX_LINES];
    int geometry, body_medium, light, sensor;
    float z0, z1;
    float bc[3], br2;
    float lo[3], hi[3];
    int open_face;
    // the open face's plane: unit vectors of its axis and of the two others
    // (one-hot), the plane's coordinate and the face's extent along the others
    float vis_e[3][3];
    float vis_plane, vis_lo1, vis_hi1, vis_lo2, vis_hi2;
    float lpos[3], ldir[3], lu[3], lv[3], ln[3], lt1[3], lt2[3];
    float lu_inv2, lv_inv2;
    float eye[3], cf[3], cr[3], cu[3];
    float inv_tanx, inv_tany;
    int W, H;
    float splat_norm;  // N_pix / A_img
    int film_u32;      // film element indices fit 32 bits (deposits merge per wave)
    // run
    uint32_t key0, key1;
    uint32_t path_begin, path_count;
    uint32_t batches;
    float wscale;  // batches / total_paths
    uint32_t max_scatter, max_emissions;
    int fluo_only, exc_scatter;
    float splat_rr, inv_splat_rr;
    uint32_t max_vertices;
    int hist_words;  // > 0: escape counts go through a per-block LDS histogram of this size
    int np;
    int refill_lanes;
    uint32_t block_min_v;  // paths with at least this many vertices walk in wave blocks
    int max_segments;      // long paths served per block round: 1, 2 or 4
    int wide_rounds;       // forward: deep paths walk 128 vertices per round (0 off); a path is
                           // deep after any full round (1) or a full whole-wave round (2)
    // Fields added after the rest: the box forward kernel keeps the earlier ones in
    // scalar registers, and moving them (by inserting fields before them) changed
    // its scalar-register spills enough to cost 9 % of its instructions.
    // camera-side estimator (box + pinhole + quad light), at the end of the image:
    int off_src;    // float [n_media][N][n_lines]: w_l sum_d QY_d pmf_d(k) sigma_a,d(lambda_l) / (4 pi^2)
    int off_csig;   // float [n_spheres][n_lines]: sigma_t of sphere s's medium at line l
    float tanx, tany;
    float ior;  // refractive index of the body medium (1: index-matched boundary)
    // bit s: every point of sphere s passes a camera connection's geometric
    // tests (in the image, through the open face, clear of the light quad) with
    // margin, and its medium can reach an optical depth of kTauZero inside it
    uint32_t sph_clear;
    // glossy walls: word offset of the walls' Phong exponents (6 floats, 0 =
    // Lambertian) in the table image, and whether any wall is glossy
    int off_gloss;
    int glossy;
    // pinhole connections from medium vertices: bit s of geo_clear when every
    // point of sphere s passes the connection's geometric tests with margin
    // (sph_clear adds the optical-depth condition), and sph_occl[s] the
    // spheres whose chord a connection from inside sphere s can have nonzero
    // (s itself included; a sphere outside it meets no such segment)
    uint32_t geo_clear;
    uint32_t sph_occl[FPT_MAX_SPHERES];
    // optical depth from which a medium vertex's connection deposits exactly 0
    // (at most kTauZero; set per run from the deposit's weight)
    float tau_zero;
};

// Optical depth past which a transmittance is exactly 0 in fp32: exp(-103.3)
// is already below the smallest subnormal.
constexpr float kTauZero = 110.f;

// Words per queued camera connection (structure of arrays): x, y, z, two packed
// words (roulette bits, vertex kind, wall face, component; wavelength bin,
// parity slice) and the path's throughput weight (glossy walls only).
constexpr int kEntryWords = 6;

struct KBuffers {
    const uint32_t* tables;        // table image in device memory
    float* film;                   // camera film (pinhole)
    uint32_t* counts;              // escape counts [B][2][2][N]
    unsigned long long* tallies;   // FPT_N_TALLIES
    unsigned long long* counter;   // path queue head
    const float* gfilm;            // adjoint seed (film shape)
    float* partials;               // adjoint: [grid blocks][kMaxNP]
    fpt_path_record* rec;          // records mode
    float* rec_grad;               // records mode, [path_count][np]
    uint32_t* sjobs;               // deferred pinhole connections: per wave [5][sjob_slice] words, or null
    uint32_t* sjob_counts;         // entries written per wave
    uint32_t sjob_slice;
};

// Batched form: one work item = a path range of one instance.
struct KWorkItem {
    uint32_t instance;  // index into the instance arrays
    uint32_t path_lo;   // path indices [path_lo, path_hi) relative to the instance's path_begin
    uint32_t path_hi;
    uint32_t pad;
};

struct KBatch {
    const KParams* params;          // [n_instances] complete per-instance launch parameters
    const uint32_t* tables;         // concatenated table images
    const uint32_t* table_off;      // [n_instances] word offset of each image
    const KWorkItem* items;         // [n_items], largest expected cost first
    int n_items;
    int n_instances;
    int slot_words;                 // LDS words per wave: tally | histogram | table
    int hist_words;                 // 4 * n_bins
    uint32_t* counts;               // [n_instances][hist_words] escape counts
    unsigned long long* tallies;    // [n_instances][FPT_N_TALLIES] or null
    unsigned long long* item_counter;
    int refractive;                 // some instance has a refracting body boundary
};

}  // namespace fpt
