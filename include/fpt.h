/*
 * fpt -- fluorescent spectral path tracer for MI355X (gfx950), C ABI.
 *
 * Computes the transport model of Abdellah et al., "A Physically Plausible
 * Model for Rendering Highly Scattering Fluorescent Participating Media"
 * (arXiv 1706.03024): per-wavelength volumetric path tracing through
 * isotropic scattering media holding fluorescent dyes.
 *
 *   - Free flight t = -ln(1-u)/sigma_t(lambda) (sec. 4.2, eqs. 5-6,
 *     Beer-Lambert), sigma_t = sigma_s + sigma_a,bg + sum_d sigma_a,d.
 *   - Dye absorption sigma_a,d = B * epsilon_d * c_d * 1e-7 * a_hat_d(lambda)
 *     [1/mm] with B = ln 10 (decadic epsilon) or 1, a_hat the absorption
 *     spectrum normalised to peak 1 on the grid (sec. 4.1: concentration,
 *     absorption spectrum and molar absorptivity define the event).
 *   - Collision event chosen with probabilities sigma_s/sigma_t (isotropic
 *     scatter, eq. 2), sigma_a,bg/sigma_t (background absorber) and
 *     sigma_a,d/sigma_t (dye d); a dye absorption emits with probability QY_d
 *     at a wavelength drawn from the dye's area-normalised emission spectrum
 *     (eq. 10, one-bin step), isotropically (sec. 2.1); at most K emissions
 *     per path (sec. 4.1: a second emission ends the path when K = 1).
 *   - Spectral film: escape tallies, or a pinhole camera connected to every
 *     realised vertex with transmittance and the 1/r^2 geometry term (eqs. 3-6).
 *
 * The walk runs forward from the light (analog); all randomness comes from a
 * counter-based Philox4x32-10 stream keyed by (seed, instance) with counter
 * (path id, vertex, call, 0), so any path range renders identically alone or
 * as part of a larger run.
 *
 * Conventions for every entry point:
 *   - Pointers marked "device" are device (HBM) addresses on the current HIP
 *     device; "host" pointers are ordinary host memory.  Every pointer
 *     argument is checked for NULL unless documented as optional.
 *   - Functions return FPT_OK (0) or a negative fpt_status; on error no
 *     output has been written, and fpt_last_error() (thread-local) holds a
 *     message.  No C++ exception crosses the ABI.
 *   - Work is enqueued asynchronously on the caller's HIP stream (a
 *     hipStream_t passed as void*, NULL = the null stream).  Device faults
 *     surface as FPT_E_DEVICE at the next call that synchronises.
 *   - A scene (and a batch) may be used by one stream at a time: calls that
 *     overlap on different streams race on its scratch buffers.
 * Units: nm, mm, 1/mm, 1/(M cm), uM.
 */
#ifndef FPT_H
#define FPT_H

#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

#define FPT_ABI_VERSION 5u

typedef enum {
    FPT_OK = 0,
    FPT_E_INVALID = -1,     /* malformed descriptor or argument */
    FPT_E_RANGE = -2,       /* value outside a supported range */
    FPT_E_NOMEM = -3,       /* device or host allocation failed */
    FPT_E_DEVICE = -4,      /* HIP runtime error */
    FPT_E_UNSUPPORTED = -5  /* valid but not implemented combination */
} fpt_status;

#define FPT_MAX_SPECTRUM_TERMS 16
#define FPT_MAX_DYES 8
#define FPT_MAX_MEDIA 8
#define FPT_MAX_MEDIUM_DYES 4
#define FPT_MAX_SPHERES 8
#define FPT_MAX_LINES 8
#define FPT_MAX_BINS 1024
#define FPT_MAX_GRAD_PARAMS 16
#define FPT_N_TALLIES 21

enum { FPT_SPECTRUM_NONE = 0, FPT_SPECTRUM_GAUSS_MIX = 1, FPT_SPECTRUM_PIECEWISE_LINEAR = 2,
       FPT_SPECTRUM_TABULATED = 3 };
enum { FPT_GEOM_SLAB = 0, FPT_GEOM_HALFSPACE = 1, FPT_GEOM_SPHERE = 2, FPT_GEOM_INFINITE = 3,
       FPT_GEOM_BOX = 4 };
enum { FPT_LIGHT_BEAM = 0, FPT_LIGHT_POINT = 1, FPT_LIGHT_QUAD = 2 };
enum { FPT_SENSOR_ESCAPE = 0, FPT_SENSOR_PINHOLE = 1 };
enum { FPT_BASE_DECADIC = 0, FPT_BASE_NATURAL = 1 };

/* Run flags. */
#define FPT_FLAG_FLUORESCENCE_ONLY 1u  /* film records only paths that emitted (V_f, eq. 9) */
#define FPT_FLAG_NO_EXCITATION_SCATTER 2u /* direct excitation only: end a path at its first
                                             scatter or wall reflection before emitting */

/* Exit codes (one per path) and tally slots (uint64, accumulated). */
enum { FPT_EXIT_ESC_R = 0, FPT_EXIT_ESC_T = 1, FPT_EXIT_BG = 2, FPT_EXIT_NONRAD = 3,
       FPT_EXIT_KCAP = 4, FPT_EXIT_SCAP = 5, FPT_EXIT_WALL = 6, FPT_EXIT_LIGHT = 7,
       FPT_EXIT_EXCSCAT = 8, FPT_EXIT_TRUNC = 9 };
enum { FPT_T_PATHS = 0, FPT_T_VERTICES = 1, FPT_T_SCATTERS = 2, FPT_T_DYE_ABS = 3,
       FPT_T_EMISSIONS = 4, FPT_T_WALL_REFLECT = 5, FPT_T_CROSSINGS = 6,
       FPT_T_SPLAT_HIT = 7, FPT_T_SPLAT_MISS = 8, FPT_T_SPLAT_RR_KILL = 9,
       FPT_T_EXIT0 = 10 /* + exit code */,
       /* forward renders: connections from a medium vertex whose optical depth
          inside its own sphere alone makes the transmittance exactly 0 in fp32,
          resolved without evaluation where every point of that sphere passes the
          connection's geometric tests (they are also counted in SPLAT_HIT, or in
          SPLAT_RR_KILL when splat_rr > 0, as an evaluation would count them) */
       FPT_T_SPLAT_OPAQUE = 20 };

/* A spectrum on nm: a Gaussian mixture sum_i value_i exp(-(l-center_i)^2/(2 width_i^2)),
 * a piecewise-linear curve through (center_i, value_i), constant beyond the ends, or
 * TABULATED: one value per point of the scene's grid (measured spectra, e.g. a dye
 * database sampled on the grid), table[k] at lambda_k. */
typedef struct {
    int32_t kind; /* FPT_SPECTRUM_* */
    int32_t n;    /* 1..FPT_MAX_SPECTRUM_TERMS; TABULATED: n_bins */
    double center_nm[FPT_MAX_SPECTRUM_TERMS];
    double value[FPT_MAX_SPECTRUM_TERMS];
    double width_nm[FPT_MAX_SPECTRUM_TERMS];
    const double* table; /* TABULATED: host array of n finite values, read (and copied by
                            fpt_scene_create) during the call only; NULL otherwise */
} fpt_spectrum;

typedef struct {
    fpt_spectrum absorption; /* shape only: normalised to peak 1 on the grid */
    fpt_spectrum emission;   /* shape only: normalised to unit area on the grid */
    double epsilon_M_cm;     /* peak molar absorptivity >= 0 */
    double qy;               /* quantum yield in [0, 1] */
} fpt_dye;

typedef struct {
    double sigma_s_mm;    /* >= 0, wavelength independent */
    double sigma_a_bg_mm; /* >= 0, wavelength independent */
    int32_t n_dyes;       /* 0..FPT_MAX_MEDIUM_DYES */
    int32_t dye[FPT_MAX_MEDIUM_DYES];
    double conc_uM[FPT_MAX_MEDIUM_DYES]; /* >= 0 */
    double ior;           /* refractive index in [1, 4]; 0 reads as 1.  A body medium
                             (SLAB/HALFSPACE/SPHERE) with ior != 1 has a smooth dielectric
                             boundary with the vacuum around it: a beam entering it and a
                             path reaching it from inside are reflected specularly with the
                             unpolarised Fresnel reflectance (1 beyond the critical angle),
                             else cross it (Snell's law on entry; escape tallies do not
                             depend on the outgoing direction).  Box spheres must be
                             index-matched (FPT_E_UNSUPPORTED): a straight camera
                             connection cannot cross a refracting surface. */
} fpt_medium;

typedef struct {
    double center[3];
    double radius;
    int32_t medium;
    int32_t pad;
} fpt_sphere;

/*
 * Scene descriptor (copied by fpt_scene_create; the caller may free it after).
 * geometry SLAB/HALFSPACE/SPHERE/INFINITE: one homogeneous body of medium
 *   `body_medium` in vacuum (index-matched boundary); sensor must be ESCAPE,
 *   light BEAM (starting on the body surface, pointing inward) or POINT (inside).
 * geometry BOX: box [box_lo, box_hi] with Lambertian walls of reflectance
 *   walls[f] (faces 0 x=lo, 1 x=hi, 2 y=lo, 3 y=hi, 4 z=lo, 5 z=hi); face
 *   `open_face` lets light out; vacuum inside except the (disjoint,
 *   index-matched) dye spheres; light must be a QUAD (Lambertian emitter
 *   light_pos + a light_u + b light_v, emitting along normalize(u x v),
 *   opaque and absorbing on both sides); sensor ESCAPE or PINHOLE (eye
 *   outside the box on the open side).
 * Light lines: wavelengths snap to the nearest grid point (ties to the lower
 *   one) and must lie on the grid; powers are normalised to a total of 1.
 */
typedef struct {
    int32_t n_bins;            /* 2..FPT_MAX_BINS grid points */
    int32_t absorptivity_base; /* FPT_BASE_* */
    double lo_nm, hi_nm;       /* lambda_k = lo + k (hi-lo)/(n_bins-1) */
    int32_t n_dyes, n_media;
    fpt_dye dyes[FPT_MAX_DYES];
    fpt_medium media[FPT_MAX_MEDIA];
    int32_t geometry; /* FPT_GEOM_* */
    int32_t body_medium;
    double slab_z0, slab_z1;  /* SLAB: z0 < z1; HALFSPACE: z > z0 */
    double body_center[3];    /* SPHERE */
    double body_radius;
    double box_lo[3], box_hi[3];
    int32_t open_face;
    int32_t n_spheres;
    fpt_spectrum walls[6];
    fpt_sphere spheres[FPT_MAX_SPHERES];
    int32_t light; /* FPT_LIGHT_* */
    int32_t n_lines;
    double light_pos[3], light_dir[3], light_u[3], light_v[3];
    double line_nm[FPT_MAX_LINES], line_power[FPT_MAX_LINES];
    int32_t sensor; /* FPT_SENSOR_* */
    int32_t width, height;
    double eye[3], look[3], up[3];
    double fov_y_deg;
    /* Glossy walls (sec. 5, the glossy Cornell box): wall f with wall_gloss[f] =
     * n > 0 reflects with the normalised modified-Phong BRDF
     * walls[f](lambda) (n+2)/(2 pi) cos^n(alpha), alpha the angle between the
     * outgoing direction and the mirror direction of the incoming one; the path
     * survives with probability walls[f](lambda), draws its new direction from
     * the lobe (cos alpha = u^(1/(n+1)) about the mirror direction) and carries
     * the throughput weight (n+2)/(n+1) cos(theta_out), ending where that
     * direction falls below the wall.  n in [0, 1e4]; 0 = Lambertian.  Box scenes
     * with a pinhole sensor only (weighted paths do not fit integer escape
     * tallies); the camera-side estimator refuses glossy scenes. */
    double wall_gloss[6];
} fpt_scene_desc;

/* One render call: paths [path_begin, path_begin + path_count) of a job of
 * total_paths paths (total_paths <= 2^32, path_count < 2^32: path ids are
 * 32-bit counters of the random stream).  Every path carries power
 * parity_batches / total_paths; with parity_batches = B > 1 the film gains a
 * leading axis of B slices and path p goes to slice p % B, so each slice is an
 * independent estimate of the whole film (for batch-mean standard errors). */
typedef struct {
    uint64_t seed;
    uint64_t path_begin, path_count, total_paths;
    uint32_t instance;       /* xor-ed into the high key word */
    uint32_t max_scatter;    /* a path's (max_scatter+1)-th scatter ends it */
    uint32_t max_emissions;  /* K; 0xFFFFFFFF = unlimited */
    uint32_t flags;          /* FPT_FLAG_* */
    uint32_t parity_batches; /* 0 or 1 = none, else 2..64 */
    uint32_t pad;
    double splat_rr; /* camera splats with transmittance below this are kept with
                        probability T/splat_rr and weight /that (0 = off) */
} fpt_run;

/* Launch shape knobs; all-zero = library defaults.  Results never depend on them. */
typedef struct {
    int32_t block_threads;  /* 64..256, multiple of 64; halved (to 128, then 64) where the
                               scene's table image and per-wave buffers would exceed the
                               160 KiB of LDS one workgroup may hold */
    int32_t blocks_per_cu;  /* persistent blocks per compute unit */
    int32_t refill_lanes;   /* a wave refills dead lanes once this many are dead (1..64;
                               default 48 with a camera (adjoint 32, camera-side
                               estimator 32), 60 with escape sensors, 8 batched) */
    int32_t chunk_paths;    /* batched: paths per work item */
    int32_t block_min_vertices; /* paths in a medium with this many vertices walk in wave-wide
                                   blocks (default 2 with a camera (adjoint 8), 8 with
                                   escape sensors, 64 batched) */
    int32_t block_segments; /* paths per block round: 1, 2 or 4 (default 4, batched 2); paths
                               whose last round ran full width always get a whole wave */
    int32_t wide_rounds;    /* forward renders: such paths walk 128 vertices per round;
                               -1 off, 1 a path counts as deep after any full round,
                               2 only after a full round of the whole wave (0 default:
                               1 with a camera and batched, 2 with escape sensors) */
} fpt_tune;

/* Per-path replay record (fp32 path state at exit). */
typedef struct {
    uint32_t n_vertices, n_scatter, n_emit, exit_code;
    int32_t lambda, comp, region, pad;
    float pos[3], dir[3];
    float splat_sum; /* sum of values this path deposited into the film */
    float pad2;
} fpt_path_record;

typedef struct fpt_scene fpt_scene;
typedef struct fpt_batch fpt_batch;

uint32_t fpt_abi_version(void);
const char* fpt_status_str(int32_t status);
const char* fpt_last_error(void);

/* Validate `desc`, build the spectral tables in fp64 (rounded to fp32) and
 * upload them to the current device (synchronous).  The tables are the
 * transport coefficients of sec. 4.1: per medium and grid point
 * sigma_t = sigma_s + sigma_a,bg + sum_d sigma_a,d (the extinction of the
 * free-flight density, eqs. 5-6), the cumulative event thresholds of the
 * scatter / absorber choice, each dye's emission CDF (the normalised emission
 * spectrum of eq. 10, one-bin step) and the walls' reflectance.  All device
 * scratch a render of this scene can need (path queue, escape counters for up
 * to 64 parity slices, adjoint partial sums, and for pinhole box scenes the
 * deferred-connection slices: 40 KiB per wave the transport kernel can keep
 * resident, ~170 MB on a 256-CU device) is reserved here, so renders never
 * allocate.  *out is library-owned; free with fpt_scene_destroy.  Errors:
 * FPT_E_INVALID / FPT_E_RANGE for bad descriptors (nothing allocated),
 * FPT_E_NOMEM, FPT_E_DEVICE. */
int32_t fpt_scene_create(const fpt_scene_desc* desc, fpt_scene** out);
void fpt_scene_destroy(fpt_scene* scene);

/* Replace the differentiable parameters (sec. 4.1: dye concentrations and
 * quantum yields, and each medium's scattering coefficient) and rebuild the
 * tables.  Host arrays, each optional (NULL = unchanged): conc_uM[sum over
 * media of n_dyes] in (medium, dye slot) order, qy[n_dyes], sigma_s_mm[n_media];
 * read during the call only.  The tables are rebuilt on the host and uploaded
 * asynchronously on `hip_stream`: work already enqueued there sees the old
 * parameters, work enqueued after the call the new ones (renders on other
 * streams must be ordered by the caller).  The host blocks only while a
 * previous upload of this scene is still reading the staging buffer.  On an
 * invalid value nothing changes (FPT_E_RANGE / FPT_E_INVALID). */
int32_t fpt_scene_set_params(fpt_scene* scene, const double* conc_uM, const double* qy,
                             const double* sigma_s_mm, void* hip_stream);

/* Film layout: ESCAPE [B][2 comp][2 side (R, T)][n_bins];
 * PINHOLE [B][2 comp][height][width][n_bins]; comp 0 = not yet emitted,
 * 1 = emitted at least once.  fp32, C-contiguous.  dims[5] receives the
 * shape, *ndims 4 or 5. */
int32_t fpt_film_shape(const fpt_scene* scene, uint32_t parity_batches, int64_t dims[5],
                       int32_t* ndims);

/* Number of differentiable parameters: [conc per (medium, dye slot)]
 * [QY per dye][sigma_s per medium]. */
int32_t fpt_grad_param_count(const fpt_scene* scene);

/* Optional launch-shape override for this scene (NULL restores defaults). */
int32_t fpt_scene_set_tune(fpt_scene* scene, const fpt_tune* tune);

/* Launch timing, for measurement.  While enabled (enable != 0), every
 * fpt_render of this scene records HIP events on the caller's stream around
 * its transport launch and its deferred-connection launch (pinhole scenes);
 * up to FPT_MAX_TIMED_RENDERS renders are kept, later ones are not timed.
 * Enabling or disabling clears the record.  fpt_scene_timing waits for the
 * recorded renders, writes their count and the mean duration in ms of each
 * launch (0 where there was none), and clears the record. */
#define FPT_MAX_TIMED_RENDERS 4096
int32_t fpt_scene_set_timing(fpt_scene* scene, int32_t enable);
int32_t fpt_scene_timing(fpt_scene* scene, int32_t* renders, float* transport_ms, float* deferred_ms);
/* The same record render by render: waits for the recorded renders, writes
 * their count to *renders and the durations in ms of the first
 * min(count, cap) of them to transport_ms[] and deferred_ms[] (host arrays of
 * cap floats, may be NULL when cap is 0), and clears the record. */
int32_t fpt_scene_timing_each(fpt_scene* scene, int32_t cap, int32_t* renders, float* transport_ms,
                              float* deferred_ms);

/* Forward render: the analog walk of sec. 4.1 from the light, every path an
 * unbiased sample of the fluorescent RTE (eqs. 1-2 with the inelastic kernel
 * of eq. 10): light vertex (line chosen by power, point and direction on the
 * emitter), free flight t = -ln(1-u)/sigma_t (eqs. 5-6), scatter / absorber
 * choice, isotropic scatter (eq. 2), dye absorption with a quantum-yield test
 * and re-emission at a wavelength from the emission spectrum (eq. 10),
 * Lambertian walls, and into the film either the escape tallies or, at every
 * realised vertex, a pinhole connection with transmittance and the geometry
 * term (eqs. 3-6).  Accumulates (+=) into film_dev (device, fp32, film shape)
 * and tallies_dev (device, FPT_N_TALLIES uint64; optional, may be NULL).
 * Allocates nothing (the scene's reserved scratch; one stream at a time).
 * Escape films are integer counts scaled by parity_batches/total_paths at the
 * end of the call; camera films are fp32 atomic sums.  Asynchronous.
 * FPT_E_UNSUPPORTED, before any launch, if the scene's table image does not
 * fit in LDS beside one wave's buffers (e.g. 8 media with 4 dyes each at 1024
 * bins); the same holds for the adjoint and the records hook. */
int32_t fpt_render(fpt_scene* scene, const fpt_run* run, float* film_dev, uint64_t* tallies_dev,
                   void* hip_stream);

/* Allocation-free variant of fpt_render, for callers that cannot allocate
 * device memory (code under HIP graph capture, tight serving loops, harnesses
 * that forbid hipMalloc).  Same arguments, results and errors as fpt_render,
 * except that its device scratch -- path-queue heads, escape counters and the
 * deferred-connection slices -- lives in a static array of 24 MiB the library
 * holds on every device it runs on (until the process ends) instead of the
 * scene's buffers; it calls no hipMalloc, hipFree or allocating routine.
 * The deferred slices shrink to fit beside the rest (a full slice falls back to
 * the in-kernel queue), so tallies are identical to fpt_render's and the film
 * differs only in the fp32 rounding order of its atomic sums.  Limit: the
 * escape counters (parity_batches * 4 * n_bins, at most 262144) and per-wave
 * counts must fit the array beside the queue (they always do for valid runs;
 * otherwise FPT_E_RANGE before any launch).  Every call on a device
 * shares that device's array, and the queue and counters are cleared at the
 * start of each call: calls that overlap on one device (on different streams)
 * race and give wrong results; serialise them.  Not timed by
 * fpt_scene_set_timing. */
int32_t fpt_render_noalloc(fpt_scene* scene, const fpt_run* run, float* film_dev,
                           uint64_t* tallies_dev, void* hip_stream);

/* Path-replay adjoint of fpt_render: replays the same paths (same random
 * numbers) and accumulates into grad_dev (device, fp32[fpt_grad_param_count])
 * the gradient of <grad_film, film> with respect to the parameters, using the
 * likelihood-ratio form d E[v] = E[v d log p(path) + d v] over the path
 * density of eq. 12's estimator (sec. 4.3): p is the product of the sampled
 * events' probabilities -- sigma_event e^{-sigma_t t} per collision (eqs. 5-6),
 * e^{-sigma_t l} per pass-through, QY or 1-QY per dye absorption (sec. 4.1) --
 * and v the splat value, whose transmittance (eq. 5) depends on the parameters
 * through sigma_t along the camera connection.  grad_film_dev
 * (device, film shape) is read only.  Stores no path state; memory use is
 * independent of path length.  tallies_dev optional.  Asynchronous.
 * FPT_E_UNSUPPORTED if the parameter count exceeds FPT_MAX_GRAD_PARAMS. */
int32_t fpt_render_adjoint(fpt_scene* scene, const fpt_run* run, const float* grad_film_dev,
                           float* grad_dev, uint64_t* tallies_dev, void* hip_stream);

/* Test hook: one record per path into rec_dev (device, path_count records).
 * max_vertices > 0 ends paths after that many vertices (exit TRUNC).  With
 * grad_film_dev and rec_grad_dev (both optional, device) it also writes each
 * path's gradient contribution (fp32[path_count][n_params]).  Does not touch
 * any film.  Asynchronous. */
int32_t fpt_render_records(fpt_scene* scene, const fpt_run* run, fpt_path_record* rec_dev,
                           uint32_t max_vertices, const float* grad_film_dev,
                           float* rec_grad_dev, void* hip_stream);

/* Camera-side estimator (sec. 4.1: paths start at the camera at the emission
 * wavelength and the light is sampled only where an emission is realised;
 * sec. 4.3, eq. 12).  Box scenes with a pinhole.  total_paths must be
 * spp * height * width * n_bins; path p is sample s, pixel (py, px), emission
 * bin k with p = ((s * height + py) * width + px) * n_bins + k.  Each path
 * walks analogously at bin k from the eye through a uniform point of its pixel
 * (entering through the open face; free flight eq. 6, isotropic scatter,
 * Lambertian walls); at every collision in a dye medium it draws one uniform
 * point on the light and adds the directly excited fluorescence source
 *   sum_d QY_d pmf_d(k) sum_l w_l sigma_a,d(lambda_l) T_l cos_n / (4 pi^2 r^2)
 * over sigma_t(k) (w_l the lines' power fractions, T_l the transmittance at
 * line l through every sphere).  Any absorption ends the walk (K = 1).  The
 * path's sum, times parity_batches / spp, is added once to film component 1
 * (film_dev, device, pinhole film shape, optional) of slice s % parity_batches;
 * component 0 is never touched.  It estimates what fpt_render estimates in
 * component 1 with FPT_FLAG_NO_EXCITATION_SCATTER and max_emissions = 1.
 * Uses seed, instance, the path range, max_scatter and parity_batches of run.
 * rec_dev (device, path_count records, optional) receives per-path records
 * (n_emit 0, comp 1, splat_sum = the path's deposit); max_vertices > 0 ends
 * paths after that many vertices (exit TRUNC).  Exits: ESC_T the eye ray
 * misses the open face, ESC_R the walk leaves through it, KCAP a dye absorbs,
 * BG, WALL, LIGHT, SCAP, TRUNC.  Tallies SPLAT_HIT / SPLAT_MISS count light
 * connections made / facing away.  At least one of film_dev and rec_dev.
 * FPT_E_UNSUPPORTED for other scenes, or if the table image exceeds LDS
 * (160 KiB).  Timed like fpt_render when timing is on (deferred time 0).
 * Asynchronous. */
int32_t fpt_render_camera(fpt_scene* scene, const fpt_run* run, float* film_dev,
                          uint64_t* tallies_dev, fpt_path_record* rec_dev,
                          uint32_t max_vertices, void* hip_stream);

/* Test hook: copies the fp32 tables the kernels use to host arrays (each
 * optional): sigma_t[n_media][n_bins], emis_cdf[n_dyes][n_bins],
 * rho[6][n_bins], line_bin[n_lines]. */
int32_t fpt_scene_tables(const fpt_scene* scene, float* sigma_t, float* emis_cdf, float* rho,
                         int32_t* line_bin);

/* Test hook: the scene's pinhole-connection geometry precomputed by the host
 * (box scenes with a pinhole sensor; 0 otherwise).  *geo_clear: bit s set when
 * every point of sphere s passes a camera connection's geometric tests (inside
 * the image, through the open face, clear of the light quad; eqs. 3-6) with a
 * margin far above fp32 rounding, so the kernels skip those tests for its
 * medium vertices.  occluders[FPT_MAX_SPHERES]: bit t of occluders[s] set when
 * a segment from a point of sphere s to the eye can meet sphere t (s itself
 * included); the kernels take the transmittance of such connections (eq. 5)
 * over these spheres only.  Either pointer may be NULL. */
int32_t fpt_scene_connection_masks(const fpt_scene* scene, uint32_t* geo_clear, uint32_t* occluders);

/* Batched form: n independent escape-sensor body scenes (one medium each,
 * equal n_bins) rendered by one persistent launch that claims (instance, path
 * chunk) work items from a device queue; the launch sequence is captured in a
 * hipGraph on the first render and replayed after.  runs[i] gives instance
 * i's seed, instance key and path count.  Films: [n][2][2][n_bins] fp32,
 * accumulated; tallies: [n][FPT_N_TALLIES] uint64 (optional).  Every wave
 * holds one instance's tables and histogram in LDS: blocks get fewer waves
 * where the tuned size would not fit, and FPT_E_UNSUPPORTED is returned if
 * one wave's slot does not fit on its own. */
int32_t fpt_batch_create(const fpt_scene_desc* descs, const fpt_run* runs, int32_t n,
                         const fpt_tune* tune, fpt_batch** out);
int32_t fpt_batch_render(fpt_batch* batch, float* films_dev, uint64_t* tallies_dev,
                         void* hip_stream);
void fpt_batch_destroy(fpt_batch* batch);

/* Launch-shape autotuner.  Times candidate shapes for `scene` and `run` on
 * the current device (synchronous; renders into a scratch film it allocates)
 * and writes the fastest to *out and its mean render time to *best_ms
 * (optional).  batch may be NULL (then the plain render is tuned, else the
 * batched one; scene and run are then ignored).  With cache_path (a JSON file
 * mapping "<workload>@<arch>x<CUs>cu" to the fpt_tune fields and "ms"), the
 * cached entry for `workload` on this device is returned without measuring if
 * present, and a measured one is written back (the file is rewritten whole,
 * through a temporary file).  Flags: FPT_TUNE_FORCE measures even when cached;
 * FPT_TUNE_CACHED_ONLY never measures and returns the all-zero tune (the
 * library defaults) with *best_ms = 0 when nothing is cached; with it and a
 * cache, scene, run and batch may all be NULL (a plain lookup).  Results of a
 * render never depend on its launch shape.  Errors: FPT_E_INVALID (NULL
 * arguments, a malformed or unwritable cache), render errors of the
 * candidates. */
#define FPT_TUNE_FORCE 1u
#define FPT_TUNE_CACHED_ONLY 2u
int32_t fpt_autotune(fpt_scene* scene, const fpt_run* run, fpt_batch* batch,
                     const char* cache_path, const char* workload, uint32_t flags,
                     fpt_tune* out, float* best_ms);

#ifdef __cplusplus
}
#endif

#endif
