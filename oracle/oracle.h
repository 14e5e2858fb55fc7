/*
 * CPU oracle for the fluorescent spectral path tracer.
 *
 * TEST INFRASTRUCTURE ONLY.  This is a plain, slow, single-threaded fp64
 * implementation of what the GPU path computes, written from the paper
 * (Abdellah et al., "A Physically Plausible Model for Rendering Highly
 * Scattering Fluorescent Participating Media", arXiv 1706.03024) and checked
 * against closed forms.  Only the tests, the smoke check and the benchmark's
 * CPU-baseline leg may load it.  It shares no code, header, table or helper
 * with the GPU library.
 *
 * Model (paper section 4.1, equations 1-12, with the readings recorded in the
 * design notes):
 *   - forward analog walk from the light, per discrete wavelength bin;
 *   - free flight t = -ln(1-u)/sigma_t(lambda) (eq. 6, Beer-Lambert);
 *   - collision event chosen among scatter / background absorber / dye d with
 *     probabilities sigma_s/sigma_t, sigma_a_bg/sigma_t, sigma_a_d/sigma_t;
 *   - dye absorption: quantum-yield test, then re-emission at a wavelength drawn
 *     from the dye's normalised emission spectrum (eq. 10), isotropic (sec. 2.1);
 *   - at most K emissions per path (sec. 4.1: a second emission terminates);
 *   - a body medium with refractive index n != 1 has a smooth dielectric
 *     boundary: an entering beam and every path reaching the boundary from
 *     inside are reflected specularly with the unpolarised Fresnel reflectance
 *     (1 beyond the critical angle), else cross it (Snell's law on entry);
 *   - spectral film: escape tallies, or a pinhole camera splat at every
 *     realised vertex (eqs. 3-6: transmittance, geometry term 1/r^2).
 *
 * Parity status: every function below is pinned by the CPU tests against a
 * closed form, an invariant or a library routine, except the camera splat of
 * multi-sphere Cornell scenes, which is pinned only through its components
 * (direct light radiance, single-scatter radiance, wall irradiance).
 */
#ifndef FPT_ORACLE_H
#define FPT_ORACLE_H

#include <stdint.h>

#define ORC_MAX_TERMS 16
#define ORC_MAX_DYES 8
#define ORC_MAX_MEDIA 8
#define ORC_MAX_MEDIUM_DYES 4
#define ORC_MAX_SPHERES 8
#define ORC_MAX_LINES 8
#define ORC_MAX_BINS 2048
#define ORC_MAX_PARAMS (ORC_MAX_MEDIA * ORC_MAX_MEDIUM_DYES + ORC_MAX_DYES + ORC_MAX_MEDIA)

enum { ORC_SPEC_NONE = 0, ORC_SPEC_GAUSS = 1, ORC_SPEC_PWL = 2, ORC_SPEC_TAB = 3 };
enum { ORC_GEOM_SLAB = 0, ORC_GEOM_HALFSPACE = 1, ORC_GEOM_SPHERE = 2,
       ORC_GEOM_INFINITE = 3, ORC_GEOM_BOX = 4 };
enum { ORC_LIGHT_BEAM = 0, ORC_LIGHT_POINT = 1, ORC_LIGHT_QUAD = 2 };
enum { ORC_SENSOR_ESCAPE = 0, ORC_SENSOR_PINHOLE = 1 };

/* Exit codes: exactly one per path. */
enum { ORC_EXIT_ESC_R = 0, ORC_EXIT_ESC_T = 1, ORC_EXIT_BG = 2, ORC_EXIT_NONRAD = 3,
       ORC_EXIT_KCAP = 4, ORC_EXIT_SCAP = 5, ORC_EXIT_WALL = 6, ORC_EXIT_LIGHT = 7,
       ORC_EXIT_EXCSCAT = 8, ORC_EXIT_TRUNC = 9, ORC_N_EXITS = 10 };

/* Tally slots (uint64, accumulated). */
enum { ORC_T_PATHS = 0, ORC_T_VERTICES = 1, ORC_T_SCATTERS = 2, ORC_T_DYE_ABS = 3,
       ORC_T_EMISSIONS = 4, ORC_T_WALL_REFLECT = 5, ORC_T_CROSSINGS = 6,
       ORC_T_SPLAT_HIT = 7, ORC_T_SPLAT_MISS = 8, ORC_T_SPLAT_RR_KILL = 9,
       ORC_T_EXIT0 = 10, ORC_N_TALLIES = 20 };

typedef struct {
    int32_t kind; /* ORC_SPEC_* */
    int32_t n;
    double x[ORC_MAX_TERMS]; /* Gaussian mean (nm) or knot position (nm) */
    double y[ORC_MAX_TERMS]; /* Gaussian weight or knot value */
    double s[ORC_MAX_TERMS]; /* Gaussian standard deviation (nm) */
    const double* tab;       /* ORC_SPEC_TAB: n = n_bins values, one per grid point */
} orc_spectrum;

typedef struct {
    orc_spectrum absorption, emission;
    double epsilon; /* peak molar absorptivity, 1/(M cm) */
    double qy;      /* quantum yield in [0,1] */
} orc_dye;

typedef struct {
    double sigma_s, sigma_a_bg; /* 1/mm, wavelength independent */
    int32_t n_dyes;
    int32_t dye[ORC_MAX_MEDIUM_DYES];
    double conc[ORC_MAX_MEDIUM_DYES]; /* uM */
    double ior; /* refractive index; 0 or 1: index-matched to the vacuum around it */
} orc_medium;

typedef struct {
    double center[3], radius;
    int32_t medium;
} orc_sphere;

typedef struct {
    int32_t n_bins;
    double lo_nm, hi_nm;
    int32_t natural_base; /* 0: sigma_a = ln10*eps*c*a_hat, 1: eps*c*a_hat */
    int32_t n_dyes;
    orc_dye dyes[ORC_MAX_DYES];
    int32_t n_media;
    orc_medium media[ORC_MAX_MEDIA];
    int32_t geom;
    double z0, z1;             /* slab / half-space */
    double center[3], radius;  /* single sphere */
    int32_t body_medium;
    double box_lo[3], box_hi[3];
    int32_t open_face;
    orc_spectrum walls[6];
    int32_t n_spheres;
    orc_sphere spheres[ORC_MAX_SPHERES];
    int32_t light;
    double lpos[3], ldir[3], lu[3], lv[3];
    int32_t n_lines;
    double line_nm[ORC_MAX_LINES], line_power[ORC_MAX_LINES];
    int32_t sensor;
    double eye[3], look[3], up[3], fov_y_deg;
    int32_t width, height;
    /* Glossy walls (sec. 5: the glossy Cornell box): wall f reflects with the
     * normalised modified-Phong BRDF rho_f(lambda) (n+2)/(2 pi) cos^n(alpha),
     * alpha the angle between the outgoing direction and the mirror direction,
     * when wall_gloss[f] = n > 0 (pinhole scenes only); 0 = Lambertian. */
    double wall_gloss[6];
} orc_scene;

typedef struct {
    uint64_t seed;
    uint32_t instance;
    uint32_t max_scatter;
    uint64_t path_begin, path_count, total_paths;
    uint32_t max_emissions; /* K; 0xFFFFFFFF = unlimited */
    int32_t fluorescence_only;
    int32_t excitation_scatter; /* 0: end a path at its first scatter or wall reflection
                                   before emitting (direct excitation only) */
    uint32_t parity_batches;    /* B >= 1: film slice = path_id % B */
    double splat_rr;            /* transmittance roulette threshold, 0 = off */
    /* Conditioning probe for replay comparisons (0 = off, the plain walk).  With
     * perturb_eta > 0 every position and direction the walk computes is scaled,
     * coordinate by coordinate, by (1 +- perturb_eta) with a sign hashed from
     * (path, vertex, coordinate, perturb_pattern) right after it is computed
     * (a coordinate set exactly on a planar boundary stays exact).  Comparing
     * such a run with the plain one measures how much a relative error of that
     * size at every vertex moves each record field: the path's condition
     * number, which bounds what any fp32 walk of the same path can reproduce. */
    double perturb_eta;
    uint32_t perturb_pattern;
    uint32_t pad_;
} orc_run;

typedef struct {
    uint32_t n_vertices, n_scatter, n_emit, exit_code;
    int32_t lambda, comp, region, pad;
    double pos[3], dir[3];
    double splat_sum; /* sum of the values this path deposited */
    double margin;    /* smallest relative decision margin along the path */
} orc_record;

/* The glossy wall lobe (test hooks).  Directions: wi the incoming travel
 * direction, wo the outgoing one, nrm the wall's inward unit normal.
 * orc_phong_eval returns the BRDF over rho: (n+2)/(2 pi) cos^n(alpha), alpha
 * between wo and the mirror direction of wi (0 when wo or wi is on the wrong
 * side of the wall).  orc_phong_sample draws wo about the mirror direction
 * with density (n+1)/(2 pi) cos^n(alpha) from uniforms (ua, ub) and returns
 * the throughput factor BRDF cos(theta_o) / (rho pdf) = (n+2)/(n+1) cos(theta_o),
 * or 0 when wo falls below the wall (the path ends there). */
double orc_phong_eval(double n, const double* wi, const double* wo, const double* nrm);
double orc_phong_sample(double n, const double* wi, const double* nrm, double ua, double ub,
                        double* wo);

/* Philox4x32-10 (Salmon et al., SC'11): out = bijection(ctr) under key. */
void orc_philox4x32_10(const uint32_t ctr[4], const uint32_t key[2], uint32_t out[4]);

/* Number of film floats for this scene and B batches; 0 on error. */
int64_t orc_film_size(const orc_scene* sc, uint32_t batches);
int32_t orc_n_params(const orc_scene* sc);
const char* orc_last_error(void);

/* Tables as the walk uses them (fp64).  Arrays of n_bins per entry:
 *   lambda[N], a_hat[n_dyes*N], emis_cdf[n_dyes*N], sigma_t[n_media*N],
 *   sigma_a[n_media*4*N] (per medium dye slot), rho[6*N].  Any may be NULL. */
int32_t orc_tables(const orc_scene* sc, double* lambda, double* a_hat, double* emis_pmf,
                   double* emis_cdf, double* sigma_t, double* sigma_a, double* rho,
                   int32_t* line_bin);

/* Run the walk for paths [path_begin, path_begin+path_count).
 *   film      accumulates (+=) the spectral film, may be NULL
 *   tallies   accumulates ORC_N_TALLIES counters, may be NULL
 *   gfilm     adjoint seed (same shape as the film); with grad != NULL the
 *             path-replay gradient estimator accumulates into grad[n_params]
 *   rec       one record per path, may be NULL
 *   rec_grad  n_params per path (needs gfilm), may be NULL
 *   max_vertices  > 0 truncates paths (exit TRUNC) for records
 * Returns 0 on success, negative on invalid input. */
int32_t orc_render(const orc_scene* sc, const orc_run* run, double* film, uint64_t* tallies,
                   const double* gfilm, double* grad, orc_record* rec, double* rec_grad,
                   uint32_t max_vertices);

/* Camera-side estimator (sec. 4.1, eq. 12): paths start at the eye at the
 * emission wavelength and connect to the light at every collision in a dye
 * medium (direct excitation, lines summed with their power fractions).  Box
 * scenes with a pinhole and a quad light.  Path p of total_paths =
 * spp * height * width * n_bins is (sample s, pixel (py, px), bin k) with
 *   p = ((s * height + py) * width + px) * n_bins + k,
 * and adds to film component 1 of slice s % parity_batches with weight
 * parity_batches / spp.  Uses seed, instance, the path range, max_scatter and
 * parity_batches of run.  Record fields as for orc_render (n_emit 0, comp 1,
 * splat_sum = the path's deposit).  Exits: ESC_T the eye ray misses the open
 * face, ESC_R the walk leaves through it, KCAP a dye absorbs at the emission
 * wavelength, BG, WALL, LIGHT, SCAP, TRUNC as for orc_render.  Tallies
 * SPLAT_HIT / SPLAT_MISS count light connections made / facing away. */
int32_t orc_render_camera(const orc_scene* sc, const orc_run* run, double* film,
                          uint64_t* tallies, orc_record* rec, uint32_t max_vertices);

#endif
