/*
 * CPU oracle for the fluorescent spectral path tracer (fp64, single thread).
 * TEST INFRASTRUCTURE ONLY: see oracle.h.  Each step cites the paper passage
 * (section / equation) it follows.
 */
#define _GNU_SOURCE
#include "oracle.h"

#include <math.h>
#include <stdio.h>
#include <stdlib.h>
#include <string.h>

#ifndef M_PI
#define M_PI 3.14159265358979323846
#endif

static char g_err[256];

const char* orc_last_error(void) { return g_err; }

static int fail(const char* msg) {
    snprintf(g_err, sizeof g_err, "%s", msg);
    return -1;
}

/* ------------------------------------------------------------------------- */
/* Philox4x32-10, from the published description (Salmon, Moraes, Dror, Shaw,
 * "Parallel random numbers: as easy as 1, 2, 3", SC'11): ten rounds of two
 * 32x32->64 multiplies with fixed multipliers, the high halves xor-ed with the
 * other two counter words and the round key, the key bumped by the Weyl
 * constants (golden ratio and sqrt(3)-1 in 32-bit fixed point) between rounds. */
void orc_philox4x32_10(const uint32_t ctr[4], const uint32_t key[2], uint32_t out[4]) {
    uint32_t x0 = ctr[0], x1 = ctr[1], x2 = ctr[2], x3 = ctr[3];
    uint32_t k0 = key[0], k1 = key[1];
    for (int round = 0; round < 10; ++round) {
        uint64_t p0 = (uint64_t)0xD2511F53u * (uint64_t)x0;
        uint64_t p1 = (uint64_t)0xCD9E8D57u * (uint64_t)x2;
        uint32_t y0 = (uint32_t)(p1 >> 32) ^ x1 ^ k0;
        uint32_t y1 = (uint32_t)p1;
        uint32_t y2 = (uint32_t)(p0 >> 32) ^ x3 ^ k1;
        uint32_t y3 = (uint32_t)p0;
        x0 = y0; x1 = y1; x2 = y2; x3 = y3;
        k0 += 0x9E3779B9u;
        k1 += 0xBB67AE85u;
    }
    out[0] = x0; out[1] = x1; out[2] = x2; out[3] = x3;
}

/* 24-bit uniform in [0,1). */
static double unif(uint32_t w) { return (double)(w >> 8) * (1.0 / 16777216.0); }

typedef struct {
    uint32_t key[2];
    uint32_t pid;
} rng_t;

static void draw(const rng_t* r, uint32_t vertex, uint32_t call, uint32_t out[4]) {
    uint32_t ctr[4] = {r->pid, vertex, call, 0u};
    orc_philox4x32_10(ctr, r->key, out);
}

/* ------------------------------------------------------------------------- */
/* Spectral tables (sec. 4.1: absorption spectrum, molar absorptivity and
 * concentration define the dye absorption; eq. 10: the emitted wavelength
 * follows the area-normalised emission spectrum with a one-bin step). */

typedef struct {
    int N;
    double lo, delta;
    double* lambda;   /* N */
    double* a_hat;    /* n_dyes x N, peak-normalised absorption */
    double* pmf;      /* n_dyes x N, emission probability per bin */
    double* cdf;      /* n_dyes x N */
    double* sigma_t;  /* n_media x N */
    double* sigma_a;  /* n_media x 4 x N */
    double* kappa;    /* n_media x 4 x N: d sigma_a / d conc */
    double* rho;      /* 6 x N */
    int line_bin[ORC_MAX_LINES];
    double line_cum[ORC_MAX_LINES];
} tables_t;

/* Value at grid point k (wavelength lam): tabulated spectra are given on the grid. */
static double eval_spectrum(const orc_spectrum* s, double lam, int k) {
    if (s->kind == ORC_SPEC_TAB) return s->tab[k];
    if (s->kind == ORC_SPEC_GAUSS) {
        double v = 0.0;
        for (int i = 0; i < s->n; ++i) {
            double z = (lam - s->x[i]) / s->s[i];
            v += s->y[i] * exp(-0.5 * z * z);
        }
        return v;
    }
    if (s->kind == ORC_SPEC_PWL) {
        if (lam <= s->x[0]) return s->y[0];
        if (lam >= s->x[s->n - 1]) return s->y[s->n - 1];
        for (int i = 0; i + 1 < s->n; ++i) {
            if (lam <= s->x[i + 1]) {
                double f = (lam - s->x[i]) / (s->x[i + 1] - s->x[i]);
                return s->y[i] + f * (s->y[i + 1] - s->y[i]);
            }
        }
        return s->y[s->n - 1];
    }
    return 0.0;
}

static int check_spectrum(const orc_spectrum* s, int allow_none, int n_bins) {
    if (s->kind == ORC_SPEC_NONE) return allow_none ? 0 : fail("spectrum missing");
    if (s->kind == ORC_SPEC_TAB) {
        if (!s->tab || s->n != n_bins) return fail("tabulated spectrum needs n_bins values");
        for (int k = 0; k < n_bins; ++k)
            if (!isfinite(s->tab[k])) return fail("spectrum not finite");
        return 0;
    }
    if (s->kind != ORC_SPEC_GAUSS && s->kind != ORC_SPEC_PWL) return fail("unknown spectrum kind");
    if (s->n < 1 || s->n > ORC_MAX_TERMS) return fail("spectrum term count out of range");
    for (int i = 0; i < s->n; ++i) {
        if (!isfinite(s->x[i]) || !isfinite(s->y[i])) return fail("spectrum not finite");
        if (s->kind == ORC_SPEC_GAUSS && !(s->s[i] > 0.0)) return fail("gaussian sd <= 0");
        if (s->kind == ORC_SPEC_GAUSS && s->y[i] < 0.0) return fail("gaussian weight < 0");
        if (s->kind == ORC_SPEC_PWL && i > 0 && !(s->x[i] > s->x[i - 1]))
            return fail("pwl knots not increasing");
    }
    return 0;
}

static int line_bin_of(double nm, double lo, double delta, int N) {
    /* nearest grid point, ties to the lower index */
    double q = (nm - lo) / delta;
    double k = ceil(q - 0.5);
    if (!(k >= 0.0) || k > (double)(N - 1)) return -1;
    return (int)k;
}

static void free_tables(tables_t* t) {
    free(t->lambda); free(t->a_hat); free(t->pmf); free(t->cdf);
    free(t->sigma_t); free(t->sigma_a); free(t->kappa); free(t->rho);
    memset(t, 0, sizeof *t);
}

static int validate(const orc_scene* sc) {
    if (sc->n_bins < 2 || sc->n_bins > ORC_MAX_BINS) return fail("n_bins out of range");
    if (!(sc->hi_nm > sc->lo_nm)) return fail("grid hi <= lo");
    if (sc->n_dyes < 0 || sc->n_dyes > ORC_MAX_DYES) return fail("n_dyes out of range");
    if (sc->n_media < 0 || sc->n_media > ORC_MAX_MEDIA) return fail("n_media out of range");
    for (int d = 0; d < sc->n_dyes; ++d) {
        const orc_dye* dy = &sc->dyes[d];
        if (check_spectrum(&dy->absorption, 0, sc->n_bins) || check_spectrum(&dy->emission, 0, sc->n_bins))
            return -1;
        if (!(dy->qy >= 0.0 && dy->qy <= 1.0)) return fail("qy outside [0,1]");
        if (!(dy->epsilon >= 0.0) || !isfinite(dy->epsilon)) return fail("epsilon < 0");
    }
    for (int m = 0; m < sc->n_media; ++m) {
        const orc_medium* md = &sc->media[m];
        if (!(md->sigma_s >= 0.0) || !isfinite(md->sigma_s)) return fail("sigma_s < 0");
        if (!(md->sigma_a_bg >= 0.0) || !isfinite(md->sigma_a_bg)) return fail("sigma_a_bg < 0");
        if (md->n_dyes < 0 || md->n_dyes > ORC_MAX_MEDIUM_DYES) return fail("medium dyes");
        for (int j = 0; j < md->n_dyes; ++j) {
            if (md->dye[j] < 0 || md->dye[j] >= sc->n_dyes) return fail("dye index");
            if (!(md->conc[j] >= 0.0) || !isfinite(md->conc[j])) return fail("conc < 0");
        }
    }
    if (sc->n_lines < 1 || sc->n_lines > ORC_MAX_LINES) return fail("n_lines out of range");
    double tot = 0.0;
    for (int i = 0; i < sc->n_lines; ++i) {
        if (!(sc->line_power[i] >= 0.0)) return fail("line power < 0");
        tot += sc->line_power[i];
    }
    if (!(tot > 0.0)) return fail("total light power is 0");
    if (sc->geom == ORC_GEOM_BOX) {
        if (sc->light != ORC_LIGHT_QUAD) return fail("box scenes need a quad light");
        for (int f = 0; f < 6; ++f) {
            if (f != sc->open_face && check_spectrum(&sc->walls[f], 0, sc->n_bins)) return -1;
            if (!(sc->wall_gloss[f] >= 0.0 && sc->wall_gloss[f] <= 1e4)) return fail("wall gloss outside [0, 1e4]");
            if (sc->wall_gloss[f] > 0.0 && sc->sensor != ORC_SENSOR_PINHOLE)
                return fail("glossy walls need a pinhole sensor");
        }
        if (sc->n_spheres < 0 || sc->n_spheres > ORC_MAX_SPHERES) return fail("n_spheres");
        for (int s = 0; s < sc->n_spheres; ++s) {
            const orc_sphere* sp = &sc->spheres[s];
            if (sp->medium < 0 || sp->medium >= sc->n_media) return fail("sphere medium");
            if (!(sp->radius > 0.0)) return fail("sphere radius");
        }
    } else {
        for (int f = 0; f < 6; ++f)
            if (sc->wall_gloss[f] != 0.0) return fail("glossy walls need a box scene");
        if (sc->body_medium < 0 || sc->body_medium >= sc->n_media) return fail("body medium");
        if (sc->sensor != ORC_SENSOR_ESCAPE) return fail("pinhole needs a box scene");
        if (sc->light == ORC_LIGHT_QUAD) return fail("quad light needs a box scene");
    }
    return 0;
}

static int build_tables(const orc_scene* sc, tables_t* t) {
    memset(t, 0, sizeof *t);
    if (validate(sc)) return -1;
    int N = sc->n_bins;
    t->N = N;
    t->lo = sc->lo_nm;
    t->delta = (sc->hi_nm - sc->lo_nm) / (double)(N - 1);
    t->lambda = calloc((size_t)N, sizeof(double));
    t->a_hat = calloc((size_t)(ORC_MAX_DYES * N), sizeof(double));
    t->pmf = calloc((size_t)(ORC_MAX_DYES * N), sizeof(double));
    t->cdf = calloc((size_t)(ORC_MAX_DYES * N), sizeof(double));
    t->sigma_t = calloc((size_t)(ORC_MAX_MEDIA * N), sizeof(double));
    t->sigma_a = calloc((size_t)(ORC_MAX_MEDIA * ORC_MAX_MEDIUM_DYES * N), sizeof(double));
    t->kappa = calloc((size_t)(ORC_MAX_MEDIA * ORC_MAX_MEDIUM_DYES * N), sizeof(double));
    t->rho = calloc((size_t)(6 * N), sizeof(double));
    if (!t->lambda || !t->a_hat || !t->pmf || !t->cdf || !t->sigma_t || !t->sigma_a ||
        !t->kappa || !t->rho) {
        free_tables(t);
        return fail("out of memory");
    }
    for (int k = 0; k < N; ++k) t->lambda[k] = sc->lo_nm + t->delta * (double)k;

    for (int d = 0; d < sc->n_dyes; ++d) {
        const orc_dye* dy = &sc->dyes[d];
        double amax = 0.0, esum = 0.0;
        for (int k = 0; k < N; ++k) {
            double a = eval_spectrum(&dy->absorption, t->lambda[k], k);
            double e = eval_spectrum(&dy->emission, t->lambda[k], k);
            if (a < 0.0 || e < 0.0) { free_tables(t); return fail("negative spectrum value"); }
            t->a_hat[d * N + k] = a;
            t->pmf[d * N + k] = e;
            if (a > amax) amax = a;
            esum += e;
        }
        if (!(amax > 0.0) || !(esum > 0.0)) { free_tables(t); return fail("empty dye spectrum"); }
        double c = 0.0;
        for (int k = 0; k < N; ++k) {
            t->a_hat[d * N + k] /= amax;   /* peak-normalised: epsilon is the peak value */
            t->pmf[d * N + k] /= esum;     /* eq. 10: f_m / integral f_m, one-bin step */
            c += t->pmf[d * N + k];
            t->cdf[d * N + k] = c;
        }
        t->cdf[d * N + N - 1] = 1.0;
    }

    /* sigma_a,d = base * epsilon [1/(M cm)] * c [uM] * 1e-6 [M/uM] * 0.1 [cm/mm] * a_hat */
    double base = sc->natural_base ? 1.0 : log(10.0);
    for (int m = 0; m < sc->n_media; ++m) {
        const orc_medium* md = &sc->media[m];
        for (int k = 0; k < N; ++k) {
            double st = md->sigma_s + md->sigma_a_bg; /* eq. 6: sigma_t = sigma_a + sigma_s */
            for (int j = 0; j < md->n_dyes; ++j) {
                const orc_dye* dy = &sc->dyes[md->dye[j]];
                double kap = base * dy->epsilon * 1e-7 * t->a_hat[md->dye[j] * N + k];
                double sa = kap * md->conc[j];
                t->kappa[(m * ORC_MAX_MEDIUM_DYES + j) * N + k] = kap;
                t->sigma_a[(m * ORC_MAX_MEDIUM_DYES + j) * N + k] = sa;
                st += sa;
            }
            t->sigma_t[m * N + k] = st;
        }
    }
    if (sc->geom == ORC_GEOM_BOX) {
        for (int f = 0; f < 6; ++f) {
            for (int k = 0; k < N; ++k) {
                double r = (f == sc->open_face) ? 0.0 : eval_spectrum(&sc->walls[f], t->lambda[k], k);
                if (!(r >= 0.0 && r <= 1.0)) { free_tables(t); return fail("wall rho outside [0,1]"); }
                t->rho[f * N + k] = r;
            }
        }
    }
    double tot = 0.0;
    for (int i = 0; i < sc->n_lines; ++i) tot += sc->line_power[i];
    double c = 0.0;
    for (int i = 0; i < sc->n_lines; ++i) {
        t->line_bin[i] = line_bin_of(sc->line_nm[i], sc->lo_nm, t->delta, N);
        if (t->line_bin[i] < 0) { free_tables(t); return fail("light line off the grid"); }
        c += sc->line_power[i] / tot;
        t->line_cum[i] = c;
    }
    t->line_cum[sc->n_lines - 1] = 1.0;
    return 0;
}

int32_t orc_tables(const orc_scene* sc, double* lambda, double* a_hat, double* emis_pmf,
                   double* emis_cdf, double* sigma_t, double* sigma_a, double* rho,
                   int32_t* line_bin) {
    tables_t t;
    if (build_tables(sc, &t)) return -1;
    int N = t.N;
    if (lambda) memcpy(lambda, t.lambda, sizeof(double) * (size_t)N);
    if (a_hat) memcpy(a_hat, t.a_hat, sizeof(double) * (size_t)(sc->n_dyes * N));
    if (emis_pmf) memcpy(emis_pmf, t.pmf, sizeof(double) * (size_t)(sc->n_dyes * N));
    if (emis_cdf) memcpy(emis_cdf, t.cdf, sizeof(double) * (size_t)(sc->n_dyes * N));
    if (sigma_t) memcpy(sigma_t, t.sigma_t, sizeof(double) * (size_t)(sc->n_media * N));
    if (sigma_a)
        memcpy(sigma_a, t.sigma_a,
               sizeof(double) * (size_t)(sc->n_media * ORC_MAX_MEDIUM_DYES * N));
    if (rho) memcpy(rho, t.rho, sizeof(double) * (size_t)(6 * N));
    if (line_bin)
        for (int i = 0; i < sc->n_lines; ++i) line_bin[i] = t.line_bin[i];
    free_tables(&t);
    return 0;
}

int64_t orc_film_size(const orc_scene* sc, uint32_t batches) {
    int64_t B = batches ? batches : 1;
    if (sc->sensor == ORC_SENSOR_PINHOLE)
        return B * 2 * (int64_t)sc->height * sc->width * sc->n_bins;
    return B * 2 * 2 * (int64_t)sc->n_bins;
}

int32_t orc_n_params(const orc_scene* sc) {
    int n = sc->n_dyes + sc->n_media;
    for (int m = 0; m < sc->n_media; ++m) n += sc->media[m].n_dyes;
    return n;
}

/* ------------------------------------------------------------------------- */
/* Vector helpers. */
static double dot3(const double* a, const double* b) { return a[0] * b[0] + a[1] * b[1] + a[2] * b[2]; }
static void cross3(const double* a, const double* b, double* o) {
    o[0] = a[1] * b[2] - a[2] * b[1];
    o[1] = a[2] * b[0] - a[0] * b[2];
    o[2] = a[0] * b[1] - a[1] * b[0];
}
static void normalize3(double* a) {
    double l = sqrt(dot3(a, a));
    a[0] /= l; a[1] /= l; a[2] /= l;
}

/* Isotropic direction (sec. 2.1: emission and scattering are isotropic). */
static void iso_dir(double ua, double ub, double* w) {
    double ct = 1.0 - 2.0 * ua;
    double st = sqrt(fmax(0.0, 1.0 - ct * ct));
    double ph = 2.0 * M_PI * ub;
    w[0] = st * cos(ph);
    w[1] = st * sin(ph);
    w[2] = ct;
}

/* Cosine-weighted direction about normal n with tangent t1 (Lambertian). */
static void cos_dir(const double* n, const double* t1, double ua, double ub, double* w) {
    double t2[3];
    cross3(n, t1, t2);
    double r = sqrt(ua), ph = 2.0 * M_PI * ub;
    double lx = r * cos(ph), ly = r * sin(ph), lz = sqrt(fmax(0.0, 1.0 - ua));
    for (int i = 0; i < 3; ++i) w[i] = lx * t1[i] + ly * t2[i] + lz * n[i];
}

/* Glossy walls: the normalised modified-Phong lobe (a cosine power about the
 * mirror direction, normalised by (n+2)/(2 pi) so that at normal incidence all
 * of the reflected energy rho leaves the wall; reciprocal in wi and wo). */
static void mirror_dir(const double* wi, const double* nrm, double* r) {
    double d = 2.0 * dot3(wi, nrm);
    for (int i = 0; i < 3; ++i) r[i] = wi[i] - d * nrm[i];
}

double orc_phong_eval(double n, const double* wi, const double* wo, const double* nrm) {
    if (!(dot3(wi, nrm) < 0.0) || !(dot3(wo, nrm) > 0.0)) return 0.0;
    double r[3];
    mirror_dir(wi, nrm, r);
    double c = dot3(r, wo);
    if (!(c > 0.0)) return 0.0;
    return (n + 2.0) / (2.0 * M_PI) * pow(c, n);
}

/* Orthonormal basis (t1, t2) completing unit r (Duff et al., "Building an
 * Orthonormal Basis, Revisited", JCGT 2017). */
static void basis_about(const double* r, double* t1, double* t2) {
    double sg = r[2] >= 0.0 ? 1.0 : -1.0;
    double a = -1.0 / (sg + r[2]);
    double b = r[0] * r[1] * a;
    t1[0] = 1.0 + sg * r[0] * r[0] * a;
    t1[1] = sg * b;
    t1[2] = -sg * r[0];
    t2[0] = b;
    t2[1] = sg + r[1] * r[1] * a;
    t2[2] = -r[1];
}

double orc_phong_sample(double n, const double* wi, const double* nrm, double ua, double ub,
                        double* wo) {
    double r[3], t1[3], t2[3];
    mirror_dir(wi, nrm, r);
    basis_about(r, t1, t2);
    double ca = pow(ua, 1.0 / (n + 1.0));
    double sa = sqrt(fmax(0.0, 1.0 - ca * ca));
    double ph = 2.0 * M_PI * ub;
    for (int i = 0; i < 3; ++i) wo[i] = sa * cos(ph) * t1[i] + sa * sin(ph) * t2[i] + ca * r[i];
    double co = dot3(wo, nrm);
    return co > 0.0 ? (n + 2.0) / (n + 1.0) * co : 0.0;
}

/* Inward normal and tangent of box face f (0 x=lo, 1 x=hi, 2 y=lo, ...). */
static void face_frame(int f, double* n, double* t1) {
    int a = f / 2;
    n[0] = n[1] = n[2] = 0.0;
    t1[0] = t1[1] = t1[2] = 0.0;
    n[a] = (f % 2 == 0) ? 1.0 : -1.0;
    t1[(a + 1) % 3] = 1.0;
}

/* ------------------------------------------------------------------------- */
/* Geometry: distance to the next surface along the ray. */
enum { SURF_NONE = 0, SURF_ESCAPE, SURF_WALL, SURF_LIGHT, SURF_ENTER, SURF_EXIT };

typedef struct {
    double d;
    int kind;
    int index; /* wall face or sphere */
    double margin;
} hit_t;

static void upd_margin(double* m, double v) { if (v < *m) *m = v; }

/* skip_light: the ray starts on the light quad and leaves it (a plane is not
 * hit twice by one straight segment). */
static hit_t next_surface(const orc_scene* sc, const double* x, const double* w, int region,
                          int skip_light) {
    hit_t h = {INFINITY, SURF_ESCAPE, -1, INFINITY};
    switch (sc->geom) {
    case ORC_GEOM_SLAB:
        if (w[2] > 0.0) h.d = (sc->z1 - x[2]) / w[2];
        else if (w[2] < 0.0) h.d = (sc->z0 - x[2]) / w[2];
        if (h.d < 0.0) h.d = 0.0;
        return h;
    case ORC_GEOM_HALFSPACE:
        if (w[2] < 0.0) h.d = fmax(0.0, (sc->z0 - x[2]) / w[2]);
        return h;
    case ORC_GEOM_SPHERE: {
        double oc[3] = {x[0] - sc->center[0], x[1] - sc->center[1], x[2] - sc->center[2]};
        double b = dot3(oc, w), c = dot3(oc, oc) - sc->radius * sc->radius;
        double disc = b * b - c;
        h.d = fmax(0.0, -b + sqrt(fmax(disc, 0.0)));
        return h;
    }
    case ORC_GEOM_INFINITE:
        return h;
    default:
        break;
    }
    /* box scene */
    if (region >= 0) {
        const orc_sphere* sp = &sc->spheres[region];
        double oc[3] = {x[0] - sp->center[0], x[1] - sp->center[1], x[2] - sp->center[2]};
        double b = dot3(oc, w), c = dot3(oc, oc) - sp->radius * sp->radius;
        double disc = b * b - c;
        h.d = fmax(0.0, -b + sqrt(fmax(disc, 0.0)));
        h.kind = SURF_EXIT;
        h.index = region;
        return h;
    }
    /* vacuum inside the box: walls, light quad, sphere entries */
    for (int a = 0; a < 3; ++a) {
        double t;
        int f;
        if (w[a] > 0.0) { t = (sc->box_hi[a] - x[a]) / w[a]; f = 2 * a + 1; }
        else if (w[a] < 0.0) { t = (sc->box_lo[a] - x[a]) / w[a]; f = 2 * a; }
        else continue;
        if (t < 0.0) t = 0.0;
        if (t < h.d) { h.d = t; h.index = f; }
    }
    h.kind = (h.index == sc->open_face) ? SURF_ESCAPE : SURF_WALL;
    if (!skip_light) {
        double n[3];
        cross3(sc->lu, sc->lv, n);
        normalize3(n);
        double dn = dot3(n, w);
        if (dn != 0.0) {
            double pc[3] = {sc->lpos[0] - x[0], sc->lpos[1] - x[1], sc->lpos[2] - x[2]};
            double t = dot3(n, pc) / dn;
            if (t > 0.0 && t < h.d) {
                double q[3] = {x[0] + t * w[0] - sc->lpos[0], x[1] + t * w[1] - sc->lpos[1],
                               x[2] + t * w[2] - sc->lpos[2]};
                double a = dot3(q, sc->lu) / dot3(sc->lu, sc->lu);
                double b = dot3(q, sc->lv) / dot3(sc->lv, sc->lv);
                if (a >= 0.0 && a <= 1.0 && b >= 0.0 && b <= 1.0) {
                    h.d = t;
                    h.kind = SURF_LIGHT;
                    h.index = -1;
                }
                upd_margin(&h.margin, fmin(fmin(fabs(a), fabs(1.0 - a)), fmin(fabs(b), fabs(1.0 - b))));
            }
        }
    }
    for (int s = 0; s < sc->n_spheres; ++s) {
        const orc_sphere* sp = &sc->spheres[s];
        double oc[3] = {x[0] - sp->center[0], x[1] - sp->center[1], x[2] - sp->center[2]};
        double b = dot3(oc, w);
        if (!(b < 0.0)) continue;
        double c = dot3(oc, oc) - sp->radius * sp->radius;
        double disc = b * b - c;
        upd_margin(&h.margin, fabs(disc) / (sp->radius * sp->radius));
        if (!(disc > 0.0)) continue;
        double t = -b - sqrt(disc);
        if (t < 0.0) t = 0.0;
        if (t < h.d) { h.d = t; h.kind = SURF_ENTER; h.index = s; }
    }
    return h;
}

/* Length of segment [0, len] of ray (x, w) inside a sphere. */
static double chord(const double* x, const double* w, double len, const orc_sphere* sp,
                    double* margin) {
    double oc[3] = {x[0] - sp->center[0], x[1] - sp->center[1], x[2] - sp->center[2]};
    double b = dot3(oc, w), c = dot3(oc, oc) - sp->radius * sp->radius;
    double disc = b * b - c;
    if (margin && c > 0.0) upd_margin(margin, fabs(disc) / (sp->radius * sp->radius));
    if (!(disc > 0.0)) return 0.0;
    double sq = sqrt(disc);
    double t0 = -b - sq, t1 = -b + sq;
    double lo = t0 > 0.0 ? t0 : 0.0, hi = t1 < len ? t1 : len;
    return hi > lo ? hi - lo : 0.0;
}

/* ------------------------------------------------------------------------- */
/* The walk. */

typedef struct {
    const orc_scene* sc;
    const orc_run* run;
    const tables_t* t;
    double* film;
    const double* gfilm;
    double* grad;     /* accumulated gradient of <gfilm, film> */
    double* pgrad;    /* this path's gradient (records) */
    int n_params;
    int param_c[ORC_MAX_MEDIA][ORC_MAX_MEDIUM_DYES];
    int param_qy[ORC_MAX_DYES];
    int param_ss[ORC_MAX_MEDIA];
    /* camera */
    double cf[3], cr[3], cu[3], tanx, tany, area_img;
    double qn[3], qt1[3];
    double wscale;
    uint64_t* tally;
} ctx_t;

typedef struct {
    double x[3], w[3];
    int lam, region, medium, comp;
    uint32_t n_scatter, n_emit, v;
    uint32_t batch;
    uint32_t pid;
    double S[ORC_MAX_PARAMS]; /* running score: d/dtheta log p(path prefix) */
    double weight;            /* throughput weight (glossy reflections; 1 otherwise) */
    double splat_sum;
    double margin;
} path_t;

/* Conditioning probe (orc_run.perturb_eta): scale each entry of a freshly
 * computed vector -- a position (slot 0), a direction (slot 1), the running
 * score (slot 2), the path's gradient sum (slot 3) or a point drawn on the
 * light for a connection (slot 4) -- by 1 +- eta, the sign
 * from a 64-bit mix (splitmix64 finaliser) of path, vertex, slot, entry and
 * pattern.  No effect when eta is 0. */
static void perturb_vec(const ctx_t* c, const path_t* p, int slot, double* a, int n) {
    double eta = c->run->perturb_eta;
    if (!(eta > 0.0)) return;
    for (int i = 0; i < n; ++i) {
        uint64_t z = ((uint64_t)p->pid << 32) ^ ((uint64_t)p->v << 10) ^ (uint64_t)(slot * 32 + i) ^
                     ((uint64_t)c->run->perturb_pattern << 56);
        z += 0x9E3779B97F4A7C15ull;
        z = (z ^ (z >> 30)) * 0xBF58476D1CE4E5B9ull;
        z = (z ^ (z >> 27)) * 0x94D049BB133111EBull;
        z ^= z >> 31;
        a[i] *= (z & 1u) ? 1.0 + eta : 1.0 - eta;
    }
}
static void perturb3(const ctx_t* c, const path_t* p, int slot, double* a) {
    perturb_vec(c, p, slot, a, 3);
}

static void deposit(ctx_t* c, path_t* p, int64_t idx, double v, const double* dv) {
    c->film[idx] += v;
    p->splat_sum += v;
    if (c->gfilm) {
        double g = c->gfilm[idx];
        for (int i = 0; i < c->n_params; ++i) {
            double gi = g * (v * p->S[i] + (dv ? dv[i] : 0.0));
            c->grad[i] += gi;
            if (c->pgrad) c->pgrad[i] += gi;
        }
        if (c->pgrad) perturb_vec(c, p, 3, c->pgrad, c->n_params);
    }
}

/* Escape tally: film[b][comp][side][lambda] += B / total_paths. */
static void tally_escape(ctx_t* c, path_t* p, int side) {
    int N = c->t->N;
    if (c->sc->sensor != ORC_SENSOR_ESCAPE) return;
    int64_t idx = (((int64_t)p->batch * 2 + p->comp) * 2 + side) * N + p->lam;
    if (c->run->fluorescence_only && p->comp == 0) return;
    if (c->film) deposit(c, p, idx, c->wscale, NULL);
}

/* Pinhole splat at a realised vertex (eqs. 3-6): value
 *   (power/paths) * f * T_r * W_e / r^2,  W_e = N_pix / (A_img cos^3 theta)
 * so that a uniform radiance L reads L in every pixel.
 * f = 1/(4 pi) in a medium, cos/pi on a Lambertian surface. */
static void splat(ctx_t* c, path_t* p, const double* nrm, int is_light_vertex, uint32_t rr_bits,
                  const double* gloss_wi, double gloss_n) {
    const orc_scene* sc = c->sc;
    if (sc->sensor != ORC_SENSOR_PINHOLE) return;
    if (c->run->fluorescence_only && p->comp == 0) return;
    uint64_t* T = c->tally;
    double d[3] = {sc->eye[0] - p->x[0], sc->eye[1] - p->x[1], sc->eye[2] - p->x[2]};
    double dist = sqrt(dot3(d, d));
    double wc[3] = {d[0] / dist, d[1] / dist, d[2] / dist};
    double f;
    if (nrm) {
        double cs = dot3(nrm, wc);
        upd_margin(&p->margin, fabs(cs));
        if (!(cs > 0.0)) { T[ORC_T_SPLAT_MISS]++; return; }
        /* BRDF over rho (the path survived the reflection with probability
         * rho) times the cosine toward the eye */
        f = gloss_wi ? orc_phong_eval(gloss_n, gloss_wi, wc, nrm) * cs : cs / M_PI;
    } else {
        f = 1.0 / (4.0 * M_PI);
    }
    double pv[3] = {-d[0], -d[1], -d[2]};
    double zc = dot3(pv, c->cf);
    if (!(zc > 0.0)) { T[ORC_T_SPLAT_MISS]++; return; }
    double xi = dot3(pv, c->cr) / zc / c->tanx; /* [-1, 1] across the image */
    double yi = dot3(pv, c->cu) / zc / c->tany;
    upd_margin(&p->margin, fmin(fabs(1.0 - fabs(xi)), fabs(1.0 - fabs(yi))));
    double fx = (xi + 1.0) * 0.5 * sc->width;
    double fy = (1.0 - yi) * 0.5 * sc->height;
    if (!(fx >= 0.0 && fx < sc->width && fy >= 0.0 && fy < sc->height)) {
        T[ORC_T_SPLAT_MISS]++;
        return;
    }
    int px = (int)floor(fx), py = (int)floor(fy);
    /* visibility: the segment must leave the box through the open face */
    {
        double tmin = INFINITY;
        int fmin_ = -1;
        for (int a = 0; a < 3; ++a) {
            double t;
            int fc;
            if (d[a] > 0.0) { t = (sc->box_hi[a] - p->x[a]) / d[a]; fc = 2 * a + 1; }
            else if (d[a] < 0.0) { t = (sc->box_lo[a] - p->x[a]) / d[a]; fc = 2 * a; }
            else continue;
            if (t < tmin) { tmin = t; fmin_ = fc; }
        }
        /* margin: distance of the open-face plane crossing to that face's edges */
        {
            int a = sc->open_face / 2;
            double plane = (sc->open_face % 2) ? sc->box_hi[a] : sc->box_lo[a];
            double tf = d[a] != 0.0 ? (plane - p->x[a]) / d[a] : INFINITY;
            if (isfinite(tf) && tf > 0.0) {
                for (int b = 0; b < 3; ++b) {
                    if (b == a) continue;
                    double q = p->x[b] + tf * d[b];
                    double ext = sc->box_hi[b] - sc->box_lo[b];
                    upd_margin(&p->margin,
                               fmin(fabs(q - sc->box_lo[b]), fabs(sc->box_hi[b] - q)) / ext);
                }
            }
        }
        if (fmin_ != sc->open_face || !(tmin < 1.0)) { T[ORC_T_SPLAT_MISS]++; return; }
    }
    if (!is_light_vertex) {
        /* the light quad occludes */
        double dn = dot3(c->qn, d);
        if (dn != 0.0) {
            double pc[3] = {sc->lpos[0] - p->x[0], sc->lpos[1] - p->x[1], sc->lpos[2] - p->x[2]};
            double t = dot3(c->qn, pc) / dn;
            if (t > 0.0 && t < 1.0) {
                double q[3] = {p->x[0] + t * d[0] - sc->lpos[0], p->x[1] + t * d[1] - sc->lpos[1],
                               p->x[2] + t * d[2] - sc->lpos[2]};
                double a = dot3(q, sc->lu) / dot3(sc->lu, sc->lu);
                double b = dot3(q, sc->lv) / dot3(sc->lv, sc->lv);
                upd_margin(&p->margin, fmin(fmin(fabs(a), fabs(1.0 - a)), fmin(fabs(b), fabs(1.0 - b))));
                if (a >= 0.0 && a <= 1.0 && b >= 0.0 && b <= 1.0) { T[ORC_T_SPLAT_MISS]++; return; }
            }
        }
    }
    /* transmittance along the connection (eq. 6), through every sphere */
    double len[ORC_MAX_SPHERES];
    double tau = 0.0;
    for (int s = 0; s < sc->n_spheres; ++s) {
        len[s] = chord(p->x, wc, dist, &sc->spheres[s], &p->margin);
        tau += c->t->sigma_t[sc->spheres[s].medium * c->t->N + p->lam] * len[s];
    }
    double tr = exp(-tau);
    double cosc = zc / dist;
    double npix = (double)sc->width * (double)sc->height;
    double v = c->wscale * f * tr * npix / (c->area_img * cosc * cosc * cosc * dist * dist) * p->weight;
    double rr = c->run->splat_rr;
    if (rr > 0.0 && tr < rr) {
        double u = (double)rr_bits * (1.0 / 16777216.0);
        double q = tr / rr;
        upd_margin(&p->margin, fabs(u - q));
        if (!(u < q)) { T[ORC_T_SPLAT_RR_KILL]++; return; }
        v = v / q;
    }
    T[ORC_T_SPLAT_HIT]++;
    int N = c->t->N;
    int64_t idx = ((((int64_t)p->batch * 2 + p->comp) * sc->height + py) * sc->width + px) * N + p->lam;
    double dv[ORC_MAX_PARAMS];
    if (c->gfilm) {
        /* d v / d theta = -v * sum_s d sigma_t / d theta * chord_s */
        for (int i = 0; i < c->n_params; ++i) dv[i] = 0.0;
        for (int s = 0; s < sc->n_spheres; ++s) {
            int m = sc->spheres[s].medium;
            if (len[s] <= 0.0) continue;
            dv[c->param_ss[m]] -= v * len[s];
            for (int j = 0; j < sc->media[m].n_dyes; ++j)
                dv[c->param_c[m][j]] -=
                    v * c->t->kappa[(m * ORC_MAX_MEDIUM_DYES + j) * N + p->lam] * len[s];
        }
    }
    if (c->film) deposit(c, p, idx, v, c->gfilm ? dv : NULL);
}

/* d sigma_t / d theta applied as S -= d sigma_t * length. */
static void score_path_length(ctx_t* c, path_t* p, double len) {
    if (!c->gfilm || p->medium < 0) return;
    int m = p->medium, N = c->t->N;
    p->S[c->param_ss[m]] -= len;
    for (int j = 0; j < c->sc->media[m].n_dyes; ++j)
        p->S[c->param_c[m][j]] -= c->t->kappa[(m * ORC_MAX_MEDIUM_DYES + j) * N + p->lam] * len;
}

static uint32_t rr_bits_of(const uint32_t r[4]) {
    return ((r[0] & 0xFFu) << 16) | ((r[1] & 0xFFu) << 8) | (r[2] & 0xFFu);
}

/* ------------------------------------------------------------------------- */
/* Smooth dielectric boundary of a body medium (glass beads and vials, sec. 5:
 * refractive media; textbook Fresnel equations and Snell's law). */

/* Refractive index of the body medium (1 when index-matched or in a box). */
static double body_ior(const orc_scene* sc) {
    if (sc->geom == ORC_GEOM_BOX || sc->geom == ORC_GEOM_INFINITE) return 1.0;
    double n = sc->media[sc->body_medium].ior;
    return n > 0.0 ? n : 1.0;
}

/* Unpolarised reflectance (mean of the s and p intensities) for light going
 * from index n1 into index n2 with incidence cosine ci > 0; 1 beyond the
 * critical angle.  *ct receives the transmitted cosine (0 on total internal
 * reflection). */
static double fresnel(double ci, double n1, double n2, double* ct) {
    double eta = n1 / n2;
    double st2 = eta * eta * (1.0 - ci * ci);
    if (st2 >= 1.0) { *ct = 0.0; return 1.0; }
    double c2 = sqrt(1.0 - st2);
    double rs = (n1 * ci - n2 * c2) / (n1 * ci + n2 * c2);
    double rp = (n1 * c2 - n2 * ci) / (n1 * c2 + n2 * ci);
    *ct = c2;
    return 0.5 * (rs * rs + rp * rp);
}

/* Outward unit normal of the body's boundary at x, for a path moving along w
 * (slab: the face it is heading for). */
static void body_normal(const orc_scene* sc, const double* x, const double* w, double* nrm) {
    nrm[0] = nrm[1] = nrm[2] = 0.0;
    if (sc->geom == ORC_GEOM_SLAB) nrm[2] = w[2] > 0.0 ? 1.0 : -1.0;
    else if (sc->geom == ORC_GEOM_HALFSPACE) nrm[2] = -1.0;
    else {
        for (int i = 0; i < 3; ++i) nrm[i] = x[i] - sc->center[i];
        normalize3(nrm);
    }
}

static void mirror(double* w, const double* nrm) {
    double d = 2.0 * dot3(w, nrm);
    for (int i = 0; i < 3; ++i) w[i] -= d * nrm[i];
}

static int region_medium(const orc_scene* sc, int region) {
    if (sc->geom == ORC_GEOM_BOX) return region >= 0 ? sc->spheres[region].medium : -1;
    return sc->body_medium;
}

static double scene_scale(const orc_scene* sc) {
    switch (sc->geom) {
    case ORC_GEOM_SLAB: return fmax(sc->z1 - sc->z0, 1e-3);
    case ORC_GEOM_SPHERE: return sc->radius;
    case ORC_GEOM_BOX: return 0.5 * (sc->box_hi[0] - sc->box_lo[0]);
    default: return 1.0;
    }
}

static void run_path(ctx_t* c, uint32_t pid, orc_record* rec, uint32_t max_vertices) {
    const orc_scene* sc = c->sc;
    const tables_t* t = c->t;
    const orc_run* run = c->run;
    uint64_t* T = c->tally;
    int N = t->N;
    rng_t rng;
    rng.key[0] = (uint32_t)run->seed;
    rng.key[1] = (uint32_t)(run->seed >> 32) ^ run->instance;
    rng.pid = pid;
    path_t p;
    memset(&p, 0, sizeof p);
    p.pid = pid;
    p.weight = 1.0;
    p.batch = pid % (run->parity_batches ? run->parity_batches : 1);
    p.margin = INFINITY;
    double L = scene_scale(sc);
    int exit_code = -1;
    uint32_t r[4], r1[4];

    /* vertex 0: the light (eq. 12: light point and excitation wavelength sampled) */
    draw(&rng, 0, 0, r);
    double u = unif(r[0]);
    int line = 0;
    while (line < sc->n_lines - 1 && !(u < t->line_cum[line])) ++line;
    for (int i = 0; i < sc->n_lines - 1; ++i) upd_margin(&p.margin, fabs(u - t->line_cum[i]));
    p.lam = t->line_bin[line];
    double n_b = body_ior(sc);
    if (sc->light == ORC_LIGHT_BEAM) {
        memcpy(p.x, sc->lpos, sizeof p.x);
        memcpy(p.w, sc->ldir, sizeof p.w);
        normalize3(p.w);
        p.region = 0;
        if (n_b != 1.0) {
            /* entering a refractive body: Fresnel reflection (the path leaves at
             * once) or refraction, with uniform 1 of the light vertex */
            double nrm[3], ct;
            double ws[3] = {-p.w[0], -p.w[1], -p.w[2]};
            body_normal(sc, p.x, ws, nrm);
            double ci = -dot3(p.w, nrm);
            double R = fresnel(ci, 1.0, n_b, &ct);
            double ur = unif(r[1]);
            upd_margin(&p.margin, fabs(ur - R));
            if (ur < R) {
                mirror(p.w, nrm);
                T[ORC_T_WALL_REFLECT]++;
                exit_code = -2;
            } else {
                double eta = 1.0 / n_b;
                for (int i = 0; i < 3; ++i) p.w[i] = eta * p.w[i] + (eta * ci - ct) * nrm[i];
                normalize3(p.w);
                perturb3(c, &p, 1, p.w);
            }
        }
    } else if (sc->light == ORC_LIGHT_POINT) {
        draw(&rng, 0, 1, r1);
        memcpy(p.x, sc->lpos, sizeof p.x);
        iso_dir(unif(r1[0]), unif(r1[1]), p.w);
        perturb3(c, &p, 1, p.w);
        p.region = 0;
    } else {
        double a = unif(r[1]), b = unif(r[2]);
        for (int i = 0; i < 3; ++i) p.x[i] = sc->lpos[i] + a * sc->lu[i] + b * sc->lv[i];
        perturb3(c, &p, 0, p.x);
        draw(&rng, 0, 1, r1);
        cos_dir(c->qn, c->qt1, unif(r1[0]), unif(r1[1]), p.w);
        perturb3(c, &p, 1, p.w);
        p.region = -1;
    }
    p.medium = region_medium(sc, p.region);
    T[ORC_T_PATHS]++;
    T[ORC_T_VERTICES]++;
    if (sc->light == ORC_LIGHT_QUAD) splat(c, &p, c->qn, 1, rr_bits_of(r), NULL, 0.0);
    if (exit_code == -2) {
        /* reflected off the body on entry: escapes from the light vertex */
        int side = p.w[2] < 0.0 ? 0 : 1;
        upd_margin(&p.margin, fabs(p.w[2]));
        tally_escape(c, &p, side);
        exit_code = side == 0 ? ORC_EXIT_ESC_R : ORC_EXIT_ESC_T;
    }

    while (exit_code < 0) {
        p.v++;
        if (max_vertices && p.v >= max_vertices) { exit_code = ORC_EXIT_TRUNC; break; }
        /* hard bound on path length: 2^28 vertices, counted as a scatter-cap exit */
        if (p.v >= (1u << 28)) { exit_code = ORC_EXIT_SCAP; break; }
        T[ORC_T_VERTICES]++;
        draw(&rng, p.v, 0, r);
        double u0 = unif(r[0]), u1 = unif(r[1]), u2 = unif(r[2]), u3 = unif(r[3]);
        double st = p.medium >= 0 ? t->sigma_t[p.medium * N + p.lam] : 0.0;
        /* eq. 6: free flight distance with density sigma_t exp(-sigma_t t) */
        double tf = st > 0.0 ? -log(1.0 - u0) / st : INFINITY;
        hit_t h = next_surface(sc, p.x, p.w, p.region,
                               sc->light == ORC_LIGHT_QUAD && p.v == 1);
        upd_margin(&p.margin, h.margin);
        if (isfinite(tf) && isfinite(h.d))
            upd_margin(&p.margin, fabs(tf - h.d) / fmax(fmax(tf, h.d), L));
        if (tf < h.d) {
            /* collision inside the medium */
            for (int i = 0; i < 3; ++i) p.x[i] += tf * p.w[i];
            perturb3(c, &p, 0, p.x);
            score_path_length(c, &p, tf);
            if (c->gfilm) perturb_vec(c, &p, 2, p.S, c->n_params);
            const orc_medium* md = &sc->media[p.medium];
            double s = u1 * st;
            double thr = md->sigma_s;
            upd_margin(&p.margin, fabs(s - thr) / st);
            if (s < thr) {
                /* elastic scattering, isotropic phase function (eq. 2) */
                if (c->gfilm) p.S[c->param_ss[p.medium]] += 1.0 / md->sigma_s;
                T[ORC_T_SCATTERS]++;
                p.n_scatter++;
                if (!run->excitation_scatter && p.n_emit == 0) { exit_code = ORC_EXIT_EXCSCAT; break; }
                if (p.n_scatter > run->max_scatter) { exit_code = ORC_EXIT_SCAP; break; }
                iso_dir(u2, u3, p.w);
                perturb3(c, &p, 1, p.w);
                splat(c, &p, NULL, 0, rr_bits_of(r), NULL, 0.0);
                continue;
            }
            thr += md->sigma_a_bg;
            upd_margin(&p.margin, fabs(s - thr) / st);
            if (s < thr || md->n_dyes == 0) { exit_code = ORC_EXIT_BG; break; }
            /* a fluorescent particle: which dye (sec. 4.1) */
            int j = 0;
            for (; j < md->n_dyes - 1; ++j) {
                thr += t->sigma_a[(p.medium * ORC_MAX_MEDIUM_DYES + j) * N + p.lam];
                upd_margin(&p.margin, fabs(s - thr) / st);
                if (s < thr) break;
            }
            int dye = md->dye[j];
            if (c->gfilm) p.S[c->param_c[p.medium][j]] += 1.0 / md->conc[j];
            T[ORC_T_DYE_ABS]++;
            if (p.n_emit >= run->max_emissions) { exit_code = ORC_EXIT_KCAP; break; }
            draw(&rng, p.v, 1, r1);
            double uq = unif(r1[0]);
            double qy = sc->dyes[dye].qy;
            upd_margin(&p.margin, fabs(uq - qy));
            if (!(uq < qy)) {
                if (c->gfilm) p.S[c->param_qy[dye]] -= 1.0 / (1.0 - qy);
                exit_code = ORC_EXIT_NONRAD;
                break;
            }
            if (c->gfilm) p.S[c->param_qy[dye]] += 1.0 / qy;
            /* eq. 10: emitted wavelength from the normalised emission spectrum,
             * independent of the excitation wavelength (sec. 2.1) */
            double ul = unif(r1[1]);
            const double* cdf = &t->cdf[dye * N];
            int k = 0;
            while (k < N - 1 && !(ul < cdf[k])) ++k;
            upd_margin(&p.margin, fabs(ul - cdf[k]));
            if (k > 0) upd_margin(&p.margin, fabs(ul - cdf[k - 1]));
            p.lam = k;
            iso_dir(u2, u3, p.w);
            perturb3(c, &p, 1, p.w);
            p.n_emit++;
            p.comp = 1;
            T[ORC_T_EMISSIONS]++;
            splat(c, &p, NULL, 0, rr_bits_of(r), NULL, 0.0);
            continue;
        }
        /* reached a surface */
        double dd = h.d;
        if (isfinite(dd)) {
            for (int i = 0; i < 3; ++i) p.x[i] += dd * p.w[i];
            perturb3(c, &p, 0, p.x);
            score_path_length(c, &p, dd);
            if (c->gfilm) perturb_vec(c, &p, 2, p.S, c->n_params);
            /* a point on a planar boundary lies exactly on its plane */
            if (sc->geom == ORC_GEOM_SLAB) p.x[2] = p.w[2] < 0.0 ? sc->z0 : sc->z1;
            else if (sc->geom == ORC_GEOM_HALFSPACE) p.x[2] = sc->z0;
            else if (sc->geom == ORC_GEOM_BOX && (h.kind == SURF_WALL || h.kind == SURF_ESCAPE) &&
                     h.index >= 0)
                p.x[h.index / 2] = (h.index % 2) ? sc->box_hi[h.index / 2] : sc->box_lo[h.index / 2];
        }
        if (h.kind == SURF_ESCAPE && n_b != 1.0 && isfinite(dd)) {
            /* the body's dielectric boundary: specular reflection with the
             * Fresnel probability (total internal reflection beyond the critical
             * angle), else the path crosses out; the event uniform decides */
            double nrm[3], ct;
            body_normal(sc, p.x, p.w, nrm);
            double R = fresnel(dot3(p.w, nrm), n_b, 1.0, &ct);
            upd_margin(&p.margin, fabs(u1 - R));
            if (u1 < R) {
                mirror(p.w, nrm);
                perturb3(c, &p, 1, p.w);
                T[ORC_T_WALL_REFLECT]++;
                continue;
            }
        }
        if (h.kind == SURF_ESCAPE) {
            int side = p.w[2] < 0.0 ? 0 : 1;
            upd_margin(&p.margin, fabs(p.w[2]));
            tally_escape(c, &p, side);
            exit_code = side == 0 ? ORC_EXIT_ESC_R : ORC_EXIT_ESC_T;
            break;
        }
        if (h.kind == SURF_LIGHT) { exit_code = ORC_EXIT_LIGHT; break; }
        if (h.kind == SURF_WALL) {
            double rho = t->rho[h.index * N + p.lam];
            upd_margin(&p.margin, fabs(u1 - rho));
            if (!(u1 < rho)) { exit_code = ORC_EXIT_WALL; break; }
            T[ORC_T_WALL_REFLECT]++;
            /* direct excitation only: a wall reflection before the emission is an
             * elastic event at the excitation wavelength like a scatter */
            if (!run->excitation_scatter && p.n_emit == 0) { exit_code = ORC_EXIT_EXCSCAT; break; }
            double n[3], t1[3];
            face_frame(h.index, n, t1);
            double gn = sc->wall_gloss[h.index];
            if (gn > 0.0) {
                /* glossy wall: the realised vertex splats with the lobe about the
                 * mirror of the incoming direction, then the path continues in a
                 * direction drawn from the lobe with its throughput factor, or
                 * ends when that direction falls below the wall */
                double wi[3] = {p.w[0], p.w[1], p.w[2]}, wo[3];
                splat(c, &p, n, 0, rr_bits_of(r), wi, gn);
                double fw = orc_phong_sample(gn, wi, n, u2, u3, wo);
                upd_margin(&p.margin, fabs(dot3(wo, n)));
                if (!(fw > 0.0)) { exit_code = ORC_EXIT_WALL; break; }
                memcpy(p.w, wo, sizeof p.w);
                perturb3(c, &p, 1, p.w);
                p.weight *= fw;
                continue;
            }
            cos_dir(n, t1, u2, u3, p.w);
            perturb3(c, &p, 1, p.w);
            splat(c, &p, n, 0, rr_bits_of(r), NULL, 0.0);
            continue;
        }
        /* index-matched interface: change medium, no deflection */
        T[ORC_T_CROSSINGS]++;
        p.region = (h.kind == SURF_ENTER) ? h.index : -1;
        p.medium = region_medium(sc, p.region);
    }
    T[ORC_T_EXIT0 + exit_code]++;
    if (rec) {
        rec->n_vertices = p.v + (exit_code == ORC_EXIT_TRUNC ? 0u : 1u);
        rec->n_scatter = p.n_scatter;
        rec->n_emit = p.n_emit;
        rec->exit_code = (uint32_t)exit_code;
        rec->lambda = p.lam;
        rec->comp = p.comp;
        rec->region = p.region;
        memcpy(rec->pos, p.x, sizeof p.x);
        memcpy(rec->dir, p.w, sizeof p.w);
        rec->splat_sum = p.splat_sum;
        rec->margin = p.margin;
    }
}

int32_t orc_render(const orc_scene* sc, const orc_run* run, double* film, uint64_t* tallies,
                   const double* gfilm, double* grad, orc_record* rec, double* rec_grad,
                   uint32_t max_vertices) {
    g_err[0] = 0;
    if (!sc || !run) return fail("null argument");
    if (run->total_paths == 0 || run->path_begin + run->path_count > run->total_paths)
        return fail("path range outside total_paths");
    if (run->total_paths > (1ull << 32)) return fail("total_paths exceeds 2^32");
    if (run->path_count > 0xFFFFFFFFull) return fail("path_count must be below 2^32");
    if (gfilm && !grad) return fail("gfilm needs grad");
    if (rec_grad && !gfilm) return fail("rec_grad needs gfilm");
    tables_t t;
    if (build_tables(sc, &t)) return -1;
    ctx_t c;
    memset(&c, 0, sizeof c);
    c.sc = sc;
    c.run = run;
    c.t = &t;
    c.gfilm = gfilm;
    c.grad = grad;
    uint64_t local_tally[ORC_N_TALLIES];
    memset(local_tally, 0, sizeof local_tally);
    c.tally = local_tally;
    /* parameters: conc per (medium, dye slot), quantum yield per dye, sigma_s per medium */
    int np = 0;
    for (int m = 0; m < sc->n_media; ++m)
        for (int j = 0; j < sc->media[m].n_dyes; ++j) c.param_c[m][j] = np++;
    for (int d = 0; d < sc->n_dyes; ++d) c.param_qy[d] = np++;
    for (int m = 0; m < sc->n_media; ++m) c.param_ss[m] = np++;
    c.n_params = np;
    uint32_t B = run->parity_batches ? run->parity_batches : 1;
    c.wscale = (double)B / (double)run->total_paths;
    double* scratch_film = NULL;
    if (gfilm && !film) {
        scratch_film = calloc((size_t)orc_film_size(sc, B), sizeof(double));
        if (!scratch_film) { free_tables(&t); return fail("out of memory"); }
        c.film = scratch_film;
    } else {
        c.film = film;
    }
    if (sc->light == ORC_LIGHT_QUAD) {
        cross3(sc->lu, sc->lv, c.qn);
        normalize3(c.qn);
        memcpy(c.qt1, sc->lu, sizeof c.qt1);
        normalize3(c.qt1);
    }
    if (sc->sensor == ORC_SENSOR_PINHOLE) {
        for (int i = 0; i < 3; ++i) c.cf[i] = sc->look[i] - sc->eye[i];
        normalize3(c.cf);
        cross3(c.cf, sc->up, c.cr);
        normalize3(c.cr);
        cross3(c.cr, c.cf, c.cu);
        c.tany = tan(0.5 * sc->fov_y_deg * M_PI / 180.0);
        c.tanx = c.tany * (double)sc->width / (double)sc->height;
        c.area_img = 4.0 * c.tanx * c.tany;
    }
    for (uint64_t i = 0; i < run->path_count; ++i) {
        uint32_t pid = (uint32_t)(run->path_begin + i);
        c.pgrad = rec_grad ? rec_grad + i * (uint64_t)np : NULL;
        if (c.pgrad) memset(c.pgrad, 0, sizeof(double) * (size_t)np);
        run_path(&c, pid, rec ? rec + i : NULL, max_vertices);
    }
    if (tallies)
        for (int i = 0; i < ORC_N_TALLIES; ++i) tallies[i] += local_tally[i];
    free(scratch_film);
    free_tables(&t);
    return 0;
}

/* ------------------------------------------------------------------------- */
/* Camera-side estimator (sec. 4.1: paths start at the camera at the emission
 * wavelength and the light is sampled only where a fluorescence emission is
 * realised; sec. 4.3, eq. 12).
 *
 * One path per (sample s, pixel, emission bin k): a ray from the eye through
 * a uniform point of the pixel enters the box through its open face and walks
 * analogously at wavelength k (free flight eq. 6, isotropic scatter with
 * probability sigma_s/sigma_t, Lambertian walls with probability rho(k)); any
 * absorption ends it, a dye absorption included (one emission per path, K = 1),
 * as do the light quad and the open face.  Every collision in a dye medium is
 * a candidate emission vertex x_{n-1} of the paper's path: a uniform point x_n
 * on the light is drawn, the light is connected directly (V = 1 inside the
 * convex box, eq. 4 geometry term, eq. 5 transmittance at each line
 * wavelength, Lambertian emitter of radiance 1/(pi A) per unit power) and the
 * fluorescence source
 *     Q = 1/(4 pi) sum_d QY_d pmf_d(k) sum_l w_l sigma_a,d(lambda_l) T_l cos_n / (pi r^2)
 * (eq. 9 with F_f of eq. 10; w_l the light's line power fractions, summed
 * exactly) is scored divided by sigma_t(k): the collision estimate of the
 * radiance reaching the eye along the ray.  The pixel weight is
 * parity_batches / spp: a uniform point of the pixel has direction density
 * equal to the pinhole importance N_pix / (A_img cos^3), so no further factor
 * enters.  The forward walk with excitation_scatter = 0 and max_emissions = 1
 * estimates the same film component (comp 1). */

static void camera_frame(const orc_scene* sc, ctx_t* c) {
    cross3(sc->lu, sc->lv, c->qn);
    normalize3(c->qn);
    for (int i = 0; i < 3; ++i) c->cf[i] = sc->look[i] - sc->eye[i];
    normalize3(c->cf);
    cross3(c->cf, sc->up, c->cr);
    normalize3(c->cr);
    cross3(c->cr, c->cf, c->cu);
    c->tany = tan(0.5 * sc->fov_y_deg * M_PI / 180.0);
    c->tanx = c->tany * (double)sc->width / (double)sc->height;
}

/* Fluorescence source Q at the path's position for emission bin k, from one
 * light point drawn with (ua, ub). */
static double cam_source(ctx_t* c, path_t* p, int k, double ua, double ub) {
    const orc_scene* sc = c->sc;
    const tables_t* t = c->t;
    int N = t->N, m = p->medium;
    const orc_medium* md = &sc->media[m];
    double xn[3], d[3];
    for (int i = 0; i < 3; ++i) xn[i] = sc->lpos[i] + ua * sc->lu[i] + ub * sc->lv[i];
    perturb3(c, p, 4, xn);
    for (int i = 0; i < 3; ++i) d[i] = xn[i] - p->x[i];
    double r2 = dot3(d, d), r = sqrt(r2);
    double cos_n = -dot3(c->qn, d) / r; /* the light emits along +qn */
    upd_margin(&p->margin, fabs(cos_n));
    if (!(cos_n > 0.0)) { c->tally[ORC_T_SPLAT_MISS]++; return 0.0; }
    double wc[3] = {d[0] / r, d[1] / r, d[2] / r};
    double len[ORC_MAX_SPHERES];
    for (int s = 0; s < sc->n_spheres; ++s) len[s] = chord(p->x, wc, r, &sc->spheres[s], &p->margin);
    double total = 0.0;
    for (int l = 0; l < sc->n_lines; ++l) total += sc->line_power[l];
    double sum = 0.0;
    for (int l = 0; l < sc->n_lines; ++l) {
        int bl = t->line_bin[l];
        double tau = 0.0;
        for (int s = 0; s < sc->n_spheres; ++s)
            tau += t->sigma_t[sc->spheres[s].medium * N + bl] * len[s];
        double conv = 0.0;
        for (int j = 0; j < md->n_dyes; ++j) {
            int dye = md->dye[j];
            conv += t->sigma_a[(m * ORC_MAX_MEDIUM_DYES + j) * N + bl] * sc->dyes[dye].qy *
                    t->pmf[dye * N + k];
        }
        sum += sc->line_power[l] / total * exp(-tau) * conv;
    }
    c->tally[ORC_T_SPLAT_HIT]++;
    return sum * cos_n / (M_PI * r2) / (4.0 * M_PI);
}

static void run_camera_path(ctx_t* c, uint32_t pid, uint32_t spp, orc_record* rec,
                            uint32_t max_vertices) {
    const orc_scene* sc = c->sc;
    const tables_t* t = c->t;
    const orc_run* run = c->run;
    uint64_t* T = c->tally;
    int N = t->N, W = sc->width, H = sc->height;
    rng_t rng;
    rng.key[0] = (uint32_t)run->seed;
    rng.key[1] = (uint32_t)(run->seed >> 32) ^ run->instance;
    rng.pid = pid;
    path_t p;
    memset(&p, 0, sizeof p);
    p.pid = pid;
    p.margin = INFINITY;
    int k = (int)(pid % (uint32_t)N);
    uint32_t pix = (pid / (uint32_t)N) % (uint32_t)(W * H);
    uint32_t s = pid / ((uint32_t)N * (uint32_t)(W * H));
    int px = (int)(pix % (uint32_t)W), py = (int)(pix / (uint32_t)W);
    (void)spp;
    p.batch = s % (run->parity_batches ? run->parity_batches : 1);
    p.lam = k;
    p.comp = 1;
    p.region = -1;
    p.medium = -1;
    double L = scene_scale(sc);
    int exit_code = -1;
    uint32_t r[4], r1[4];
    int64_t idx = ((((int64_t)p.batch * 2 + 1) * H + py) * W + px) * N + k;
    double acc = 0.0;

    /* vertex 0: the eye ray through a uniform point of the pixel */
    draw(&rng, 0, 0, r);
    double xi = 2.0 * (px + unif(r[0])) / W - 1.0;
    double yi = 1.0 - 2.0 * (py + unif(r[1])) / H;
    for (int i = 0; i < 3; ++i) p.w[i] = c->cf[i] + xi * c->tanx * c->cr[i] + yi * c->tany * c->cu[i];
    normalize3(p.w);
    perturb3(c, &p, 1, p.w);
    T[ORC_T_PATHS]++;
    T[ORC_T_VERTICES]++;
    {
        /* entry into the box from outside: the last of the three slab entries */
        double t_in = -INFINITY, t_out = INFINITY;
        int face = -1, inside = 1;
        for (int a = 0; a < 3; ++a) {
            if (p.w[a] == 0.0) {
                if (sc->eye[a] < sc->box_lo[a] || sc->eye[a] > sc->box_hi[a]) inside = 0;
                continue;
            }
            double t0 = (sc->box_lo[a] - sc->eye[a]) / p.w[a];
            double t1 = (sc->box_hi[a] - sc->eye[a]) / p.w[a];
            double tn = p.w[a] > 0.0 ? t0 : t1, tf = p.w[a] > 0.0 ? t1 : t0;
            if (tn > t_in) { t_in = tn; face = p.w[a] > 0.0 ? 2 * a : 2 * a + 1; }
            if (tf < t_out) t_out = tf;
        }
        int enters = inside && face == sc->open_face && t_in > 0.0 && t_in < t_out;
        /* margin: the crossing of the open face's plane against that face's edges */
        int oa = sc->open_face / 2;
        double plane = (sc->open_face % 2) ? sc->box_hi[oa] : sc->box_lo[oa];
        double tp = p.w[oa] != 0.0 ? (plane - sc->eye[oa]) / p.w[oa] : INFINITY;
        if (isfinite(tp) && tp > 0.0)
            for (int b = 0; b < 3; ++b) {
                if (b == oa) continue;
                double q = sc->eye[b] + tp * p.w[b];
                double ext = sc->box_hi[b] - sc->box_lo[b];
                upd_margin(&p.margin, fmin(fabs(q - sc->box_lo[b]), fabs(sc->box_hi[b] - q)) / ext);
            }
        if (!enters) {
            exit_code = ORC_EXIT_ESC_T;
        } else {
            for (int i = 0; i < 3; ++i) p.x[i] = sc->eye[i] + t_in * p.w[i];
            perturb3(c, &p, 0, p.x);
            p.x[oa] = plane;
        }
    }

    while (exit_code < 0) {
        p.v++;
        if (max_vertices && p.v >= max_vertices) { exit_code = ORC_EXIT_TRUNC; break; }
        if (p.v >= (1u << 28)) { exit_code = ORC_EXIT_SCAP; break; }
        T[ORC_T_VERTICES]++;
        draw(&rng, p.v, 0, r);
        double u0 = unif(r[0]), u1 = unif(r[1]), u2 = unif(r[2]), u3 = unif(r[3]);
        double st = p.medium >= 0 ? t->sigma_t[p.medium * N + k] : 0.0;
        double tf = st > 0.0 ? -log(1.0 - u0) / st : INFINITY;
        hit_t h = next_surface(sc, p.x, p.w, p.region, 0);
        upd_margin(&p.margin, h.margin);
        if (isfinite(tf) && isfinite(h.d))
            upd_margin(&p.margin, fabs(tf - h.d) / fmax(fmax(tf, h.d), L));
        if (tf < h.d) {
            for (int i = 0; i < 3; ++i) p.x[i] += tf * p.w[i];
            perturb3(c, &p, 0, p.x);
            const orc_medium* md = &sc->media[p.medium];
            if (md->n_dyes > 0) {
                /* a candidate emission vertex: connect to the light */
                draw(&rng, p.v, 1, r1);
                double q = cam_source(c, &p, k, unif(r1[0]), unif(r1[1]));
                acc += c->wscale * q / st;
            }
            double sv = u1 * st;
            double thr = md->sigma_s;
            upd_margin(&p.margin, fabs(sv - thr) / st);
            if (sv < thr) {
                T[ORC_T_SCATTERS]++;
                p.n_scatter++;
                if (p.n_scatter > run->max_scatter) { exit_code = ORC_EXIT_SCAP; break; }
                iso_dir(u2, u3, p.w);
                perturb3(c, &p, 1, p.w);
                continue;
            }
            thr += md->sigma_a_bg;
            upd_margin(&p.margin, fabs(sv - thr) / st);
            if (sv < thr || md->n_dyes == 0) { exit_code = ORC_EXIT_BG; break; }
            /* a dye absorbs at the emission wavelength: a second emission ends the path */
            T[ORC_T_DYE_ABS]++;
            exit_code = ORC_EXIT_KCAP;
            break;
        }
        double dd = h.d;
        if (isfinite(dd)) {
            for (int i = 0; i < 3; ++i) p.x[i] += dd * p.w[i];
            perturb3(c, &p, 0, p.x);
            if ((h.kind == SURF_WALL || h.kind == SURF_ESCAPE) && h.index >= 0)
                p.x[h.index / 2] = (h.index % 2) ? sc->box_hi[h.index / 2] : sc->box_lo[h.index / 2];
        }
        if (h.kind == SURF_ESCAPE) { exit_code = ORC_EXIT_ESC_R; break; }
        if (h.kind == SURF_LIGHT) { exit_code = ORC_EXIT_LIGHT; break; }
        if (h.kind == SURF_WALL) {
            double rho = t->rho[h.index * N + k];
            upd_margin(&p.margin, fabs(u1 - rho));
            if (!(u1 < rho)) { exit_code = ORC_EXIT_WALL; break; }
            double n[3], t1[3];
            face_frame(h.index, n, t1);
            cos_dir(n, t1, u2, u3, p.w);
            perturb3(c, &p, 1, p.w);
            T[ORC_T_WALL_REFLECT]++;
            continue;
        }
        T[ORC_T_CROSSINGS]++;
        p.region = (h.kind == SURF_ENTER) ? h.index : -1;
        p.medium = region_medium(sc, p.region);
    }
    if (acc != 0.0 && c->film) deposit(c, &p, idx, acc, NULL);
    p.splat_sum = acc;
    T[ORC_T_EXIT0 + exit_code]++;
    if (rec) {
        rec->n_vertices = p.v + (exit_code == ORC_EXIT_TRUNC ? 0u : 1u);
        rec->n_scatter = p.n_scatter;
        rec->n_emit = 0;
        rec->exit_code = (uint32_t)exit_code;
        rec->lambda = k;
        rec->comp = 1;
        rec->region = p.region;
        memcpy(rec->pos, p.x, sizeof p.x);
        memcpy(rec->dir, p.w, sizeof p.w);
        rec->splat_sum = acc;
        rec->margin = p.margin;
    }
}

int32_t orc_render_camera(const orc_scene* sc, const orc_run* run, double* film,
                          uint64_t* tallies, orc_record* rec, uint32_t max_vertices) {
    g_err[0] = 0;
    if (!sc || !run) return fail("null argument");
    if (sc->geom != ORC_GEOM_BOX || sc->sensor != ORC_SENSOR_PINHOLE || sc->light != ORC_LIGHT_QUAD)
        return fail("the camera-side estimator needs a box scene with a pinhole and a quad light");
    for (int f = 0; f < 6; ++f)
        if (sc->wall_gloss[f] > 0.0) return fail("the camera-side estimator has Lambertian walls only");
    uint64_t per_sample = (uint64_t)sc->width * (uint64_t)sc->height * (uint64_t)sc->n_bins;
    if (per_sample == 0 || run->total_paths == 0 || run->total_paths % per_sample != 0)
        return fail("total_paths must be spp * width * height * n_bins");
    if (run->path_begin + run->path_count > run->total_paths)
        return fail("path range outside total_paths");
    if (run->total_paths > (1ull << 32)) return fail("total_paths exceeds 2^32");
    if (run->path_count > 0xFFFFFFFFull) return fail("path_count must be below 2^32");
    uint32_t spp = (uint32_t)(run->total_paths / per_sample);
    tables_t t;
    if (build_tables(sc, &t)) return -1;
    ctx_t c;
    memset(&c, 0, sizeof c);
    c.sc = sc;
    c.run = run;
    c.t = &t;
    c.film = film;
    uint64_t local_tally[ORC_N_TALLIES];
    memset(local_tally, 0, sizeof local_tally);
    c.tally = local_tally;
    uint32_t B = run->parity_batches ? run->parity_batches : 1;
    c.wscale = (double)B / (double)spp;
    camera_frame(sc, &c);
    for (uint64_t i = 0; i < run->path_count; ++i)
        run_camera_path(&c, (uint32_t)(run->path_begin + i), spp, rec ? rec + i : NULL,
                        max_vertices);
    if (tallies)
        for (int i = 0; i < ORC_N_TALLIES; ++i) tallies[i] += local_tally[i];
    free_tables(&t);
    return 0;
}
