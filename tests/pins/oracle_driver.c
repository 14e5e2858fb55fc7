/* Drives the oracle's entry points on a box scene (three dye spheres,
 * glossy and Lambertian walls, a camera), on a refractive dye slab and on an
 * unbounded medium, for the sanitizer builds run by the CPU tests (address,
 * undefined behaviour and leak checks): renders with film, tallies, records,
 * the gradient and per-path gradients, the camera-side estimator, the tables,
 * and rejected inputs.  Exits 0 when every call returns what it should. */
#include <stdio.h>
#include <stdlib.h>
#include <string.h>

#include "oracle.h"

static void gauss(orc_spectrum* s, double mu, double sd) {
    s->kind = ORC_SPEC_GAUSS;
    s->n = 1;
    s->x[0] = mu;
    s->y[0] = 1.0;
    s->s[0] = sd;
}

static void flat(orc_spectrum* s, double v) {
    s->kind = ORC_SPEC_PWL;
    s->n = 2;
    s->x[0] = 300.0;
    s->y[0] = v;
    s->x[1] = 800.0;
    s->y[1] = v;
}

static int check(int rc, int want, const char* what) {
    if ((rc == 0) != (want == 0)) {
        fprintf(stderr, "%s: rc %d (%s)\n", what, rc, orc_last_error());
        return 1;
    }
    return 0;
}

static int run_all(const orc_scene* sc, const orc_run* run) {
    int bad = 0;
    int64_t nf = orc_film_size(sc, run->parity_batches ? run->parity_batches : 1);
    int np = orc_n_params(sc);
    double* film = calloc((size_t)nf, sizeof(double));
    double* gfilm = malloc((size_t)nf * sizeof(double));
    double* grad = calloc((size_t)(np > 0 ? np : 1), sizeof(double));
    double* rec_grad = calloc((size_t)run->path_count * (size_t)(np > 0 ? np : 1), sizeof(double));
    orc_record* rec = calloc((size_t)run->path_count, sizeof(orc_record));
    uint64_t tallies[ORC_N_TALLIES] = {0};
    if (!film || !gfilm || !grad || !rec_grad || !rec) return 1;
    for (int64_t i = 0; i < nf; ++i) gfilm[i] = 1.0 + (double)(i % 7) * 0.125;
    bad |= check(orc_render(sc, run, film, tallies, NULL, NULL, NULL, NULL, 0), 0, "render");
    bad |= check(orc_render(sc, run, film, tallies, gfilm, grad, rec, rec_grad, 0), 0, "render+grad");
    bad |= check(orc_render(sc, run, NULL, tallies, NULL, NULL, rec, NULL, 17), 0, "records");
    bad |= check(orc_render(sc, run, film, NULL, gfilm, NULL, NULL, NULL, 0), 1, "gfilm without grad");
    free(film);
    free(gfilm);
    free(grad);
    free(rec_grad);
    free(rec);
    return bad;
}

int main(void) {
    int bad = 0;
    static orc_scene box, slab, inf;
    memset(&box, 0, sizeof box);
    box.n_bins = 101;
    box.lo_nm = 300.0;
    box.hi_nm = 800.0;
    box.n_dyes = 3;
    box.n_media = 3;
    for (int i = 0; i < 3; ++i) {
        gauss(&box.dyes[i].absorption, 450.0 + 100.0 * i, 20.0);
        gauss(&box.dyes[i].emission, 480.0 + 100.0 * i, 25.0);
        box.dyes[i].epsilon = 5e4;
        box.dyes[i].qy = 0.5 + 0.2 * i;
        box.media[i].sigma_s = 50.0 * (i + 1);
        box.media[i].sigma_a_bg = 0.01;
        box.media[i].n_dyes = 1;
        box.media[i].dye[0] = i;
        box.media[i].conc[0] = 10.0;
    }
    box.geom = ORC_GEOM_BOX;
    for (int a = 0; a < 3; ++a) {
        box.box_lo[a] = -1.0;
        box.box_hi[a] = 1.0;
    }
    box.open_face = 5;
    for (int f = 0; f < 5; ++f) flat(&box.walls[f], 0.7);
    box.wall_gloss[2] = 8.0;
    box.wall_gloss[4] = 40.0;
    box.n_spheres = 3;
    for (int i = 0; i < 3; ++i) {
        box.spheres[i].center[0] = -0.5 + 0.5 * i;
        box.spheres[i].center[1] = -0.79;
        box.spheres[i].center[2] = (i % 2) ? 0.2 : -0.2;
        box.spheres[i].radius = 0.2;
        box.spheres[i].medium = i;
    }
    box.light = ORC_LIGHT_QUAD;
    double lp[3] = {-0.25, 0.999, -0.25}, lu[3] = {0.5, 0.0, 0.0}, lv[3] = {0.0, 0.0, 0.5};
    memcpy(box.lpos, lp, sizeof lp);
    memcpy(box.lu, lu, sizeof lu);
    memcpy(box.lv, lv, sizeof lv);
    box.n_lines = 3;
    for (int i = 0; i < 3; ++i) {
        box.line_nm[i] = 450.0 + 100.0 * i;
        box.line_power[i] = 1.0;
    }
    box.sensor = ORC_SENSOR_PINHOLE;
    box.eye[2] = 3.4;
    box.up[1] = 1.0;
    box.fov_y_deg = 40.0;
    box.width = box.height = 12;
    orc_run run;
    memset(&run, 0, sizeof run);
    run.max_scatter = 10000;
    run.max_emissions = 1;
    run.excitation_scatter = 1;
    run.path_count = run.total_paths = 1500;
    run.parity_batches = 4;
    run.splat_rr = 0.05;
    bad |= run_all(&box, &run);
    run.perturb_eta = 1.0 / 8388608.0;
    run.perturb_pattern = 1;
    bad |= run_all(&box, &run);
    run.perturb_eta = 0.0;

    /* the camera-side estimator on the Lambertian box (glossy walls are refused) */
    {
        orc_scene lam = box;
        memset(lam.wall_gloss, 0, sizeof lam.wall_gloss);
        orc_run cr = run;
        cr.total_paths = (uint64_t)lam.width * lam.height * lam.n_bins * 2;
        cr.path_count = 3000;
        int64_t nf = orc_film_size(&lam, 4);
        double* film = calloc((size_t)nf, sizeof(double));
        orc_record* rec = calloc(3000, sizeof(orc_record));
        uint64_t t[ORC_N_TALLIES] = {0};
        if (!film || !rec) return 1;
        bad |= check(orc_render_camera(&lam, &cr, film, t, rec, 40), 0, "camera");
        bad |= check(orc_render_camera(&box, &cr, film, t, rec, 0), 1, "camera refuses glossy");
        free(film);
        free(rec);
    }
    /* tables */
    {
        int N = box.n_bins;
        double* v = calloc((size_t)N * 64, sizeof(double));
        int32_t lb[ORC_MAX_LINES];
        if (!v) return 1;
        bad |= check(orc_tables(&box, v, v + N, v + 4 * N, v + 8 * N, v + 12 * N, v + 16 * N, v + 40 * N, lb), 0,
                     "tables");
        free(v);
    }
    /* a refractive dye slab with an escape film, and an unbounded medium */
    memset(&slab, 0, sizeof slab);
    slab.n_bins = 51;
    slab.lo_nm = 300.0;
    slab.hi_nm = 800.0;
    slab.n_dyes = 1;
    gauss(&slab.dyes[0].absorption, 490.0, 20.0);
    gauss(&slab.dyes[0].emission, 520.0, 25.0);
    slab.dyes[0].epsilon = 7e4;
    slab.dyes[0].qy = 0.9;
    slab.n_media = 1;
    slab.media[0].sigma_s = 10.0;
    slab.media[0].sigma_a_bg = 0.01;
    slab.media[0].n_dyes = 1;
    slab.media[0].conc[0] = 10.0;
    slab.media[0].ior = 1.33;
    slab.geom = ORC_GEOM_SLAB;
    slab.z1 = 1.0;
    slab.light = ORC_LIGHT_BEAM;
    slab.ldir[2] = 1.0;
    slab.n_lines = 1;
    slab.line_nm[0] = 490.0;
    slab.line_power[0] = 1.0;
    slab.sensor = ORC_SENSOR_ESCAPE;
    run.splat_rr = 0.0;
    run.max_emissions = 0xFFFFFFFFu;
    bad |= run_all(&slab, &run);
    inf = slab;
    inf.geom = ORC_GEOM_INFINITE;
    inf.media[0].ior = 0.0;
    inf.light = ORC_LIGHT_POINT;
    bad |= run_all(&inf, &run);
    /* rejected inputs */
    slab.wall_gloss[0] = 5.0;
    bad |= check(orc_render(&slab, &run, NULL, NULL, NULL, NULL, NULL, NULL, 0), 1, "gloss without a box");
    slab.wall_gloss[0] = 0.0;
    run.total_paths = 10;
    bad |= check(orc_render(&slab, &run, NULL, NULL, NULL, NULL, NULL, NULL, 0), 1, "range");
    printf(bad ? "FAILED\n" : "ok\n");
    return bad;
}
