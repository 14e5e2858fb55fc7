// C-ABI implementation of the fpt library: descriptor validation, spectral
// table construction (fp64, rounded to fp32), device residency of scenes and
// the launch sequences of each entry point.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <array>
#include <cmath>
#include <cstdarg>
#include <cstdio>
#include <cstring>
#include <new>
#include <string>
#include <deque>
#include <map>
#include <vector>

#include "fpt.h"
#include "fpt_internal.h"

namespace fpt {
size_t transport_lds_bytes(const KParams& P, int block_threads, int mode);
size_t splat_jobs_lds_bytes(const KParams& P);
hipError_t launch_transport(const KParams& P, const KBuffers& B, int mode, int grid, int block,
                            hipStream_t s);
hipError_t transport_occupancy(const KParams& P, int mode, int block, int* blocks_per_cu);
hipError_t launch_zero_u32(uint32_t* p, size_t n, hipStream_t s);
hipError_t launch_zero_u64(unsigned long long* p, size_t n, hipStream_t s);
hipError_t launch_finalize_counts(const uint32_t* counts, float* film, size_t n, float scale,
                                  hipStream_t s);
size_t queue_words();
hipError_t launch_splat_jobs(const KParams& P, const KBuffers& B, int grid, hipStream_t s);
hipError_t launch_reduce_partials(const float* partials, int nblocks, int np, float* grad,
                                  hipStream_t s);
int batch_slot_words(int hist_words, int max_table_words);
size_t batch_lds_bytes(const KBatch& Bt, int block);
hipError_t batch_occupancy(const KBatch& Bt, int block, int* n);
hipError_t launch_batch(const KBatch& Bt, int grid, int block, hipStream_t s);
hipError_t launch_finalize_batch(const uint32_t* counts, float* films, const float* wscale,
                                 int hist_words, size_t n, hipStream_t s);
size_t camera_lds_bytes(const KParams& P);
hipError_t camera_occupancy(const KParams& P, bool rec, int block, int* blocks_per_cu);
hipError_t launch_camera(const KParams& P, const KBuffers& B, bool rec, int grid, int block,
                         hipStream_t s);
hipError_t static_scratch(void** ptr, size_t* bytes);
}  // namespace fpt

using namespace fpt;

namespace {

enum { MODE_FWD = 0, MODE_ADJ = 1, MODE_REC = 2, MODE_REC_ADJ = 3 };

thread_local std::string g_err;

int32_t set_err(int32_t code, const char* fmt, ...) {
    char buf[512];
    va_list ap;
    va_start(ap, fmt);
    vsnprintf(buf, sizeof buf, fmt, ap);
    va_end(ap);
    g_err = buf;
    return code;
}

int32_t hip_err(hipError_t e, const char* what) {
    if (e == hipErrorOutOfMemory) return set_err(FPT_E_NOMEM, "%s: %s", what, hipGetErrorString(e));
    return set_err(FPT_E_DEVICE, "%s: %s", what, hipGetErrorString(e));
}

// Allocation-failure injection for robustness tests: with FPT_FAULT_INJECT=N
// in the environment, the N-th allocation (device, pinned host, or the scene /
// batch object itself) made by one fpt_scene_create or fpt_batch_create call
// fails as out of memory; the call must then return FPT_E_NOMEM having freed
// everything it had allocated.  Armed at the start of those calls only.
thread_local int g_alloc_n = 0, g_alloc_fail = 0;

void alloc_fault_arm(bool on) {
    const char* e = on ? std::getenv("FPT_FAULT_INJECT") : nullptr;
    g_alloc_fail = e ? std::atoi(e) : 0;
    g_alloc_n = 0;
}

bool alloc_fault_hit() { return g_alloc_fail > 0 && ++g_alloc_n == g_alloc_fail; }

hipError_t dev_malloc(void** p, size_t bytes) {
    if (alloc_fault_hit()) return hipErrorOutOfMemory;
    return hipMalloc(p, bytes);
}

hipError_t pinned_malloc(void** p, size_t bytes) {
    if (alloc_fault_hit()) return hipErrorOutOfMemory;
    return hipHostMalloc(p, bytes, hipHostMallocDefault);
}

template <class T>
T* new_object() {
    if (alloc_fault_hit()) return nullptr;
    return new (std::nothrow) T();
}

#define HIP_TRY(expr, what)                       \
    do {                                          \
        hipError_t e_ = (expr);                   \
        if (e_ != hipSuccess) return hip_err(e_, what); \
    } while (0)

bool finite3(const double* v) { return std::isfinite(v[0]) && std::isfinite(v[1]) && std::isfinite(v[2]); }

double spectrum_at(const fpt_spectrum& s, double lam) {
    if (s.kind == FPT_SPECTRUM_GAUSS_MIX) {
        double acc = 0.0;
        for (int i = 0; i < s.n; ++i) {
            const double z = (lam - s.center_nm[i]) / s.width_nm[i];
            acc += s.value[i] * std::exp(-0.5 * z * z);
        }
        return acc;
    }
    // piecewise linear, constant beyond the end knots
    if (lam <= s.center_nm[0]) return s.value[0];
    if (lam >= s.center_nm[s.n - 1]) return s.value[s.n - 1];
    int i = 1;
    while (i < s.n - 1 && lam > s.center_nm[i]) ++i;
    const double x0 = s.center_nm[i - 1], x1 = s.center_nm[i];
    return s.value[i - 1] + (lam - x0) / (x1 - x0) * (s.value[i] - s.value[i - 1]);
}

// Value at grid point k (wavelength lam).
double spectrum_on_grid(const fpt_spectrum& s, double lam, int k) {
    return s.kind == FPT_SPECTRUM_TABULATED ? s.table[k] : spectrum_at(s, lam);
}

int32_t check_spectrum(const fpt_spectrum& s, const char* what, int n_bins) {
    if (s.kind == FPT_SPECTRUM_TABULATED) {
        if (!s.table) return set_err(FPT_E_INVALID, "%s: tabulated spectrum without a table", what);
        if (s.n != n_bins) return set_err(FPT_E_RANGE, "%s: %d tabulated values for %d grid points", what, s.n, n_bins);
        for (int k = 0; k < s.n; ++k)
            if (!std::isfinite(s.table[k])) return set_err(FPT_E_INVALID, "%s: non-finite tabulated value", what);
        return FPT_OK;
    }
    if (s.kind != FPT_SPECTRUM_GAUSS_MIX && s.kind != FPT_SPECTRUM_PIECEWISE_LINEAR)
        return set_err(FPT_E_INVALID, "%s: unknown spectrum kind %d", what, s.kind);
    if (s.n < 1 || s.n > FPT_MAX_SPECTRUM_TERMS)
        return set_err(FPT_E_RANGE, "%s: %d spectrum terms", what, s.n);
    for (int i = 0; i < s.n; ++i) {
        if (!std::isfinite(s.center_nm[i]) || !std::isfinite(s.value[i]))
            return set_err(FPT_E_INVALID, "%s: non-finite spectrum term", what);
        if (s.kind == FPT_SPECTRUM_GAUSS_MIX) {
            if (!(s.width_nm[i] > 0.0) || !std::isfinite(s.width_nm[i]))
                return set_err(FPT_E_INVALID, "%s: Gaussian width must be > 0", what);
            if (s.value[i] < 0.0) return set_err(FPT_E_INVALID, "%s: negative Gaussian weight", what);
        } else if (i > 0 && !(s.center_nm[i] > s.center_nm[i - 1])) {
            return set_err(FPT_E_INVALID, "%s: knots must increase", what);
        }
    }
    return FPT_OK;
}

int snap_line(double nm, double lo, double delta, int n) {
    const double k = std::ceil((nm - lo) / delta - 0.5);  // nearest, ties to the lower point
    if (!(k >= 0.0) || k > (double)(n - 1)) return -1;
    return (int)k;
}

}  // namespace

struct fpt_scene {
    fpt_scene_desc desc;
    int device = 0;
    int n_cu = 256;
    int np = 0;
    std::vector<uint32_t> image;
    KParams base;
    uint32_t* d_tables = nullptr;
    // device scratch, reserved once at creation for the largest launch any
    // launch shape gives on this device (renders never allocate)
    uint32_t* d_counts = nullptr;  // escape counts, up to 64 parity slices
    size_t counts_words = 0;
    unsigned long long* d_counter = nullptr;  // path queue heads
    float* d_partials = nullptr;   // adjoint per-block partial gradients
    size_t partials_blocks = 0;
    uint32_t* d_sjobs = nullptr;   // deferred pinhole connections, kSjobSlice entries per wave
    size_t sjob_waves = 0;         // waves d_sjobs has slices for
    uint32_t* d_sjob_counts = nullptr;
    uint32_t* h_stage = nullptr;   // pinned staging of the table image (fpt_scene_set_params)
    hipEvent_t staged = nullptr;   // the last upload from h_stage has completed
    bool timing = false;             // record events around launches (fpt_scene_set_timing)
    std::vector<hipEvent_t> events;  // 3 per timed render: transport start, end, deferred end
    int timed = 0;
    fpt_tune tune;
    std::vector<float> h_st, h_cdf, h_rho;
    std::vector<int> h_line_bin;
    std::deque<std::vector<double>> tabs;  // copies of tabulated spectra the descriptor points at
};

namespace {

int32_t validate(const fpt_scene_desc* d) {
    if (d->n_bins < 2 || d->n_bins > FPT_MAX_BINS)
        return set_err(FPT_E_RANGE, "n_bins %d outside [2, %d]", d->n_bins, FPT_MAX_BINS);
    if (!(d->hi_nm > d->lo_nm) || !std::isfinite(d->lo_nm) || !std::isfinite(d->hi_nm))
        return set_err(FPT_E_INVALID, "grid needs finite lo_nm < hi_nm");
    if (d->absorptivity_base != FPT_BASE_DECADIC && d->absorptivity_base != FPT_BASE_NATURAL)
        return set_err(FPT_E_INVALID, "absorptivity_base %d", d->absorptivity_base);
    if (d->n_dyes < 0 || d->n_dyes > FPT_MAX_DYES) return set_err(FPT_E_RANGE, "n_dyes %d", d->n_dyes);
    if (d->n_media < 1 || d->n_media > FPT_MAX_MEDIA) return set_err(FPT_E_RANGE, "n_media %d", d->n_media);
    for (int i = 0; i < d->n_dyes; ++i) {
        const fpt_dye& y = d->dyes[i];
        int32_t rc;
        if ((rc = check_spectrum(y.absorption, "dye absorption", d->n_bins)) != FPT_OK) return rc;
        if ((rc = check_spectrum(y.emission, "dye emission", d->n_bins)) != FPT_OK) return rc;
        if (!(y.qy >= 0.0 && y.qy <= 1.0)) return set_err(FPT_E_RANGE, "dye %d: qy %g outside [0,1]", i, y.qy);
        if (!(y.epsilon_M_cm >= 0.0) || !std::isfinite(y.epsilon_M_cm))
            return set_err(FPT_E_RANGE, "dye %d: epsilon must be finite and >= 0", i);
    }
    for (int m = 0; m < d->n_media; ++m) {
        const fpt_medium& md = d->media[m];
        if (!(md.sigma_s_mm >= 0.0) || !std::isfinite(md.sigma_s_mm))
            return set_err(FPT_E_RANGE, "medium %d: sigma_s must be finite and >= 0", m);
        if (!(md.sigma_a_bg_mm >= 0.0) || !std::isfinite(md.sigma_a_bg_mm))
            return set_err(FPT_E_RANGE, "medium %d: sigma_a_bg must be finite and >= 0", m);
        if (md.n_dyes < 0 || md.n_dyes > FPT_MAX_MEDIUM_DYES)
            return set_err(FPT_E_RANGE, "medium %d: %d dyes", m, md.n_dyes);
        if (!(md.ior == 0.0 || (md.ior >= 1.0 && md.ior <= 4.0)))
            return set_err(FPT_E_RANGE, "medium %d: refractive index %g outside [1, 4]", m, md.ior);
        for (int j = 0; j < md.n_dyes; ++j) {
            if (md.dye[j] < 0 || md.dye[j] >= d->n_dyes)
                return set_err(FPT_E_INVALID, "medium %d: dye index %d", m, md.dye[j]);
            if (!(md.conc_uM[j] >= 0.0) || !std::isfinite(md.conc_uM[j]))
                return set_err(FPT_E_RANGE, "medium %d: concentration must be finite and >= 0", m);
        }
    }
    if (d->n_lines < 1 || d->n_lines > FPT_MAX_LINES) return set_err(FPT_E_RANGE, "n_lines %d", d->n_lines);
    double tot = 0.0;
    for (int i = 0; i < d->n_lines; ++i) {
        if (!(d->line_power[i] >= 0.0) || !std::isfinite(d->line_power[i]))
            return set_err(FPT_E_RANGE, "line %d power", i);
        tot += d->line_power[i];
    }
    if (!(tot > 0.0)) return set_err(FPT_E_INVALID, "total light power must be > 0");
    if (d->light < FPT_LIGHT_BEAM || d->light > FPT_LIGHT_QUAD) return set_err(FPT_E_INVALID, "light kind %d", d->light);
    if (d->sensor != FPT_SENSOR_ESCAPE && d->sensor != FPT_SENSOR_PINHOLE)
        return set_err(FPT_E_INVALID, "sensor kind %d", d->sensor);
    switch (d->geometry) {
    case FPT_GEOM_SLAB:
        if (!(d->slab_z1 > d->slab_z0) || !std::isfinite(d->slab_z0) || !std::isfinite(d->slab_z1))
            return set_err(FPT_E_INVALID, "slab needs finite z0 < z1");
        break;
    case FPT_GEOM_HALFSPACE:
        if (!std::isfinite(d->slab_z0)) return set_err(FPT_E_INVALID, "half-space z0");
        break;
    case FPT_GEOM_SPHERE:
        if (!finite3(d->body_center) || !(d->body_radius > 0.0)) return set_err(FPT_E_INVALID, "body sphere");
        break;
    case FPT_GEOM_INFINITE:
        break;
    case FPT_GEOM_BOX:
        break;
    default:
        return set_err(FPT_E_INVALID, "geometry kind %d", d->geometry);
    }
    bool glossy = false;
    for (int f = 0; f < 6; ++f) {
        if (!(d->wall_gloss[f] >= 0.0 && d->wall_gloss[f] <= 1e4))
            return set_err(FPT_E_RANGE, "wall %d: Phong exponent outside [0, 1e4]", f);
        glossy = glossy || d->wall_gloss[f] > 0.0;
    }
    if (glossy && (d->geometry != FPT_GEOM_BOX || d->sensor != FPT_SENSOR_PINHOLE))
        return set_err(FPT_E_UNSUPPORTED, "glossy walls need a box scene with a pinhole "
                                          "(path weights do not fit integer escape tallies)");
    if (d->geometry != FPT_GEOM_BOX) {
        if (d->body_medium < 0 || d->body_medium >= d->n_media) return set_err(FPT_E_INVALID, "body_medium");
        if (d->sensor != FPT_SENSOR_ESCAPE) return set_err(FPT_E_UNSUPPORTED, "pinhole sensor needs a box scene");
        if (d->light == FPT_LIGHT_QUAD) return set_err(FPT_E_UNSUPPORTED, "quad light needs a box scene");
        if (!finite3(d->light_pos)) return set_err(FPT_E_INVALID, "light position");
        if (d->light == FPT_LIGHT_BEAM) {
            const double n = std::sqrt(d->light_dir[0] * d->light_dir[0] + d->light_dir[1] * d->light_dir[1] +
                                       d->light_dir[2] * d->light_dir[2]);
            if (!(n > 0.0) || !std::isfinite(n)) return set_err(FPT_E_INVALID, "beam direction");
        }
        return FPT_OK;
    }
    // box scene
    if (!finite3(d->box_lo) || !finite3(d->box_hi)) return set_err(FPT_E_INVALID, "box bounds");
    for (int a = 0; a < 3; ++a)
        if (!(d->box_hi[a] > d->box_lo[a])) return set_err(FPT_E_INVALID, "box needs lo < hi");
    if (d->open_face < 0 || d->open_face > 5) return set_err(FPT_E_INVALID, "open_face %d", d->open_face);
    for (int f = 0; f < 6; ++f) {
        if (f == d->open_face) continue;
        int32_t rc = check_spectrum(d->walls[f], "wall", d->n_bins);
        if (rc != FPT_OK) return rc;
    }
    if (d->light != FPT_LIGHT_QUAD) return set_err(FPT_E_UNSUPPORTED, "box scenes need a quad light");
    if (!finite3(d->light_pos) || !finite3(d->light_u) || !finite3(d->light_v))
        return set_err(FPT_E_INVALID, "quad light geometry");
    if (d->n_spheres < 0 || d->n_spheres > FPT_MAX_SPHERES) return set_err(FPT_E_RANGE, "n_spheres %d", d->n_spheres);
    for (int s = 0; s < d->n_spheres; ++s) {
        const fpt_sphere& sp = d->spheres[s];
        if (!finite3(sp.center) || !(sp.radius > 0.0)) return set_err(FPT_E_INVALID, "sphere %d", s);
        if (sp.medium < 0 || sp.medium >= d->n_media) return set_err(FPT_E_INVALID, "sphere %d medium", s);
        if (d->media[sp.medium].ior != 0.0 && d->media[sp.medium].ior != 1.0)
            return set_err(FPT_E_UNSUPPORTED, "sphere %d: refractive media need index-matched boundaries in "
                                              "box scenes (a camera connection cannot cross a refracting surface)", s);
        for (int a = 0; a < 3; ++a)
            if (sp.center[a] - sp.radius <= d->box_lo[a] || sp.center[a] + sp.radius >= d->box_hi[a])
                return set_err(FPT_E_INVALID, "sphere %d must lie strictly inside the box", s);
        for (int t = 0; t < s; ++t) {
            const fpt_sphere& q = d->spheres[t];
            double dd = 0.0;
            for (int a = 0; a < 3; ++a) dd += (sp.center[a] - q.center[a]) * (sp.center[a] - q.center[a]);
            if (std::sqrt(dd) <= sp.radius + q.radius) return set_err(FPT_E_INVALID, "spheres %d and %d overlap", t, s);
        }
    }
    if (d->sensor == FPT_SENSOR_PINHOLE) {
        if (d->width < 1 || d->height < 1 || (int64_t)d->width * d->height > (1ll << 26))
            return set_err(FPT_E_RANGE, "image %dx%d", d->width, d->height);
        if (!(d->fov_y_deg > 0.0 && d->fov_y_deg < 179.0)) return set_err(FPT_E_RANGE, "fov_y_deg");
        if (!finite3(d->eye) || !finite3(d->look) || !finite3(d->up)) return set_err(FPT_E_INVALID, "camera");
        bool inside = true;
        for (int a = 0; a < 3; ++a) inside = inside && d->eye[a] >= d->box_lo[a] && d->eye[a] <= d->box_hi[a];
        if (inside) return set_err(FPT_E_UNSUPPORTED, "the eye must be outside the box");
    }
    return FPT_OK;
}

void norm3(double* v) {
    const double n = std::sqrt(v[0] * v[0] + v[1] * v[1] + v[2] * v[2]);
    v[0] /= n; v[1] /= n; v[2] /= n;
}
void cross3(const double* a, const double* b, double* o) {
    o[0] = a[1] * b[2] - a[2] * b[1];
    o[1] = a[2] * b[0] - a[0] * b[2];
    o[2] = a[0] * b[1] - a[1] * b[0];
}

uint32_t fbits(float f) {
    uint32_t u;
    std::memcpy(&u, &f, 4);
    return u;
}

// Builds the fp32 table image and the scene part of the kernel parameters.
// Spheres whose every point passes a pinhole connection's geometric tests,
// with a margin far above fp32 rounding (bit s of the result): a connection
// from inside such a sphere is in the image, leaves through the open face and
// misses the light quad, so the kernels need not evaluate those tests for it.
// A ball of centre c and radius r passes when it lies inside each of these
// half-spaces through the eye with clearance r (1 + 1e-3) + 1e-4 mm:
//   - in front of the camera and inside the image: the planes through the eye
//     of the image's four edges (fov);
//   - through the open face: the planes through the eye and the face's four
//     edges (the segment to the eye then crosses the face's plane inside it,
//     the eye lying outside the box beyond that plane);
// and when the ball and the eye lie strictly on the same side of the light
// quad's plane (the segment cannot cross the quad).
uint32_t clear_spheres(const fpt_scene_desc& d) {
    auto dot = [](const double* a, const double* b) { return a[0] * b[0] + a[1] * b[1] + a[2] * b[2]; };
    auto unit = [](double* v) {
        const double n = std::sqrt(v[0] * v[0] + v[1] * v[1] + v[2] * v[2]);
        for (int i = 0; i < 3; ++i) v[i] /= n;
    };
    double f[3] = {d.look[0] - d.eye[0], d.look[1] - d.eye[1], d.look[2] - d.eye[2]}, r[3], u[3];
    unit(f);
    cross3(f, d.up, r);
    unit(r);
    cross3(r, f, u);
    const double ty = std::tan(0.5 * d.fov_y_deg * M_PI / 180.0), tx = ty * d.width / d.height;
    // inward normals of the half-spaces through the eye
    std::vector<std::array<double, 3>> planes;
    for (int sg = -1; sg <= 1; sg += 2) {
        std::array<double, 3> a, b;
        for (int i = 0; i < 3; ++i) {
            a[i] = tx * f[i] + sg * r[i];
            b[i] = ty * f[i] + sg * u[i];
        }
        planes.push_back(a);
        planes.push_back(b);
    }
    const int ax = d.open_face >> 1;
    const double plane = (d.open_face & 1) ? d.box_hi[ax] : d.box_lo[ax];
    double mid[3];
    for (int i = 0; i < 3; ++i) mid[i] = 0.5 * (d.box_lo[i] + d.box_hi[i]);
    mid[ax] = plane;
    for (int k = 1; k <= 2; ++k) {
        const int a1 = (ax + k) % 3, a2 = (ax + 3 - k) % 3;  // edge across a1, running along a2
        for (int side = 0; side < 2; ++side) {
            double p0[3] = {0.0, 0.0, 0.0}, e2[3] = {0.0, 0.0, 0.0}, v[3], n[3];
            p0[ax] = plane;
            p0[a1] = side ? d.box_hi[a1] : d.box_lo[a1];
            e2[a2] = 1.0;
            for (int i = 0; i < 3; ++i) v[i] = p0[i] - d.eye[i];
            cross3(e2, v, n);
            double m[3] = {mid[0] - d.eye[0], mid[1] - d.eye[1], mid[2] - d.eye[2]};
            if (dot(n, m) < 0.0)
                for (double& c : n) c = -c;
            planes.push_back({n[0], n[1], n[2]});
        }
    }
    double ln[3] = {0.0, 0.0, 0.0};
    cross3(d.light_u, d.light_v, ln);
    unit(ln);
    // the eye outside the box, beyond the open face's plane
    const double out = (d.open_face & 1) ? d.eye[ax] - plane : plane - d.eye[ax];
    if (!(out >= 1e-4)) return 0u;
    uint32_t bits = 0u;
    for (int s = 0; s < d.n_spheres; ++s) {
        const fpt_sphere& sp = d.spheres[s];
        const double rad = sp.radius, clear = rad * (1.0 + 1e-3) + 1e-4;
        double c[3] = {sp.center[0] - d.eye[0], sp.center[1] - d.eye[1], sp.center[2] - d.eye[2]};
        bool ok = dot(c, f) >= clear;
        for (const auto& pl : planes) {
            double n[3] = {pl[0], pl[1], pl[2]};
            unit(n);
            ok = ok && dot(c, n) >= clear;
        }
        double qc[3] = {sp.center[0] - d.light_pos[0], sp.center[1] - d.light_pos[1], sp.center[2] - d.light_pos[2]};
        double qe[3] = {d.eye[0] - d.light_pos[0], d.eye[1] - d.light_pos[1], d.eye[2] - d.light_pos[2]};
        const double sc_ = dot(ln, qc), se = dot(ln, qe);
        ok = ok && sc_ * se > 0.0 && std::fabs(sc_) >= clear && std::fabs(se) >= 1e-4;
        if (ok) bits |= 1u << s;
    }
    return bits;
}

// Spheres whose medium reaches an optical depth of tau0 across the sphere at
// some wavelength (bit s): only there can a connection be opaque within the
// sphere itself, which the kernels count as a zero-valued hit without
// evaluating it.
uint32_t opaque_capable(const fpt_scene_desc& d, const std::vector<float>& st, float tau0) {
    uint32_t bits = 0u;
    for (int s = 0; s < d.n_spheres; ++s) {
        const fpt_sphere& sp = d.spheres[s];
        float stmax = 0.f;
        for (int k = 0; k < d.n_bins; ++k) stmax = std::max(stmax, st[(size_t)sp.medium * d.n_bins + k]);
        if ((double)stmax * 2.0 * sp.radius >= (double)tau0) bits |= 1u << s;
    }
    return bits;
}

// The spheres a segment from a point of sphere s to the eye can cross
// (bit s' of occl[s]; s itself always).  Seen from the eye, sphere s fills
// the cone of half-angle asin(r_s / |c_s - e|) about its centre's direction;
// such a segment lies in that cone and ends nearer to the eye than
// |c_s - e| + r_s.  Sphere s' is left out when its own cone is separated from
// sphere s's by at least 1e-3 rad, or when all of it lies at least 1e-3 mm
// beyond that distance; either way every such segment misses it by far more
// than fp32 rounding, so the kernels' chord of s' is exactly 0 there.
void sphere_occluders(const fpt_scene_desc& d, uint32_t* occl) {
    for (int s = 0; s < FPT_MAX_SPHERES; ++s) occl[s] = 0u;
    double a[FPT_MAX_SPHERES][3], dist[FPT_MAX_SPHERES], half[FPT_MAX_SPHERES];
    bool cone[FPT_MAX_SPHERES];
    for (int s = 0; s < d.n_spheres; ++s) {
        const fpt_sphere& sp = d.spheres[s];
        double n2 = 0.0;
        for (int i = 0; i < 3; ++i) {
            a[s][i] = sp.center[i] - d.eye[i];
            n2 += a[s][i] * a[s][i];
        }
        dist[s] = std::sqrt(n2);
        cone[s] = dist[s] > sp.radius * (1.0 + 1e-6);  // the eye outside the sphere
        half[s] = cone[s] ? std::asin(sp.radius / dist[s]) : M_PI;
        if (cone[s])
            for (int i = 0; i < 3; ++i) a[s][i] /= dist[s];
    }
    for (int s = 0; s < d.n_spheres; ++s) {
        occl[s] = 1u << s;
        for (int t = 0; t < d.n_spheres; ++t) {
            if (t == s) continue;
            bool apart = false;
            if (cone[s] && cone[t]) {
                const double c = std::max(-1.0, std::min(1.0, a[s][0] * a[t][0] + a[s][1] * a[t][1] + a[s][2] * a[t][2]));
                apart = std::acos(c) >= half[s] + half[t] + 1e-3;
            }
            const bool beyond = dist[t] - d.spheres[t].radius >= dist[s] + d.spheres[s].radius + 1e-3;
            if (!(apart || beyond)) occl[s] |= 1u << t;
        }
    }
}

int32_t build_tables(fpt_scene* sc) {
    const fpt_scene_desc& d = sc->desc;
    const int N = d.n_bins;
    const double delta = (d.hi_nm - d.lo_nm) / (N - 1);
    std::vector<double> lam(N);
    for (int k = 0; k < N; ++k) lam[k] = d.lo_nm + delta * k;

    // absorption peak-normalised on the grid; emission an area-normalised PMF
    std::vector<double> ahat((size_t)std::max(1, d.n_dyes) * N), cdf((size_t)std::max(1, d.n_dyes) * N);
    std::vector<double> pmf((size_t)std::max(1, d.n_dyes) * N);
    for (int i = 0; i < d.n_dyes; ++i) {
        double peak = 0.0, area = 0.0;
        for (int k = 0; k < N; ++k) {
            const double a = spectrum_on_grid(d.dyes[i].absorption, lam[k], k);
            const double e = spectrum_on_grid(d.dyes[i].emission, lam[k], k);
            if (a < 0.0 || e < 0.0) return set_err(FPT_E_INVALID, "dye %d: negative spectrum value", i);
            ahat[(size_t)i * N + k] = a;
            cdf[(size_t)i * N + k] = e;
            peak = std::max(peak, a);
            area += e;
        }
        if (!(peak > 0.0) || !(area > 0.0)) return set_err(FPT_E_INVALID, "dye %d: spectrum vanishes on the grid", i);
        double run = 0.0;
        for (int k = 0; k < N; ++k) {
            ahat[(size_t)i * N + k] /= peak;
            pmf[(size_t)i * N + k] = cdf[(size_t)i * N + k] / area;
            run += cdf[(size_t)i * N + k] / area;
            cdf[(size_t)i * N + k] = run;
        }
        cdf[(size_t)i * N + N - 1] = 1.0;
    }
    int cum_stride = 0, kap_stride = 0;
    for (int m = 0; m < d.n_media; ++m) {
        cum_stride = std::max(cum_stride, d.media[m].n_dyes - 1);
        kap_stride = std::max(kap_stride, d.media[m].n_dyes);
    }
    const double base = d.absorptivity_base == FPT_BASE_DECADIC ? std::log(10.0) : 1.0;

    // gradient parameter indices: conc per (medium, slot), qy per dye, sigma_s per medium
    int pc[FPT_MAX_MEDIA][FPT_MAX_MEDIUM_DYES], pq[FPT_MAX_DYES], pss[FPT_MAX_MEDIA];
    int np = 0;
    for (int m = 0; m < d.n_media; ++m)
        for (int j = 0; j < d.media[m].n_dyes; ++j) pc[m][j] = np++;
    for (int i = 0; i < d.n_dyes; ++i) pq[i] = np++;
    for (int m = 0; m < d.n_media; ++m) pss[m] = np++;
    sc->np = np;

    KParams& P = sc->base;
    std::memset(&P, 0, sizeof P);
    P.N = N;
    P.n_media = d.n_media;
    P.n_dyes = d.n_dyes;
    P.cum_stride = cum_stride;
    P.kap_stride = kap_stride;
    int off = 0;
    P.off_med = off; off += d.n_media * kMedWords;
    P.off_dye = off; off += std::max(1, d.n_dyes) * kDyeWords;
    off = (off + 1) & ~1;  // float2 alignment
    P.off_st = off; off += 2 * d.n_media * N;
    P.off_cum = off; off += d.n_media * cum_stride * N;
    P.off_cdf = off; off += d.n_dyes * N;
    P.off_rho = off; off += 6 * N;
    P.off_gloss = off; off += d.geometry == FPT_GEOM_BOX ? 8 : 0;  // 6 exponents, even alignment
    P.off_kap = off; off += d.n_media * kap_stride * N;
    const bool cam = d.geometry == FPT_GEOM_BOX && d.sensor == FPT_SENSOR_PINHOLE;
    P.off_src = off; off += cam ? d.n_media * N * d.n_lines : 0;
    P.off_csig = off; off += cam ? d.n_spheres * d.n_lines : 0;
    P.table_words = off;
    std::vector<uint32_t>& img = sc->image;
    img.assign((size_t)off, 0u);
    sc->h_st.assign((size_t)d.n_media * N, 0.f);
    sc->h_cdf.assign((size_t)std::max(1, d.n_dyes) * N, 0.f);
    sc->h_rho.assign((size_t)6 * N, 0.f);

    for (int m = 0; m < d.n_media; ++m) {
        const fpt_medium& md = d.media[m];
        uint32_t* r = &img[P.off_med + m * kMedWords];
        r[MW_SS] = fbits((float)md.sigma_s_mm);
        r[MW_THR_BG] = fbits((float)(md.sigma_s_mm + md.sigma_a_bg_mm));
        r[MW_NDYES] = (uint32_t)md.n_dyes;
        r[MW_INV_SS] = fbits(md.sigma_s_mm > 0.0 ? (float)(1.0 / md.sigma_s_mm) : 0.f);
        r[MW_PSS] = (uint32_t)pss[m];
        for (int j = 0; j < md.n_dyes; ++j) {
            r[MW_DYE + j] = (uint32_t)md.dye[j];
            r[MW_INV_C + j] = fbits(md.conc_uM[j] > 0.0 ? (float)(1.0 / md.conc_uM[j]) : 0.f);
            r[MW_PC + j] = (uint32_t)pc[m][j];
        }
        for (int k = 0; k < N; ++k) {
            double acc = md.sigma_s_mm + md.sigma_a_bg_mm;
            for (int j = 0; j < md.n_dyes; ++j) {
                const int y = md.dye[j];
                const double kap = base * d.dyes[y].epsilon_M_cm * 1e-7 * ahat[(size_t)y * N + k];
                acc += kap * md.conc_uM[j];
                if (j < md.n_dyes - 1) img[P.off_cum + (m * cum_stride + j) * N + k] = fbits((float)acc);
                img[P.off_kap + (m * kap_stride + j) * N + k] = fbits((float)kap);
            }
            const float st = (float)acc;
            img[P.off_st + 2 * (m * N + k)] = fbits(st);
            img[P.off_st + 2 * (m * N + k) + 1] = fbits(acc > 0.0 ? (float)(1.0 / acc) : INFINITY);
            sc->h_st[(size_t)m * N + k] = st;
        }
    }
    for (int i = 0; i < d.n_dyes; ++i) {
        uint32_t* r = &img[P.off_dye + i * kDyeWords];
        const double q = d.dyes[i].qy;
        r[DW_QY] = fbits((float)q);
        r[DW_INV_QY] = fbits(q > 0.0 ? (float)(1.0 / q) : 0.f);
        r[DW_INV_1MQY] = fbits(q < 1.0 ? (float)(1.0 / (1.0 - q)) : 0.f);
        r[DW_PQ] = (uint32_t)pq[i];
        for (int k = 0; k < N; ++k) {
            const float c = (float)cdf[(size_t)i * N + k];
            img[P.off_cdf + i * N + k] = fbits(c);
            sc->h_cdf[(size_t)i * N + k] = c;
        }
    }
    if (d.geometry == FPT_GEOM_BOX) {
        for (int f = 0; f < 6; ++f) {
            const bool g = f != d.open_face && d.wall_gloss[f] > 0.0;
            img[P.off_gloss + f] = fbits(g ? (float)d.wall_gloss[f] : 0.f);
            P.glossy = P.glossy || g;
            for (int k = 0; k < N; ++k) {
                const double r = (f == d.open_face) ? 0.0 : spectrum_on_grid(d.walls[f], lam[k], k);
                if (!(r >= 0.0 && r <= 1.0)) return set_err(FPT_E_RANGE, "wall %d reflectance outside [0,1]", f);
                img[P.off_rho + f * N + k] = fbits((float)r);
                sc->h_rho[(size_t)f * N + k] = (float)r;
            }
        }
    }
    // light lines
    double tot = 0.0;
    for (int i = 0; i < d.n_lines; ++i) tot += d.line_power[i];
    double c = 0.0;
    sc->h_line_bin.assign(d.n_lines, 0);
    for (int i = 0; i < d.n_lines; ++i) {
        const int k = snap_line(d.line_nm[i], d.lo_nm, delta, N);
        if (k < 0) return set_err(FPT_E_RANGE, "light line %g nm lies off the grid", d.line_nm[i]);
        P.line_bin[i] = k;
        sc->h_line_bin[i] = k;
        c += d.line_power[i] / tot;
        P.line_cum[i] = (float)c;
    }
    P.line_cum[d.n_lines - 1] = 1.0f;
    P.n_lines = d.n_lines;
    if (cam) {
        // camera-side source per (medium, emission bin, line): the line's power
        // fraction times the light absorbed by each dye at the line and
        // re-emitted into bin k (QY, emission PMF), over 4 pi (isotropic) and pi
        // (Lambertian emitter of unit power per unit area)
        for (int m = 0; m < d.n_media; ++m) {
            const fpt_medium& md = d.media[m];
            for (int k = 0; k < N; ++k)
                for (int l = 0; l < d.n_lines; ++l) {
                    double v = 0.0;
                    for (int j = 0; j < md.n_dyes; ++j) {
                        const int y = md.dye[j];
                        const double sa = base * d.dyes[y].epsilon_M_cm * 1e-7 *
                                          ahat[(size_t)y * N + P.line_bin[l]] * md.conc_uM[j];
                        v += d.dyes[y].qy * pmf[(size_t)y * N + k] * sa;
                    }
                    v *= d.line_power[l] / tot / (4.0 * M_PI * M_PI);
                    img[P.off_src + (m * N + k) * d.n_lines + l] = fbits((float)v);
                }
        }
        for (int s = 0; s < d.n_spheres; ++s)
            for (int l = 0; l < d.n_lines; ++l)
                img[P.off_csig + s * d.n_lines + l] =
                    fbits(sc->h_st[(size_t)d.spheres[s].medium * N + P.line_bin[l]]);
    }
    // geometry
    P.geometry = d.geometry;
    P.body_medium = d.body_medium;
    P.light = d.light;
    P.sensor = d.sensor;
    P.z0 = (float)d.slab_z0;
    P.z1 = (float)d.slab_z1;
    for (int a = 0; a < 3; ++a) P.bc[a] = (float)d.body_center[a];
    P.br2 = (float)(d.body_radius * d.body_radius);
    P.ior = 1.f;
    if (d.geometry == FPT_GEOM_SLAB || d.geometry == FPT_GEOM_HALFSPACE || d.geometry == FPT_GEOM_SPHERE) {
        const double n = d.media[d.body_medium].ior;
        P.ior = n > 0.0 ? (float)n : 1.f;
    }
    for (int a = 0; a < 3; ++a) {
        P.lo[a] = (float)d.box_lo[a];
        P.hi[a] = (float)d.box_hi[a];
    }
    P.open_face = d.open_face;
    if (d.geometry == FPT_GEOM_BOX) {
        const int ax = d.open_face >> 1;
        const int a1 = ax == 2 ? 0 : ax + 1, a2 = ax == 0 ? 2 : ax - 1;
        for (int c = 0; c < 3; ++c) {
            P.vis_e[0][c] = c == ax ? 1.f : 0.f;
            P.vis_e[1][c] = c == a1 ? 1.f : 0.f;
            P.vis_e[2][c] = c == a2 ? 1.f : 0.f;
        }
        P.vis_plane = (d.open_face & 1) ? P.hi[ax] : P.lo[ax];
        P.vis_lo1 = P.lo[a1];
        P.vis_hi1 = P.hi[a1];
        P.vis_lo2 = P.lo[a2];
        P.vis_hi2 = P.hi[a2];
    }
    P.n_spheres = d.geometry == FPT_GEOM_BOX ? d.n_spheres : 0;
    for (int s = 0; s < P.n_spheres; ++s) {
        for (int a = 0; a < 3; ++a) P.spheres[s].c[a] = (float)d.spheres[s].center[a];
        P.spheres[s].r2 = (float)(d.spheres[s].radius * d.spheres[s].radius);
        P.spheres[s].medium = d.spheres[s].medium;
        P.spheres[s].st_row = P.off_st + 2 * d.spheres[s].medium * N;
    }
    double dir[3] = {d.light_dir[0], d.light_dir[1], d.light_dir[2]};
    if (d.light == FPT_LIGHT_BEAM) norm3(dir);
    for (int a = 0; a < 3; ++a) {
        P.lpos[a] = (float)d.light_pos[a];
        P.ldir[a] = (float)dir[a];
        P.lu[a] = (float)d.light_u[a];
        P.lv[a] = (float)d.light_v[a];
    }
    if (d.light == FPT_LIGHT_QUAD) {
        double n[3], t1[3] = {d.light_u[0], d.light_u[1], d.light_u[2]}, t2[3];
        cross3(d.light_u, d.light_v, n);
        norm3(n);
        norm3(t1);
        cross3(n, t1, t2);
        for (int a = 0; a < 3; ++a) {
            P.ln[a] = (float)n[a];
            P.lt1[a] = (float)t1[a];
            P.lt2[a] = (float)t2[a];
        }
        P.lu_inv2 = (float)(1.0 / (d.light_u[0] * d.light_u[0] + d.light_u[1] * d.light_u[1] + d.light_u[2] * d.light_u[2]));
        P.lv_inv2 = (float)(1.0 / (d.light_v[0] * d.light_v[0] + d.light_v[1] * d.light_v[1] + d.light_v[2] * d.light_v[2]));
    }
    if (d.sensor == FPT_SENSOR_PINHOLE) {
        double f[3] = {d.look[0] - d.eye[0], d.look[1] - d.eye[1], d.look[2] - d.eye[2]}, r[3], u[3];
        norm3(f);
        cross3(f, d.up, r);
        norm3(r);
        cross3(r, f, u);
        const double ty = std::tan(0.5 * d.fov_y_deg * M_PI / 180.0);
        const double tx = ty * d.width / d.height;
        for (int a = 0; a < 3; ++a) {
            P.eye[a] = (float)d.eye[a];
            P.cf[a] = (float)f[a];
            P.cr[a] = (float)r[a];
            P.cu[a] = (float)u[a];
        }
        P.inv_tanx = (float)(1.0 / tx);
        P.inv_tany = (float)(1.0 / ty);
        P.tanx = (float)tx;
        P.tany = (float)ty;
        P.W = d.width;
        P.H = d.height;
        P.splat_norm = (float)((double)d.width * d.height / (4.0 * tx * ty));
    }
    P.np = np;
    P.geo_clear = cam ? clear_spheres(d) : 0u;
    P.tau_zero = kTauZero;
    P.sph_clear = P.geo_clear & opaque_capable(d, sc->h_st, kTauZero);
    sphere_occluders(d, P.sph_occl);
    return FPT_OK;
}

int32_t upload_tables(fpt_scene* sc) {
    const size_t bytes = sc->image.size() * 4;
    if (!sc->d_tables) HIP_TRY(dev_malloc((void**)&sc->d_tables, std::max<size_t>(bytes, 4)), "hipMalloc(tables)");
    HIP_TRY(hipMemcpy(sc->d_tables, sc->image.data(), bytes, hipMemcpyHostToDevice), "upload tables");
    return FPT_OK;
}

int64_t film_elems(const fpt_scene_desc& d, uint32_t B) {
    if (d.sensor == FPT_SENSOR_PINHOLE) return (int64_t)B * 2 * d.height * (int64_t)d.width * d.n_bins;
    return (int64_t)B * 2 * 2 * d.n_bins;
}

int32_t check_run(const fpt_scene* sc, const fpt_run* run, uint32_t* B) {
    if (!run) return set_err(FPT_E_INVALID, "run is NULL");
    if (run->total_paths == 0 || run->total_paths > (1ull << 32))
        return set_err(FPT_E_RANGE, "total_paths must be in [1, 2^32]");
    if (run->path_begin > run->total_paths || run->path_count > run->total_paths - run->path_begin)
        return set_err(FPT_E_RANGE, "path range outside total_paths");
    // path ids are 32-bit: a job of 2^32 paths is rendered in at least two calls
    if (run->path_count > 0xFFFFFFFFull) return set_err(FPT_E_RANGE, "path_count must be below 2^32");
    const uint32_t b = run->parity_batches ? run->parity_batches : 1u;
    if (b > 64) return set_err(FPT_E_RANGE, "parity_batches %u > 64", b);
    if (!(run->splat_rr >= 0.0 && run->splat_rr <= 1.0)) return set_err(FPT_E_RANGE, "splat_rr outside [0,1]");
    if (run->flags & ~(FPT_FLAG_FLUORESCENCE_ONLY | FPT_FLAG_NO_EXCITATION_SCATTER))
        return set_err(FPT_E_INVALID, "unknown run flags 0x%x", run->flags);
    (void)sc;
    *B = b;
    return FPT_OK;
}

// The optical depth from which a medium vertex's pinhole connection deposits
// exactly 0 in fp32.  The kernels form the deposit as wscale * f * tr * ...
// from the left, f = 1/(4 pi) in a medium; once the first product
// (wscale f) tr is below 2^-150 it rounds to 0, and so does every later
// product (all other factors are finite for the clear spheres the shortcut
// applies to).  With tr = exp(-tau) to a few ulps that holds for
// tau >= ln(wscale f) + 150 ln 2; 0.5 of margin covers the fp32 evaluation of
// tau (the connection's own-sphere chord; other spheres only add to it).  With
// connection roulette (splat_rr > 0) a transmittance that is not exactly 0
// takes part in the roulette, so the threshold stays kTauZero.
float exact_zero_depth(const KParams& P) {
    if (P.splat_rr > 0.f) return kTauZero;
    const float a = P.wscale * 0.0795774715459476679f;  // fp32, as the kernels form it
    if (!(a > 0.f)) return kTauZero;
    const double t = std::log((double)a) + 150.0 * std::log(2.0) + 0.5;
    return (float)std::min(t, (double)kTauZero);
}

void fill_run(const fpt_scene* sc, const fpt_run* run, uint32_t B, KParams* P) {
    *P = sc->base;
    P->key0 = (uint32_t)run->seed;
    P->key1 = (uint32_t)(run->seed >> 32) ^ run->instance;
    P->path_begin = (uint32_t)run->path_begin;
    P->path_count = (uint32_t)run->path_count;  // below 2^32 (check_run)
    P->batches = B;
    // film element indices below 2^32 - 1: deposits merge per wave
    P->film_u32 = sc->desc.sensor == FPT_SENSOR_PINHOLE &&
                  (int64_t)B * 2 * sc->desc.height * (int64_t)sc->desc.width * sc->desc.n_bins < 0xFFFFFFFFll;
    P->wscale = (float)((double)B / (double)run->total_paths);
    P->max_scatter = run->max_scatter;
    P->max_emissions = run->max_emissions;
    P->fluo_only = (run->flags & FPT_FLAG_FLUORESCENCE_ONLY) ? 1 : 0;
    P->exc_scatter = (run->flags & FPT_FLAG_NO_EXCITATION_SCATTER) ? 0 : 1;
    P->splat_rr = (float)run->splat_rr;
    P->inv_splat_rr = run->splat_rr > 0.0 ? (float)(1.0 / run->splat_rr) : 0.f;
    P->max_vertices = 0;
    // defaults measured on MI355X: refill once most lanes are free, walk paths
    // in media in wave blocks from their second vertex (pinhole scenes) or
    // eighth (escape sensors), up to four paths per block round
    const bool pin = sc->desc.sensor == FPT_SENSOR_PINHOLE;
    P->refill_lanes = sc->tune.refill_lanes > 0 ? std::min(64, sc->tune.refill_lanes) : (pin ? 48 : 60);
    // escape films up to 8192 counters use a per-block LDS histogram
    const int64_t hw = sc->desc.sensor == FPT_SENSOR_ESCAPE ? film_elems(sc->desc, B) : 0;
    P->hist_words = hw <= 8192 ? (int)hw : 0;
    P->block_min_v = sc->tune.block_min_vertices > 0 ? (uint32_t)sc->tune.block_min_vertices : (pin ? 2u : 8u);
    P->max_segments = sc->tune.block_segments > 0 ? sc->tune.block_segments : 4;
    P->wide_rounds = sc->tune.wide_rounds < 0 ? 0 : (sc->tune.wide_rounds > 0 ? sc->tune.wide_rounds : (pin ? 1 : 2));
    P->tau_zero = exact_zero_depth(*P);
    P->sph_clear = P->geo_clear & opaque_capable(sc->desc, sc->h_st, P->tau_zero);
}

// Deferred-connection entries per transport wave (20 bytes each).
constexpr uint32_t kSjobSlice = 2048;

// Largest persistent grid (blocks) and wave count of a transport launch in
// `mode` over every block size a tune may ask for, at the kernel's occupancy on
// this device; 0 where the scene's tables do not fit in LDS for that mode.
int32_t max_launch(const fpt_scene* sc, const KParams& P0, int mode, size_t* blocks, size_t* waves) {
    KParams P = P0;
    P.hist_words = 0;  // the LDS histogram only lowers occupancy
    *blocks = *waves = 0;
    for (int b = 64; b <= 256; b += 64) {
        if (transport_lds_bytes(P, b, mode) > 160u * 1024u) continue;
        int per_cu = 0;
        HIP_TRY(transport_occupancy(P, mode, b, &per_cu), "occupancy query");
        const size_t g = (size_t)sc->n_cu * (size_t)std::max(per_cu, 1);
        *blocks = std::max(*blocks, g);
        *waves = std::max(*waves, g * (size_t)(b / 64));
    }
    return FPT_OK;
}

// Device scratch of a scene, sized once for every launch it can make.
int32_t reserve_scratch(fpt_scene* sc) {
    HIP_TRY(dev_malloc((void**)&sc->d_counter, queue_words() * 8), "hipMalloc(path queue)");
    if (sc->desc.sensor == FPT_SENSOR_ESCAPE) {
        sc->counts_words = (size_t)film_elems(sc->desc, 64);
        HIP_TRY(dev_malloc((void**)&sc->d_counts, sc->counts_words * 4), "hipMalloc(counts)");
    }
    fpt_run r;
    std::memset(&r, 0, sizeof r);
    r.path_count = r.total_paths = 1;
    KParams P;
    fill_run(sc, &r, 1, &P);
    size_t blocks = 0, waves = 0;
    int32_t rc = max_launch(sc, P, MODE_ADJ, &blocks, &waves);
    if (rc != FPT_OK) return rc;
    if (blocks) {
        HIP_TRY(dev_malloc((void**)&sc->d_partials, blocks * kMaxNP * 4), "hipMalloc(partials)");
        sc->partials_blocks = blocks;
    }
    if (sc->desc.geometry == FPT_GEOM_BOX && sc->desc.sensor == FPT_SENSOR_PINHOLE) {
        if ((rc = max_launch(sc, P, MODE_FWD, &blocks, &waves)) != FPT_OK) return rc;
        if (waves) {
            HIP_TRY(dev_malloc((void**)&sc->d_sjobs, waves * kEntryWords * kSjobSlice * 4),
                    "hipMalloc(deferred splats)");
            HIP_TRY(dev_malloc((void**)&sc->d_sjob_counts, waves * 4), "hipMalloc(deferred splat counts)");
            sc->sjob_waves = waves;
        }
    }
    HIP_TRY(pinned_malloc((void**)&sc->h_stage, std::max<size_t>(4, sc->image.size() * 4)),
            "hipHostMalloc(table staging)");
    HIP_TRY(hipEventCreateWithFlags(&sc->staged, hipEventDisableTiming), "hipEventCreate");
    return FPT_OK;
}

// Grid for a persistent launch: fill every CU at the kernel's occupancy, but
// never more lanes than paths.
int32_t grid_for(fpt_scene* sc, const KParams& P, int mode, int block, uint64_t paths, int* grid) {
    int per_cu = 0;
    HIP_TRY(transport_occupancy(P, mode, block, &per_cu), "occupancy query");
    if (sc->tune.blocks_per_cu > 0) per_cu = std::min(per_cu, sc->tune.blocks_per_cu);
    per_cu = std::max(per_cu, 1);
    const uint64_t full = (uint64_t)sc->n_cu * per_cu;
    const uint64_t need = (paths + block - 1) / block;
    *grid = (int)std::max<uint64_t>(1, std::min(full, need));
    return FPT_OK;
}

// The three events of the next timed render (fpt_scene_set_timing), or null.
int32_t timing_slot(fpt_scene* sc, hipEvent_t** ev) {
    *ev = nullptr;
    if (!sc->timing || sc->timed >= FPT_MAX_TIMED_RENDERS) return FPT_OK;
    while (sc->events.size() < (size_t)(sc->timed + 1) * 3) {
        hipEvent_t e;
        HIP_TRY(hipEventCreate(&e), "hipEventCreate");
        sc->events.push_back(e);
    }
    *ev = &sc->events[(size_t)sc->timed * 3];
    ++sc->timed;
    return FPT_OK;
}

int block_for(const fpt_scene* sc) {
    int b = sc->tune.block_threads > 0 ? sc->tune.block_threads : 256;
    b = std::max(64, std::min(256, (b / 64) * 64));
    return b;
}

// LDS one workgroup may allocate on gfx950.
constexpr size_t kLdsLimit = 160u * 1024u;

// Block size of a transport launch: the tuned one, halved (to 128, then 64
// threads) while the table image and the per-wave LDS areas do not fit; a scene
// whose image does not fit beside even one wave is refused before any launch.
int32_t transport_block(const fpt_scene* sc, const KParams& P, int mode, int* block) {
    int b = block_for(sc);
    while (b > 64 && transport_lds_bytes(P, b, mode) > kLdsLimit) b = b > 128 ? 128 : 64;
    size_t need = transport_lds_bytes(P, b, mode);
    // forward pinhole renders also launch the deferred-connection kernel (four waves)
    if (mode == MODE_FWD && P.geometry == FPT_GEOM_BOX && P.sensor == FPT_SENSOR_PINHOLE)
        need = std::max(need, splat_jobs_lds_bytes(P));
    if (need > kLdsLimit)
        return set_err(FPT_E_UNSUPPORTED, "table image of %d words needs %zu bytes of LDS per workgroup (limit %zu)",
                       P.table_words, need, kLdsLimit);
    *block = b;
    return FPT_OK;
}

}  // namespace

struct fpt_batch {
    int n = 0, N = 0, hist_words = 0, max_table_words = 0;
    int device = 0, n_cu = 256, grid = 1, block = 256;
    uint64_t total_paths = 0;
    fpt_tune tune;
    std::vector<KParams> params;
    std::vector<double> cost;
    std::vector<uint32_t> path_counts;
    std::vector<float> wscale;
    KParams* d_params = nullptr;
    uint32_t* d_tables = nullptr;
    uint32_t* d_toff = nullptr;
    float* d_wscale = nullptr;
    uint32_t* d_counts = nullptr;
    unsigned long long* d_counter = nullptr;
    KWorkItem* d_items = nullptr;
    size_t items_cap = 0;
    KBatch kbatch;
    hipStream_t cap_stream = nullptr;
    hipGraph_t graph = nullptr;
    hipGraphExec_t exec = nullptr;
    float* g_films = nullptr;
    uint64_t* g_tallies = nullptr;
};

namespace {

// (Re)builds the work-item queue and launch shape from the batch's tune: items
// of chunk_paths paths, instances in decreasing expected cost.
int32_t batch_build_items(fpt_batch* bt) {
    const uint32_t chunk = bt->tune.chunk_paths > 0 ? (uint32_t)bt->tune.chunk_paths : 4096u;
    std::vector<int> order((size_t)bt->n);
    for (int i = 0; i < bt->n; ++i) order[i] = i;
    std::stable_sort(order.begin(), order.end(), [&](int a, int b) { return bt->cost[a] > bt->cost[b]; });
    std::vector<KWorkItem> items;
    for (int i : order) {
        for (uint32_t lo = 0; lo < bt->path_counts[i]; lo += chunk) {
            KWorkItem w;
            w.instance = (uint32_t)i;
            w.path_lo = lo;
            w.path_hi = std::min<uint32_t>(bt->path_counts[i], lo + chunk);
            w.pad = 0;
            items.push_back(w);
        }
    }
    if (items.size() > bt->items_cap) {
        if (bt->d_items) (void)hipFree(bt->d_items);
        bt->d_items = nullptr;
        bt->items_cap = 0;
        HIP_TRY(dev_malloc((void**)&bt->d_items, std::max<size_t>(1, items.size()) * sizeof(KWorkItem)),
                "hipMalloc(items)");
        bt->items_cap = items.size();
    }
    if (!items.empty())
        HIP_TRY(hipMemcpy(bt->d_items, items.data(), items.size() * sizeof(KWorkItem), hipMemcpyHostToDevice),
                "upload items");
    const int refill = bt->tune.refill_lanes > 0 ? std::min(64, bt->tune.refill_lanes) : 8;
    const uint32_t bmin = bt->tune.block_min_vertices > 0 ? (uint32_t)bt->tune.block_min_vertices : 64u;
    const int segs = bt->tune.block_segments > 0 ? bt->tune.block_segments : 2;
    for (KParams& p : bt->params) {
        p.refill_lanes = refill;
        p.block_min_v = bmin;
        p.max_segments = segs;
        p.wide_rounds = bt->tune.wide_rounds < 0 ? 0 : (bt->tune.wide_rounds > 0 ? bt->tune.wide_rounds : 1);
    }
    HIP_TRY(hipMemcpy(bt->d_params, bt->params.data(), sizeof(KParams) * bt->n, hipMemcpyHostToDevice),
            "upload params");
    KBatch& K = bt->kbatch;
    std::memset(&K, 0, sizeof K);
    K.params = bt->d_params;
    K.tables = bt->d_tables;
    K.table_off = bt->d_toff;
    K.items = bt->d_items;
    K.n_items = (int)items.size();
    K.n_instances = bt->n;
    K.hist_words = bt->hist_words;
    K.slot_words = batch_slot_words(bt->hist_words, bt->max_table_words);
    K.counts = bt->d_counts;
    K.item_counter = bt->d_counter;
    K.refractive = 0;
    for (int i = 0; i < bt->n; ++i)
        if (bt->params[i].ior != 1.f) K.refractive = 1;
    int b = bt->tune.block_threads > 0 ? bt->tune.block_threads : 256;
    b = std::max(64, std::min(256, (b / 64) * 64));
    // every wave holds a whole slot (tables, histogram, tally): fewer waves
    // per block where the slots of the tuned size do not fit
    while (b > 64 && batch_lds_bytes(K, b) > kLdsLimit) b = b > 128 ? 128 : 64;
    if (batch_lds_bytes(K, b) > kLdsLimit)
        return set_err(FPT_E_UNSUPPORTED, "instance slot of %d words needs %zu bytes of LDS (limit %zu)",
                       K.slot_words, batch_lds_bytes(K, b), kLdsLimit);
    bt->block = b;
    int per_cu = 0;
    HIP_TRY(batch_occupancy(K, bt->block, &per_cu), "batch occupancy");
    if (bt->tune.blocks_per_cu > 0) per_cu = std::min(per_cu, bt->tune.blocks_per_cu);
    bt->grid = std::max(1, bt->n_cu * std::max(per_cu, 1));
    // a new launch shape invalidates a captured graph
    if (bt->exec) (void)hipGraphExecDestroy(bt->exec);
    if (bt->graph) (void)hipGraphDestroy(bt->graph);
    bt->exec = nullptr;
    bt->graph = nullptr;
    bt->g_films = nullptr;
    return FPT_OK;
}

}  // namespace

extern "C" {

uint32_t fpt_abi_version(void) { return FPT_ABI_VERSION; }

const char* fpt_status_str(int32_t s) {
    switch (s) {
    case FPT_OK: return "ok";
    case FPT_E_INVALID: return "invalid argument";
    case FPT_E_RANGE: return "value out of range";
    case FPT_E_NOMEM: return "out of memory";
    case FPT_E_DEVICE: return "device error";
    case FPT_E_UNSUPPORTED: return "unsupported";
    default: return "unknown status";
    }
}

const char* fpt_last_error(void) { return g_err.c_str(); }

}  // extern "C"

namespace {

// fpt_scene_create without its exception and fault-injection wrapper: `held`
// owns the scene until it is handed out, so every failure path (a status, or
// a host allocation failure thrown by the table build) frees all of it.
struct SceneHold {
    fpt_scene* p = nullptr;
    ~SceneHold() { if (p) fpt_scene_destroy(p); }
};

int32_t scene_create(const fpt_scene_desc* desc, fpt_scene** out, SceneHold& held) {
    int32_t rc = validate(desc);
    if (rc != FPT_OK) return rc;
    fpt_scene* sc = held.p = new_object<fpt_scene>();
    if (!sc) return set_err(FPT_E_NOMEM, "host allocation");
    sc->desc = *desc;
    // tabulated spectra are borrowed for the call: keep copies and point at them
    auto own = [sc](fpt_spectrum& s) {
        if (s.kind != FPT_SPECTRUM_TABULATED) return;
        sc->tabs.emplace_back(s.table, s.table + s.n);
        s.table = sc->tabs.back().data();
    };
    for (int i = 0; i < sc->desc.n_dyes; ++i) {
        own(sc->desc.dyes[i].absorption);
        own(sc->desc.dyes[i].emission);
    }
    for (int f = 0; f < 6; ++f) own(sc->desc.walls[f]);
    std::memset(&sc->tune, 0, sizeof sc->tune);
    if ((rc = build_tables(sc)) != FPT_OK) return rc;
    HIP_TRY(hipGetDevice(&sc->device), "device query");
    HIP_TRY(hipDeviceGetAttribute(&sc->n_cu, hipDeviceAttributeMultiprocessorCount, sc->device), "device query");
    if ((rc = upload_tables(sc)) != FPT_OK || (rc = reserve_scratch(sc)) != FPT_OK) return rc;
    *out = sc;
    held.p = nullptr;
    return FPT_OK;
}

}  // namespace

extern "C" {

int32_t fpt_scene_create(const fpt_scene_desc* desc, fpt_scene** out) {
    if (!desc || !out) return set_err(FPT_E_INVALID, "NULL argument");
    *out = nullptr;
    alloc_fault_arm(true);
    int32_t rc;
    try {
        SceneHold held;
        rc = scene_create(desc, out, held);
    } catch (const std::bad_alloc&) {
        rc = set_err(FPT_E_NOMEM, "host allocation");
    }
    alloc_fault_arm(false);
    return rc;
}

void fpt_scene_destroy(fpt_scene* sc) {
    if (!sc) return;
    if (sc->d_tables) (void)hipFree(sc->d_tables);
    if (sc->d_counts) (void)hipFree(sc->d_counts);
    if (sc->d_counter) (void)hipFree(sc->d_counter);
    if (sc->d_partials) (void)hipFree(sc->d_partials);
    if (sc->staged) {
        (void)hipEventSynchronize(sc->staged);
        (void)hipEventDestroy(sc->staged);
    }
    if (sc->h_stage) (void)hipHostFree(sc->h_stage);
    if (sc->d_sjobs) (void)hipFree(sc->d_sjobs);
    if (sc->d_sjob_counts) (void)hipFree(sc->d_sjob_counts);
    for (hipEvent_t e : sc->events) (void)hipEventDestroy(e);
    delete sc;
}

int32_t fpt_scene_set_params(fpt_scene* sc, const double* conc, const double* qy, const double* sigma_s,
                             void* stream) {
    if (!sc) return set_err(FPT_E_INVALID, "NULL scene");
    fpt_scene_desc d = sc->desc;
    int k = 0;
    for (int m = 0; m < d.n_media; ++m)
        for (int j = 0; j < d.media[m].n_dyes; ++j, ++k)
            if (conc) d.media[m].conc_uM[j] = conc[k];
    if (qy)
        for (int i = 0; i < d.n_dyes; ++i) d.dyes[i].qy = qy[i];
    if (sigma_s)
        for (int m = 0; m < d.n_media; ++m) d.media[m].sigma_s_mm = sigma_s[m];
    int32_t rc = validate(&d);
    if (rc != FPT_OK) return rc;
    const fpt_scene_desc old = sc->desc;
    sc->desc = d;
    if ((rc = build_tables(sc)) != FPT_OK) {
        sc->desc = old;
        build_tables(sc);
        return rc;
    }
    // stream-ordered upload through the pinned staging buffer: launches already
    // on `stream` read the old tables, later ones the new; the host waits only
    // for the previous upload out of the staging buffer
    hipStream_t s = (hipStream_t)stream;
    HIP_TRY(hipEventSynchronize(sc->staged), "wait for the previous table upload");
    std::memcpy(sc->h_stage, sc->image.data(), sc->image.size() * 4);
    HIP_TRY(hipMemcpyAsync(sc->d_tables, sc->h_stage, sc->image.size() * 4, hipMemcpyHostToDevice, s),
            "upload tables");
    HIP_TRY(hipEventRecord(sc->staged, s), "hipEventRecord");
    return FPT_OK;
}

int32_t fpt_film_shape(const fpt_scene* sc, uint32_t batches, int64_t dims[5], int32_t* ndims) {
    if (!sc || !dims || !ndims) return set_err(FPT_E_INVALID, "NULL argument");
    const int64_t B = batches ? batches : 1;
    const fpt_scene_desc& d = sc->desc;
    if (d.sensor == FPT_SENSOR_PINHOLE) {
        dims[0] = B; dims[1] = 2; dims[2] = d.height; dims[3] = d.width; dims[4] = d.n_bins;
        *ndims = 5;
    } else {
        dims[0] = B; dims[1] = 2; dims[2] = 2; dims[3] = d.n_bins; dims[4] = 0;
        *ndims = 4;
    }
    return FPT_OK;
}

int32_t fpt_grad_param_count(const fpt_scene* sc) { return sc ? sc->np : set_err(FPT_E_INVALID, "NULL scene"); }

int32_t fpt_scene_set_timing(fpt_scene* sc, int32_t enable) {
    if (!sc) return set_err(FPT_E_INVALID, "NULL scene");
    sc->timing = enable != 0;
    sc->timed = 0;
    return FPT_OK;
}

int32_t fpt_scene_timing_each(fpt_scene* sc, int32_t cap, int32_t* renders, float* transport_ms,
                              float* deferred_ms) {
    if (!sc || !renders || (cap > 0 && (!transport_ms || !deferred_ms)) || cap < 0)
        return set_err(FPT_E_INVALID, "NULL argument");
    const int n = std::min(sc->timed, cap);
    for (int k = 0; k < sc->timed; ++k) {
        hipEvent_t* ev = &sc->events[(size_t)k * 3];
        HIP_TRY(hipEventSynchronize(ev[2]), "hipEventSynchronize");
        if (k >= n) continue;
        HIP_TRY(hipEventElapsedTime(&transport_ms[k], ev[0], ev[1]), "hipEventElapsedTime");
        HIP_TRY(hipEventElapsedTime(&deferred_ms[k], ev[1], ev[2]), "hipEventElapsedTime");
    }
    *renders = sc->timed;
    sc->timed = 0;
    return FPT_OK;
}

int32_t fpt_scene_timing(fpt_scene* sc, int32_t* renders, float* transport_ms, float* deferred_ms) {
    if (!sc || !renders || !transport_ms || !deferred_ms) return set_err(FPT_E_INVALID, "NULL argument");
    std::vector<float> t((size_t)std::max(1, sc->timed)), d((size_t)std::max(1, sc->timed));
    int32_t n = 0;
    int32_t rc = fpt_scene_timing_each(sc, sc->timed, &n, t.data(), d.data());
    if (rc != FPT_OK) return rc;
    double st = 0.0, sd = 0.0;
    for (int k = 0; k < n; ++k) {
        st += t[k];
        sd += d[k];
    }
    *renders = n;
    *transport_ms = n ? (float)(st / n) : 0.f;
    *deferred_ms = n ? (float)(sd / n) : 0.f;
    return FPT_OK;
}

int32_t fpt_scene_set_tune(fpt_scene* sc, const fpt_tune* tune) {
    if (!sc) return set_err(FPT_E_INVALID, "NULL scene");
    if (!tune) {
        std::memset(&sc->tune, 0, sizeof sc->tune);
        return FPT_OK;
    }
    if (tune->block_threads && (tune->block_threads < 64 || tune->block_threads > 256 || tune->block_threads % 64))
        return set_err(FPT_E_RANGE, "block_threads must be 64..256 in steps of 64");
    if (tune->refill_lanes < 0 || tune->refill_lanes > 64) return set_err(FPT_E_RANGE, "refill_lanes 0..64");
    if (tune->blocks_per_cu < 0) return set_err(FPT_E_RANGE, "blocks_per_cu >= 0");
    if (tune->block_segments != 0 && tune->block_segments != 1 && tune->block_segments != 2 &&
        tune->block_segments != 4)
        return set_err(FPT_E_RANGE, "block_segments must be 0, 1, 2 or 4");
    if (tune->wide_rounds < -1 || tune->wide_rounds > 2) return set_err(FPT_E_RANGE, "wide_rounds must be -1..2");
    sc->tune = *tune;
    return FPT_OK;
}

int32_t fpt_scene_tables(const fpt_scene* sc, float* sigma_t, float* emis_cdf, float* rho, int32_t* line_bin) {
    if (!sc) return set_err(FPT_E_INVALID, "NULL scene");
    if (sigma_t) std::memcpy(sigma_t, sc->h_st.data(), sc->h_st.size() * 4);
    if (emis_cdf) std::memcpy(emis_cdf, sc->h_cdf.data(), (size_t)sc->desc.n_dyes * sc->desc.n_bins * 4);
    if (rho) std::memcpy(rho, sc->h_rho.data(), sc->h_rho.size() * 4);
    if (line_bin)
        for (size_t i = 0; i < sc->h_line_bin.size(); ++i) line_bin[i] = sc->h_line_bin[i];
    return FPT_OK;
}

int32_t fpt_scene_connection_masks(const fpt_scene* sc, uint32_t* geo_clear, uint32_t* occluders) {
    if (!sc) return set_err(FPT_E_INVALID, "NULL scene");
    if (geo_clear) *geo_clear = sc->base.geo_clear;
    if (occluders)
        for (int s = 0; s < FPT_MAX_SPHERES; ++s) occluders[s] = s < sc->desc.n_spheres ? sc->base.sph_occl[s] : 0u;
    return FPT_OK;
}

int32_t fpt_render(fpt_scene* sc, const fpt_run* run, float* film, uint64_t* tallies, void* stream) {
    if (!sc || !film) return set_err(FPT_E_INVALID, "NULL argument");
    uint32_t B;
    int32_t rc = check_run(sc, run, &B);
    if (rc != FPT_OK) return rc;
    if (run->path_count == 0) return FPT_OK;
    hipStream_t s = (hipStream_t)stream;
    KParams P;
    fill_run(sc, run, B, &P);
    const bool escape = sc->desc.sensor == FPT_SENSOR_ESCAPE;
    const size_t n_counts = escape ? (size_t)film_elems(sc->desc, B) : 0;
    int block;
    if ((rc = transport_block(sc, P, MODE_FWD, &block)) != FPT_OK) return rc;
    if (n_counts > sc->counts_words) return set_err(FPT_E_RANGE, "escape film of %zu counters", n_counts);
    int grid;
    if ((rc = grid_for(sc, P, MODE_FWD, block, run->path_count, &grid)) != FPT_OK) return rc;
    KBuffers Bf;
    std::memset(&Bf, 0, sizeof Bf);
    Bf.tables = sc->d_tables;
    Bf.film = film;
    Bf.counts = sc->d_counts;
    Bf.tallies = tallies ? reinterpret_cast<unsigned long long*>(tallies) : nullptr;
    Bf.counter = sc->d_counter;
    const bool defer = sc->desc.sensor == FPT_SENSOR_PINHOLE;
    const size_t waves = (size_t)grid * (block / 64);
    if (defer) {
        // slices were reserved for the largest wave count at scene creation
        if (waves > sc->sjob_waves)
            return set_err(FPT_E_DEVICE, "%zu transport waves exceed the %zu reserved", waves, sc->sjob_waves);
        Bf.sjobs = sc->d_sjobs;
        Bf.sjob_counts = sc->d_sjob_counts;
        Bf.sjob_slice = kSjobSlice;
    }
    HIP_TRY(launch_zero_u64(sc->d_counter, queue_words(), s), "zero queue");
    if (escape) HIP_TRY(launch_zero_u32(sc->d_counts, n_counts, s), "zero counts");
    hipEvent_t* ev = nullptr;
    if ((rc = timing_slot(sc, &ev)) != FPT_OK) return rc;
    if (ev) HIP_TRY(hipEventRecord(ev[0], s), "hipEventRecord");
    HIP_TRY(launch_transport(P, Bf, MODE_FWD, grid, block, s), "transport launch");
    if (ev) HIP_TRY(hipEventRecord(ev[1], s), "hipEventRecord");
    if (defer) HIP_TRY(launch_splat_jobs(P, Bf, (int)waves, s), "deferred splats");
    if (ev) HIP_TRY(hipEventRecord(ev[2], s), "hipEventRecord");
    if (escape) HIP_TRY(launch_finalize_counts(sc->d_counts, film, n_counts, P.wscale, s), "finalize");
    return FPT_OK;
}

int32_t fpt_render_noalloc(fpt_scene* sc, const fpt_run* run, float* film, uint64_t* tallies, void* stream) {
    if (!sc || !film) return set_err(FPT_E_INVALID, "NULL argument");
    uint32_t B;
    int32_t rc = check_run(sc, run, &B);
    if (rc != FPT_OK) return rc;
    if (run->path_count == 0) return FPT_OK;
    hipStream_t s = (hipStream_t)stream;
    KParams P;
    fill_run(sc, run, B, &P);
    const bool escape = sc->desc.sensor == FPT_SENSOR_ESCAPE;
    const size_t n_counts = escape ? (size_t)film_elems(sc->desc, B) : 0;
    int block;
    if ((rc = transport_block(sc, P, MODE_FWD, &block)) != FPT_OK) return rc;
    int grid;
    if ((rc = grid_for(sc, P, MODE_FWD, block, run->path_count, &grid)) != FPT_OK) return rc;
    const bool defer = sc->desc.sensor == FPT_SENSOR_PINHOLE;
    const size_t waves = (size_t)grid * (block / 64);
    // the static scratch on this device: queue heads | counts per wave | escape
    // counters | deferred slices (each part 256-byte aligned)
    void* base = nullptr;
    size_t cap = 0;
    HIP_TRY(static_scratch(&base, &cap), "static scratch address");
    auto up = [](size_t b) { return (b + 255) & ~(size_t)255; };
    const size_t q_bytes = up(queue_words() * 8);
    const size_t c_bytes = defer ? up(waves * 4) : 0;
    const size_t e_bytes = up(n_counts * 4);
    const size_t fixed = q_bytes + c_bytes + e_bytes;
    if (fixed > cap)
        return set_err(FPT_E_RANGE, "escape film of %zu counters exceeds the %zu-byte static scratch", n_counts, cap);
    char* b = static_cast<char*>(base);
    KBuffers Bf;
    std::memset(&Bf, 0, sizeof Bf);
    Bf.tables = sc->d_tables;
    Bf.film = film;
    Bf.counter = reinterpret_cast<unsigned long long*>(b);
    Bf.counts = escape ? reinterpret_cast<uint32_t*>(b + q_bytes + c_bytes) : nullptr;
    Bf.tallies = tallies ? reinterpret_cast<unsigned long long*>(tallies) : nullptr;
    uint32_t slice = 0;
    if (defer) {
        // deferred slices shrink to what is left (a full slice falls back to
        // the wave's LDS queue, so the film changes only in fp32 rounding order)
        const size_t per = (cap - fixed) / (waves * kEntryWords * 4);
        slice = (uint32_t)std::min<size_t>(kSjobSlice, per & ~(size_t)63);
        if (slice > 0) {
            Bf.sjob_counts = reinterpret_cast<uint32_t*>(b + q_bytes);
            Bf.sjobs = reinterpret_cast<uint32_t*>(b + fixed);
            Bf.sjob_slice = slice;
        }
    }
    HIP_TRY(launch_zero_u64(Bf.counter, queue_words(), s), "zero queue");
    if (escape) HIP_TRY(launch_zero_u32(Bf.counts, n_counts, s), "zero counts");
    HIP_TRY(launch_transport(P, Bf, MODE_FWD, grid, block, s), "transport launch");
    if (slice > 0) HIP_TRY(launch_splat_jobs(P, Bf, (int)waves, s), "deferred splats");
    if (escape) HIP_TRY(launch_finalize_counts(Bf.counts, film, n_counts, P.wscale, s), "finalize");
    return FPT_OK;
}

int32_t fpt_render_adjoint(fpt_scene* sc, const fpt_run* run, const float* gfilm, float* grad,
                           uint64_t* tallies, void* stream) {
    if (!sc || !gfilm || !grad) return set_err(FPT_E_INVALID, "NULL argument");
    uint32_t B;
    int32_t rc = check_run(sc, run, &B);
    if (rc != FPT_OK) return rc;
    if (sc->np > kMaxNP) return set_err(FPT_E_UNSUPPORTED, "%d gradient parameters > %d", sc->np, kMaxNP);
    if (run->path_count == 0) return FPT_OK;
    hipStream_t s = (hipStream_t)stream;
    KParams P;
    fill_run(sc, run, B, &P);
    // adjoint defaults measured on MI355X (256x256, 256 spp Cornell job): blocks
    // from a path's eighth vertex in a medium and refills at 32 dead lanes take
    // 4.95 ms against 5.45 ms with the forward's pinhole defaults (2 and 48)
    if (sc->desc.sensor == FPT_SENSOR_PINHOLE) {
        if (sc->tune.block_min_vertices <= 0) P.block_min_v = 8u;
        if (sc->tune.refill_lanes <= 0) P.refill_lanes = 32;
    }
    int block;
    if ((rc = transport_block(sc, P, MODE_ADJ, &block)) != FPT_OK) return rc;
    int grid;
    if ((rc = grid_for(sc, P, MODE_ADJ, block, run->path_count, &grid)) != FPT_OK) return rc;
    if ((size_t)grid > sc->partials_blocks)
        return set_err(FPT_E_DEVICE, "%d adjoint blocks exceed the %zu reserved", grid, sc->partials_blocks);
    KBuffers Bf;
    std::memset(&Bf, 0, sizeof Bf);
    Bf.tables = sc->d_tables;
    Bf.tallies = tallies ? reinterpret_cast<unsigned long long*>(tallies) : nullptr;
    Bf.counter = sc->d_counter;
    Bf.gfilm = gfilm;
    Bf.partials = sc->d_partials;
    HIP_TRY(launch_zero_u64(sc->d_counter, queue_words(), s), "zero queue");
    HIP_TRY(launch_transport(P, Bf, MODE_ADJ, grid, block, s), "adjoint launch");
    HIP_TRY(launch_reduce_partials(sc->d_partials, grid, sc->np, grad, s), "gradient reduction");
    return FPT_OK;
}

int32_t fpt_render_records(fpt_scene* sc, const fpt_run* run, fpt_path_record* rec, uint32_t max_vertices,
                           const float* gfilm, float* rec_grad, void* stream) {
    if (!sc || !rec) return set_err(FPT_E_INVALID, "NULL argument");
    if ((gfilm == nullptr) != (rec_grad == nullptr))
        return set_err(FPT_E_INVALID, "grad_film and rec_grad go together");
    uint32_t B;
    int32_t rc = check_run(sc, run, &B);
    if (rc != FPT_OK) return rc;
    if (gfilm && sc->np > kMaxNP) return set_err(FPT_E_UNSUPPORTED, "too many gradient parameters");
    if (run->path_count == 0) return FPT_OK;
    hipStream_t s = (hipStream_t)stream;
    KParams P;
    fill_run(sc, run, B, &P);
    P.max_vertices = max_vertices;
    const int mode = gfilm ? MODE_REC_ADJ : MODE_REC;
    int block;
    if ((rc = transport_block(sc, P, mode, &block)) != FPT_OK) return rc;
    int grid;
    if ((rc = grid_for(sc, P, mode, block, run->path_count, &grid)) != FPT_OK) return rc;
    KBuffers Bf;
    std::memset(&Bf, 0, sizeof Bf);
    Bf.tables = sc->d_tables;
    Bf.counter = sc->d_counter;
    Bf.gfilm = gfilm;
    Bf.rec = rec;
    Bf.rec_grad = rec_grad;
    HIP_TRY(launch_zero_u64(sc->d_counter, queue_words(), s), "zero queue");
    HIP_TRY(launch_transport(P, Bf, mode, grid, block, s), "records launch");
    return FPT_OK;
}

int32_t fpt_render_camera(fpt_scene* sc, const fpt_run* run, float* film, uint64_t* tallies,
                          fpt_path_record* rec, uint32_t max_vertices, void* stream) {
    if (!sc || (!film && !rec)) return set_err(FPT_E_INVALID, "NULL argument");
    const fpt_scene_desc& d = sc->desc;
    if (d.geometry != FPT_GEOM_BOX || d.sensor != FPT_SENSOR_PINHOLE)
        return set_err(FPT_E_UNSUPPORTED, "the camera-side estimator needs a box scene with a pinhole");
    if (sc->base.glossy) return set_err(FPT_E_UNSUPPORTED, "the camera-side estimator has Lambertian walls only");
    uint32_t B;
    int32_t rc = check_run(sc, run, &B);
    if (rc != FPT_OK) return rc;
    const uint64_t per_sample = (uint64_t)d.width * (uint64_t)d.height * (uint64_t)d.n_bins;
    if (run->total_paths % per_sample != 0)
        return set_err(FPT_E_RANGE, "total_paths must be spp * width * height * n_bins");
    if (run->path_count == 0) return FPT_OK;
    hipStream_t s = (hipStream_t)stream;
    KParams P;
    fill_run(sc, run, B, &P);
    P.wscale = (float)((double)B / (double)(run->total_paths / per_sample));
    P.max_vertices = max_vertices;
    P.refill_lanes = sc->tune.refill_lanes > 0 ? std::min(64, sc->tune.refill_lanes) : 32;
    if (camera_lds_bytes(P) > kLdsLimit)
        return set_err(FPT_E_UNSUPPORTED, "table image of %d words needs %zu bytes of LDS per workgroup (limit %zu)",
                       P.table_words, camera_lds_bytes(P), kLdsLimit);
    const bool records = rec != nullptr;
    const int block = block_for(sc);
    int per_cu = 0;
    HIP_TRY(camera_occupancy(P, records, block, &per_cu), "occupancy query");
    if (sc->tune.blocks_per_cu > 0) per_cu = std::min(per_cu, sc->tune.blocks_per_cu);
    per_cu = std::max(per_cu, 1);
    const uint64_t need = (run->path_count + block - 1) / block;
    const int grid = (int)std::max<uint64_t>(1, std::min<uint64_t>((uint64_t)sc->n_cu * per_cu, need));
    KBuffers Bf;
    std::memset(&Bf, 0, sizeof Bf);
    Bf.tables = sc->d_tables;
    Bf.film = film;
    Bf.tallies = tallies ? reinterpret_cast<unsigned long long*>(tallies) : nullptr;
    Bf.counter = sc->d_counter;
    Bf.rec = rec;
    HIP_TRY(launch_zero_u64(sc->d_counter, 1, s), "zero path counter");
    hipEvent_t* ev = nullptr;
    if ((rc = timing_slot(sc, &ev)) != FPT_OK) return rc;
    if (ev) HIP_TRY(hipEventRecord(ev[0], s), "hipEventRecord");
    HIP_TRY(launch_camera(P, Bf, records, grid, block, s), "camera launch");
    if (ev) HIP_TRY(hipEventRecord(ev[1], s), "hipEventRecord");
    if (ev) HIP_TRY(hipEventRecord(ev[2], s), "hipEventRecord");
    return FPT_OK;
}

}  // extern "C"

namespace {

int32_t batch_create(const fpt_scene_desc* descs, const fpt_run* runs, int32_t n, const fpt_tune* tune,
                     fpt_batch** out);

}  // namespace

extern "C" {

int32_t fpt_batch_create(const fpt_scene_desc* descs, const fpt_run* runs, int32_t n,
                         const fpt_tune* tune, fpt_batch** out) {
    if (!descs || !runs || !out) return set_err(FPT_E_INVALID, "NULL argument");
    *out = nullptr;
    if (n < 1 || n > (1 << 20)) return set_err(FPT_E_RANGE, "instance count %d", n);
    alloc_fault_arm(true);
    int32_t rc;
    try {
        rc = batch_create(descs, runs, n, tune, out);
    } catch (const std::bad_alloc&) {
        rc = set_err(FPT_E_NOMEM, "host allocation");
    }
    alloc_fault_arm(false);
    return rc;
}

}  // extern "C"

namespace {

// fpt_batch_create after its argument checks; `bt` is freed on every failure
// path, a host allocation failure thrown by the setup included.
int32_t batch_setup(fpt_batch* bt, const fpt_scene_desc* descs, const fpt_run* runs, int32_t n,
                    const fpt_tune* tune, fpt_batch** out) {
    std::memset(&bt->tune, 0, sizeof bt->tune);
    if (tune) bt->tune = *tune;
    bt->n = n;
    int32_t rc = FPT_OK;
    std::vector<KParams> params((size_t)n);
    std::vector<uint32_t> tables, toff((size_t)n);
    std::vector<float> wscale((size_t)n);
    std::vector<double> cost((size_t)n);
    int max_tw = 0;
    for (int i = 0; i < n && rc == FPT_OK; ++i) {
        const fpt_scene_desc& d = descs[i];
        if ((rc = validate(&d)) != FPT_OK) break;
        if (d.geometry != FPT_GEOM_SLAB && d.geometry != FPT_GEOM_SPHERE) {
            rc = set_err(FPT_E_UNSUPPORTED, "instance %d: batched instances are slabs or spheres", i);
            break;
        }
        if (d.sensor != FPT_SENSOR_ESCAPE) {
            rc = set_err(FPT_E_UNSUPPORTED, "instance %d: batched instances use the escape sensor", i);
            break;
        }
        if (i > 0 && d.n_bins != descs[0].n_bins) {
            rc = set_err(FPT_E_INVALID, "instance %d: all instances need the same n_bins", i);
            break;
        }
        uint32_t B;
        if ((rc = check_run(nullptr, &runs[i], &B)) != FPT_OK) break;
        if (B != 1) { rc = set_err(FPT_E_UNSUPPORTED, "batched runs have no parity batches"); break; }
        if (runs[i].path_count > 0xFFFFFFFFull) { rc = set_err(FPT_E_RANGE, "path_count"); break; }
        fpt_scene tmp;
        tmp.desc = d;
        tmp.tune = bt->tune;
        if ((rc = build_tables(&tmp)) != FPT_OK) break;
        fill_run(&tmp, &runs[i], 1, &params[i]);
        params[i].hist_words = 4 * d.n_bins;
        toff[i] = (uint32_t)tables.size();
        tables.insert(tables.end(), tmp.image.begin(), tmp.image.end());
        while (tables.size() % 4) tables.push_back(0u);
        max_tw = std::max(max_tw, params[i].off_kap);  // forward only: no d sigma_a rows
        wscale[i] = params[i].wscale;
        // expected work: paths x (1 + scattering optical size), for longest-first ordering
        const fpt_medium& md = d.media[d.body_medium];
        const double size = d.geometry == FPT_GEOM_SLAB ? d.slab_z1 - d.slab_z0 : 2.0 * d.body_radius;
        cost[i] = (double)runs[i].path_count * (1.0 + md.sigma_s_mm * size);
        bt->total_paths += runs[i].path_count;
    }
    if (rc != FPT_OK) {
        delete bt;
        return rc;
    }
    bt->N = descs[0].n_bins;
    bt->hist_words = 4 * bt->N;
    bt->params = params;
    bt->cost = cost;
    bt->path_counts.resize((size_t)n);
    for (int i = 0; i < n; ++i) bt->path_counts[i] = (uint32_t)runs[i].path_count;
    bt->wscale = wscale;
    bt->max_table_words = max_tw;
    hipError_t e = hipGetDevice(&bt->device);
    if (e == hipSuccess) e = hipDeviceGetAttribute(&bt->n_cu, hipDeviceAttributeMultiprocessorCount, bt->device);
    if (e == hipSuccess) e = dev_malloc((void**)&bt->d_params, sizeof(KParams) * n);
    if (e == hipSuccess) e = dev_malloc((void**)&bt->d_tables, std::max<size_t>(4, tables.size() * 4));
    if (e == hipSuccess) e = dev_malloc((void**)&bt->d_toff, 4 * (size_t)n);
    if (e == hipSuccess) e = dev_malloc((void**)&bt->d_wscale, 4 * (size_t)n);
    if (e == hipSuccess) e = dev_malloc((void**)&bt->d_counts, 4 * (size_t)n * bt->hist_words);
    if (e == hipSuccess) e = dev_malloc((void**)&bt->d_counter, 64);
    if (e == hipSuccess) e = hipMemcpy(bt->d_params, params.data(), sizeof(KParams) * n, hipMemcpyHostToDevice);
    if (e == hipSuccess) e = hipMemcpy(bt->d_tables, tables.data(), tables.size() * 4, hipMemcpyHostToDevice);
    if (e == hipSuccess) e = hipMemcpy(bt->d_toff, toff.data(), 4 * (size_t)n, hipMemcpyHostToDevice);
    if (e == hipSuccess) e = hipMemcpy(bt->d_wscale, wscale.data(), 4 * (size_t)n, hipMemcpyHostToDevice);
    if (e == hipSuccess) e = hipStreamCreateWithFlags(&bt->cap_stream, hipStreamNonBlocking);
    if (e != hipSuccess) {
        fpt_batch_destroy(bt);
        return hip_err(e, "batch setup");
    }
    if ((rc = batch_build_items(bt)) != FPT_OK) {
        fpt_batch_destroy(bt);
        return rc;
    }
    *out = bt;
    return FPT_OK;
}

int32_t batch_create(const fpt_scene_desc* descs, const fpt_run* runs, int32_t n, const fpt_tune* tune,
                     fpt_batch** out) {
    fpt_batch* bt = new_object<fpt_batch>();
    if (!bt) return set_err(FPT_E_NOMEM, "host allocation");
    try {
        return batch_setup(bt, descs, runs, n, tune, out);  // frees bt on its failure paths
    } catch (...) {
        fpt_batch_destroy(bt);
        throw;
    }
}

}  // namespace

extern "C" {

int32_t fpt_batch_render(fpt_batch* bt, float* films, uint64_t* tallies, void* stream) {
    if (!bt || !films) return set_err(FPT_E_INVALID, "NULL argument");
    hipStream_t s = (hipStream_t)stream;
    if (!bt->exec || bt->g_films != films || bt->g_tallies != tallies) {
        if (bt->exec) (void)hipGraphExecDestroy(bt->exec);
        if (bt->graph) (void)hipGraphDestroy(bt->graph);
        bt->exec = nullptr;
        bt->graph = nullptr;
        KBatch K = bt->kbatch;
        K.tallies = reinterpret_cast<unsigned long long*>(tallies);
        const size_t nc = (size_t)bt->n * bt->hist_words;
        HIP_TRY(hipStreamBeginCapture(bt->cap_stream, hipStreamCaptureModeThreadLocal), "begin capture");
        hipError_t e = launch_zero_u32(bt->d_counts, nc, bt->cap_stream);
        if (e == hipSuccess) e = launch_zero_u64(bt->d_counter, 1, bt->cap_stream);
        if (e == hipSuccess) e = launch_batch(K, bt->grid, bt->block, bt->cap_stream);
        if (e == hipSuccess) e = launch_finalize_batch(bt->d_counts, films, bt->d_wscale, bt->hist_words, nc, bt->cap_stream);
        hipGraph_t g = nullptr;
        hipError_t e2 = hipStreamEndCapture(bt->cap_stream, &g);
        if (e != hipSuccess) {
            if (g) (void)hipGraphDestroy(g);
            return hip_err(e, "batch capture");
        }
        if (e2 != hipSuccess) return hip_err(e2, "end capture");
        bt->graph = g;
        HIP_TRY(hipGraphInstantiate(&bt->exec, bt->graph, nullptr, nullptr, 0), "graph instantiate");
        bt->g_films = films;
        bt->g_tallies = tallies;
    }
    HIP_TRY(hipGraphLaunch(bt->exec, s), "graph launch");
    return FPT_OK;
}

void fpt_batch_destroy(fpt_batch* bt) {
    if (!bt) return;
    if (bt->exec) (void)hipGraphExecDestroy(bt->exec);
    if (bt->graph) (void)hipGraphDestroy(bt->graph);
    if (bt->cap_stream) (void)hipStreamDestroy(bt->cap_stream);
    if (bt->d_params) (void)hipFree(bt->d_params);
    if (bt->d_tables) (void)hipFree(bt->d_tables);
    if (bt->d_toff) (void)hipFree(bt->d_toff);
    if (bt->d_wscale) (void)hipFree(bt->d_wscale);
    if (bt->d_counts) (void)hipFree(bt->d_counts);
    if (bt->d_counter) (void)hipFree(bt->d_counter);
    if (bt->d_items) (void)hipFree(bt->d_items);
    delete bt;
}

}  // extern "C"

namespace {

// Launch-shape cache: a JSON object mapping "<workload>@<device>" to an object
// of the fpt_tune fields and "ms" (numbers).  Only this shape is read; fields
// other than those are ignored.
struct CachedTune {
    fpt_tune t;
    double ms;
};

void skip_ws(const char*& p) {
    while (*p == ' ' || *p == '\n' || *p == '\r' || *p == '\t') ++p;
}

bool parse_string(const char*& p, std::string* out) {
    skip_ws(p);
    if (*p != '"') return false;
    ++p;
    out->clear();
    while (*p && *p != '"') {
        if (*p == '\\') return false;  // keys of this cache never need escapes
        out->push_back(*p++);
    }
    if (*p != '"') return false;
    ++p;
    return true;
}

bool expect(const char*& p, char c) {
    skip_ws(p);
    if (*p != c) return false;
    ++p;
    return true;
}

bool parse_cache(const std::string& text, std::map<std::string, CachedTune>* out) {
    const char* p = text.c_str();
    skip_ws(p);
    if (!*p) return true;  // an empty file is an empty cache
    if (!expect(p, '{')) return false;
    skip_ws(p);
    if (*p == '}') return true;
    for (;;) {
        std::string key, field;
        if (!parse_string(p, &key) || !expect(p, ':') || !expect(p, '{')) return false;
        CachedTune ct;
        std::memset(&ct.t, 0, sizeof ct.t);
        ct.ms = 0.0;
        skip_ws(p);
        if (*p != '}') {
            for (;;) {
                if (!parse_string(p, &field) || !expect(p, ':')) return false;
                skip_ws(p);
                char* end = nullptr;
                const double v = std::strtod(p, &end);
                if (end == p) return false;
                p = end;
                if (field == "ms") ct.ms = v;
                else if (field == "block_threads") ct.t.block_threads = (int32_t)v;
                else if (field == "blocks_per_cu") ct.t.blocks_per_cu = (int32_t)v;
                else if (field == "refill_lanes") ct.t.refill_lanes = (int32_t)v;
                else if (field == "chunk_paths") ct.t.chunk_paths = (int32_t)v;
                else if (field == "block_min_vertices") ct.t.block_min_vertices = (int32_t)v;
                else if (field == "block_segments") ct.t.block_segments = (int32_t)v;
                else if (field == "wide_rounds") ct.t.wide_rounds = (int32_t)v;
                skip_ws(p);
                if (*p == ',') { ++p; continue; }
                if (*p == '}') break;
                return false;
            }
        }
        ++p;  // '}'
        (*out)[key] = ct;
        skip_ws(p);
        if (*p == ',') { ++p; continue; }
        if (*p == '}') return true;
        return false;
    }
}

int32_t read_cache(const char* path, std::map<std::string, CachedTune>* cache) {
    FILE* f = std::fopen(path, "rb");
    if (!f) return FPT_OK;  // no cache yet
    std::string text;
    char buf[4096];
    size_t n;
    while ((n = std::fread(buf, 1, sizeof buf, f)) > 0) text.append(buf, n);
    std::fclose(f);
    if (!parse_cache(text, cache)) return set_err(FPT_E_INVALID, "malformed tune cache %s", path);
    return FPT_OK;
}

// Rewrites the cache (keys and fields sorted), through a temporary file.
int32_t write_cache(const char* path, const std::map<std::string, CachedTune>& cache) {
    const std::string tmp = std::string(path) + ".tmp";
    FILE* f = std::fopen(tmp.c_str(), "wb");
    if (!f) return set_err(FPT_E_INVALID, "cannot write tune cache %s", tmp.c_str());
    std::fputs("{", f);
    bool first = true;
    for (const auto& kv : cache) {
        const fpt_tune& t = kv.second.t;
        std::fprintf(f,
                     "%s\n \"%s\": {\n  \"block_min_vertices\": %d,\n  \"block_segments\": %d,\n"
                     "  \"block_threads\": %d,\n  \"blocks_per_cu\": %d,\n  \"chunk_paths\": %d,\n"
                     "  \"ms\": %.9g,\n  \"refill_lanes\": %d,\n  \"wide_rounds\": %d\n }",
                     first ? "" : ",", kv.first.c_str(), t.block_min_vertices, t.block_segments,
                     t.block_threads, t.blocks_per_cu, t.chunk_paths, kv.second.ms, t.refill_lanes,
                     t.wide_rounds);
        first = false;
    }
    std::fputs("\n}", f);
    const bool ok = std::fclose(f) == 0;
    if (!ok || std::rename(tmp.c_str(), path) != 0)
        return set_err(FPT_E_INVALID, "cannot write tune cache %s", path);
    return FPT_OK;
}

// Cache key suffix of the current device: its architecture and CU count.
int32_t device_tag(std::string* tag) {
    int dev = 0;
    hipDeviceProp_t prop;
    HIP_TRY(hipGetDevice(&dev), "hipGetDevice");
    HIP_TRY(hipGetDeviceProperties(&prop, dev), "hipGetDeviceProperties");
    std::string arch = prop.gcnArchName;
    const size_t colon = arch.find(':');
    if (colon != std::string::npos) arch.resize(colon);
    *tag = arch + "x" + std::to_string(prop.multiProcessorCount) + "cu";
    return FPT_OK;
}

int32_t measure_tune(fpt_scene* sc, const fpt_run* run, fpt_batch* bt, fpt_tune* out, float* best_ms);

}  // namespace

extern "C" {

int32_t fpt_autotune(fpt_scene* sc, const fpt_run* run, fpt_batch* bt, const char* cache_path,
                     const char* workload, uint32_t flags, fpt_tune* out, float* best_ms) {
    // without a scene or batch only a cache lookup is possible
    const bool lookup = (flags & FPT_TUNE_CACHED_ONLY) && cache_path;
    if (!out || (!sc && !bt && !lookup) || (sc && !run)) return set_err(FPT_E_INVALID, "NULL argument");
    if (cache_path && !workload) return set_err(FPT_E_INVALID, "a cache needs a workload name");
    if (flags & ~(FPT_TUNE_FORCE | FPT_TUNE_CACHED_ONLY)) return set_err(FPT_E_INVALID, "unknown tune flags");
    std::map<std::string, CachedTune> cache;
    std::string key;
    if (cache_path) {
        int32_t rc = read_cache(cache_path, &cache);
        if (rc != FPT_OK) return rc;
        std::string tag;
        if ((rc = device_tag(&tag)) != FPT_OK) return rc;
        key = std::string(workload) + "@" + tag;
        auto it = cache.find(key);
        if (it != cache.end() && !(flags & FPT_TUNE_FORCE)) {
            *out = it->second.t;
            if (best_ms) *best_ms = (float)it->second.ms;
            return FPT_OK;
        }
    }
    if (flags & FPT_TUNE_CACHED_ONLY) {
        std::memset(out, 0, sizeof *out);  // the library defaults
        if (best_ms) *best_ms = 0.f;
        return FPT_OK;
    }
    float ms = 0.f;
    int32_t rc = measure_tune(sc, run, bt, out, &ms);
    if (rc != FPT_OK) return rc;
    if (best_ms) *best_ms = ms;
    if (!cache_path) return FPT_OK;
    cache[key] = CachedTune{*out, (double)ms};
    return write_cache(cache_path, cache);
}

}  // extern "C"

namespace {

int32_t measure_tune(fpt_scene* sc, const fpt_run* run, fpt_batch* bt, fpt_tune* out, float* best_ms) {
    hipEvent_t e0, e1;
    HIP_TRY(hipEventCreate(&e0), "event");
    HIP_TRY(hipEventCreate(&e1), "event");
    float* film = nullptr;
    size_t film_n = 0;
    if (sc) {
        uint32_t B;
        int32_t rc = check_run(sc, run, &B);
        if (rc != FPT_OK) return rc;
        film_n = (size_t)film_elems(sc->desc, B);
    } else {
        film_n = (size_t)bt->n * bt->hist_words;
    }
    HIP_TRY(hipMalloc(&film, film_n * 4), "hipMalloc(tune film)");
    const fpt_tune saved = sc ? sc->tune : bt->tune;
    std::vector<fpt_tune> cand;
    const int blocks[2] = {128, 256};
    if (sc) {
        for (int b : blocks)
            for (int r : {16, 32, 40, 48, 60})
                for (int m : {1, 2, 8})
                    for (int g : {2, 4})
                        for (int wr : {1, 2}) cand.push_back(fpt_tune{b, 0, r, 0, m, g, wr});
    } else {
        for (int b : blocks)
            for (int r : {8, 32})
                for (int m : {16, 64})
                    for (int g : {1, 2})
                        for (int c : {512, 1024, 4096}) cand.push_back(fpt_tune{b, 0, r, c, m, g, 0});
    }
    float best = 1e30f;
    fpt_tune best_t = saved;
    int32_t rc = FPT_OK;
    // one candidate: `reps` renders back to back after one untimed render, mean ms
    auto time_cand = [&](const fpt_tune& t, int reps, float* ms_out) -> int32_t {
        int32_t r = FPT_OK;
        if (sc) {
            sc->tune = t;
        } else {
            bt->tune = t;
            if ((r = batch_build_items(bt)) != FPT_OK) return r;
        }
        r = sc ? fpt_render(sc, run, film, nullptr, nullptr) : fpt_batch_render(bt, film, nullptr, nullptr);
        if (r != FPT_OK) return r;
        if (hipEventRecord(e0, nullptr) != hipSuccess) return set_err(FPT_E_DEVICE, "event record");
        for (int rep = 0; rep < reps && r == FPT_OK; ++rep)
            r = sc ? fpt_render(sc, run, film, nullptr, nullptr) : fpt_batch_render(bt, film, nullptr, nullptr);
        if (r != FPT_OK) return r;
        (void)hipEventRecord(e1, nullptr);
        (void)hipEventSynchronize(e1);
        float ms = 0.f;
        (void)hipEventElapsedTime(&ms, e0, e1);
        *ms_out = ms / reps;
        return FPT_OK;
    };
    // a short screen of every candidate, then the best few again with more
    // renders, so the choice is not decided by one lucky measurement; short
    // jobs get more renders per candidate (at least ~5 ms screened and ~50 ms
    // re-timed, in three interleaved passes over the finalists)
    float probe = 0.f;
    rc = time_cand(saved, 1, &probe);
    const int screen_reps = rc == FPT_OK ? std::max(3, std::min(200, (int)std::ceil(5.f / std::max(probe, 1e-3f)))) : 3;
    const int final_reps = rc == FPT_OK ? std::max(4, std::min(600, (int)std::ceil(17.f / std::max(probe, 1e-3f)))) : 4;
    std::vector<std::pair<float, size_t>> screen;
    for (size_t i = 0; i < cand.size() && rc == FPT_OK; ++i) {
        float ms = 0.f;
        rc = time_cand(cand[i], screen_reps, &ms);
        screen.push_back({ms, i});
    }
    if (rc == FPT_OK) {
        std::sort(screen.begin(), screen.end());
        const size_t keep = std::min<size_t>(screen.size(), 6);
        std::vector<float> total(keep, 0.f);
        for (int pass = 0; pass < 3 && rc == FPT_OK; ++pass)
            for (size_t k = 0; k < keep && rc == FPT_OK; ++k) {
                float ms = 0.f;
                rc = time_cand(cand[screen[k].second], final_reps, &ms);
                total[k] += ms / 3.f;
            }
        for (size_t k = 0; k < keep && rc == FPT_OK; ++k)
            if (total[k] < best) {
                best = total[k];
                best_t = cand[screen[k].second];
            }
    }
    if (sc) sc->tune = saved;
    else {
        bt->tune = saved;
        (void)batch_build_items(bt);
    }
    (void)hipFree(film);
    (void)hipEventDestroy(e0);
    (void)hipEventDestroy(e1);
    if (rc != FPT_OK) return rc;
    *out = best_t;
    *best_ms = best;
    return FPT_OK;
}

}  // namespace
