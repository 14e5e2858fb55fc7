// HIP kernels of the fluorescent spectral path tracer (gfx950, wave64).
//
// One persistent kernel per geometry class runs the whole per-vertex loop of
// the forward analog walk (sec. 4.1-4.3 of the paper): free flight from
// sigma_t(lambda) (eq. 6), the scatter / absorber choice, the quantum-yield
// test and re-emission from the emission CDF (eq. 10), interface and wall
// handling, and the film splat (eqs. 3-6).  Path state lives in registers;
// each wave keeps 64 paths in flight and, whenever enough of its lanes have
// finished, claims new path ids for them with one atomic on a device queue
// head (ballot + popcount + mbcnt prefix), so lanes stay busy without any
// state round trip through HBM.  Spectral tables live in LDS.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <mutex>

#include "fpt_internal.h"

namespace fpt {

#define DEV __device__ __forceinline__

constexpr float kInf = __builtin_inff();
constexpr uint32_t kMaxPathVertices = 1u << 28;
constexpr int kBlockPasses = 4;   // block passes per iteration for paths that never stop (see advance)
constexpr int kLdsSpheres = 32;
constexpr int kQueueShards = 64;   // path-queue heads (see k_transport)
constexpr int kShardStride = 16;   // u64 words between heads: separate 128-byte lines                                // word offset of the sphere table
constexpr int kLdsTable = kLdsSpheres + 8 * FPT_MAX_SPHERES;   // word offset of the table image
constexpr float kInv4Pi = 0.0795774715459476679f;
constexpr float kInvPi = 0.318309886183790672f;

enum { MODE_FWD = 0, MODE_ADJ = 1, MODE_REC = 2, MODE_REC_ADJ = 3 };
enum { EV_NONE = 0, EV_SCATTER, EV_BG, EV_DYE, EV_ESC, EV_WALL, EV_LIGHT, EV_ENTER, EV_EXIT,
       EV_INF };
enum { PEND_NONE = 0, PEND_MEDIUM = 1, PEND_SURFACE = 2, PEND_SOURCE = 3 };

// -------------------------------------------------------------------------
// Philox4x32-10 (Salmon et al., SC'11): ten rounds of two 32x32->64 products;
// the high halves are xor-ed with the other counter words and the round key,
// which advances by the two Weyl increments.  The key is uniform per launch
// (kept in scalar registers); the products map to v_mad_u64_u32.  The empty
// asm makes the key opaque at every call, so the ten round keys are formed
// by scalar adds where they are used: hoisted out of the persistent loop
// they occupied 20 scalar registers, which spilled to VGPR lanes and came
// back through one v_readlane (a vector instruction) per round.
DEV uint4 philox(uint32_t c0, uint32_t c1, uint32_t c2, uint32_t c3, uint32_t k0, uint32_t k1) {
    asm volatile("" : "+s"(k0), "+s"(k1));
#pragma unroll
    for (int i = 0; i < 10; ++i) {
        const uint64_t p0 = (uint64_t)0xD2511F53u * c0;
        const uint64_t p1 = (uint64_t)0xCD9E8D57u * c2;
        // three-input xor in one v_bitop3_b32 (truth table 0x96: odd parity)
        const uint32_t n0 = __builtin_amdgcn_bitop3_b32((uint32_t)(p1 >> 32), c1, k0, 0x96);
        const uint32_t n2 = __builtin_amdgcn_bitop3_b32((uint32_t)(p0 >> 32), c3, k1, 0x96);
        c1 = (uint32_t)p1;
        c3 = (uint32_t)p0;
        c0 = n0;
        c2 = n2;
        k0 += 0x9E3779B9u;
        k1 += 0xBB67AE85u;
    }
    return make_uint4(c0, c1, c2, c3);
}

// 24 high bits -> [0,1), exact in fp32.
DEV float u24(uint32_t x) { return (float)(x >> 8) * 5.9604644775390625e-08f; }
// -ln(1 - u) for u = u24(.) in [0, 1): the hardware base-2 logarithm times
// ln 2.  1 - u >= 2^-24 is a normal number, so the range reduction and the
// compensated ln 2 product of the library logarithm (about ten more
// instructions, under 1 ulp of difference) are not needed.
DEV float neg_log1m(float u) { return -0.693147182f * __builtin_amdgcn_logf(1.f - u); }
DEV uint32_t rr_bits(const uint4 r) {
    return ((r.x & 0xFFu) << 16) | ((r.y & 0xFFu) << 8) | (r.z & 0xFFu);
}

// Hardware square root (about 1 ulp) and sin/cos of 2 pi u: v_sin_f32 and
// v_cos_f32 take their argument in revolutions.
DEV float fsqrt(float x) { return __builtin_amdgcn_sqrtf(x); }
DEV void sincos_rev(float u, float* s, float* c) {
    *s = __builtin_amdgcn_sinf(u);
    *c = __builtin_amdgcn_cosf(u);
}

// a / b through the hardware reciprocal (about 1 ulp); b != 0 at every call site.
DEV float fdiv(float a, float b) { return a * __builtin_amdgcn_rcpf(b); }

DEV float wf(const uint32_t* S, int i) { return __uint_as_float(S[i]); }
DEV int wi(const uint32_t* S, int i) { return (int)S[i]; }
DEV float dot3(const float* a, const float* b) { return a[0] * b[0] + a[1] * b[1] + a[2] * b[2]; }

DEV uint32_t lane_id() { return __lane_id(); }
DEV uint32_t mbcnt(uint64_t m) {
    return __builtin_amdgcn_mbcnt_hi((uint32_t)(m >> 32), __builtin_amdgcn_mbcnt_lo((uint32_t)m, 0u));
}

struct Lane {
    float x[3], w[3];
    float sc[3], sr2;  // the sphere the lane is inside (box scenes)
    float st, inv;     // sigma_t and 1/sigma_t at (medium, lambda); inv = inf in vacuum
    float ss, thr_bg;  // scatter / background thresholds of the medium
    int ndy;           // dye slots of the medium
    int lam, region, medium, comp;
    uint32_t pid, v, nsc, nem, batch;
    float splat_sum;
    float wgt;  // throughput weight (glossy walls; 1 otherwise)
};

DEV void load_sigma(const KParams& P, const uint32_t* S, Lane& L) {
    if (L.medium < 0) {
        L.st = 0.f;
        L.inv = kInf;
        return;
    }
    const float2 v = *reinterpret_cast<const float2*>(S + P.off_st + 2 * (L.medium * P.N + L.lam));
    L.st = v.x;
    L.inv = v.y;
}

DEV void load_medium(const KParams& P, const uint32_t* S, Lane& L) {
    if (L.medium < 0) {
        L.ss = 0.f;
        L.thr_bg = 0.f;
        L.ndy = 0;
    } else {
        const int b = P.off_med + L.medium * kMedWords;
        L.ss = wf(S, b + MW_SS);
        L.thr_bg = wf(S, b + MW_THR_BG);
        L.ndy = wi(S, b + MW_NDYES);
    }
    load_sigma(P, S, L);
}

// -------------------------------------------------------------------------
// Geometry: distance to the next surface along the lane's ray.
struct Hit {
    float d;
    int ev;   // EV_ESC, EV_WALL, EV_LIGHT, EV_ENTER, EV_EXIT, EV_INF
    int idx;  // wall face or sphere
};

// Exit distance of the ray x + t w from the sphere (c, r2) holding x.  Every
// rounding is written out (explicit fma, contraction off): the copies of this
// code inlined into the different walk loops then give the same bits, so the
// loops take the same stop decisions (with contraction left to the compiler
// two copies fused differently, and a path near a tie walked differently
// depending on which loop served it).
DEV float sphere_exit(const float* x, const float* w, const float* c, float r2) {
#pragma clang fp contract(off)
    const float o0 = x[0] - c[0], o1 = x[1] - c[1], o2 = x[2] - c[2];
    const float b = __builtin_fmaf(o2, w[2], __builtin_fmaf(o1, w[1], o0 * w[0]));
    const float cc = __builtin_fmaf(o2, o2, __builtin_fmaf(o1, o1, o0 * o0)) - r2;
    const float disc = __builtin_fmaf(b, b, -cc);
    return fmaxf(0.f, fsqrt(fmaxf(disc, 0.f)) - b);
}

template <int GEOM>
DEV Hit next_surface(const KParams& P, const KSphere* SP, const Lane& L, bool skip_light) {
    Hit h;
    h.d = kInf;
    h.ev = EV_ESC;
    h.idx = -1;
    if constexpr (GEOM == FPT_GEOM_SLAB) {
        if (L.w[2] != 0.f) h.d = fdiv((L.w[2] > 0.f ? P.z1 : P.z0) - L.x[2], L.w[2]);
        h.d = fmaxf(h.d, 0.f);
    } else if constexpr (GEOM == FPT_GEOM_HALFSPACE) {
        if (L.w[2] < 0.f) h.d = fmaxf(fdiv(P.z0 - L.x[2], L.w[2]), 0.f);
    } else if constexpr (GEOM == FPT_GEOM_SPHERE) {
        h.d = sphere_exit(L.x, L.w, P.bc, P.br2);
    } else if constexpr (GEOM == FPT_GEOM_INFINITE) {
        h.ev = EV_ESC;
    } else {
        if (L.region >= 0) {
            h.d = sphere_exit(L.x, L.w, L.sc, L.sr2);
            h.ev = EV_EXIT;
            h.idx = L.region;
            return h;
        }
        // vacuum: box walls
#pragma unroll
        for (int a = 0; a < 3; ++a) {
            float t = kInf;
            int f = -1;
            if (L.w[a] != 0.f) {
                const bool up = L.w[a] > 0.f;
                t = fdiv((up ? P.hi[a] : P.lo[a]) - L.x[a], L.w[a]);
                f = 2 * a + (up ? 1 : 0);
            }
            t = fmaxf(t, 0.f);
            if (t < h.d) { h.d = t; h.idx = f; }
        }
        h.ev = (h.idx == P.open_face) ? EV_ESC : EV_WALL;
        // light quad (opaque, both sides)
        if (!skip_light) {
            const float dn = dot3(P.ln, L.w);
            if (dn != 0.f) {
                const float pc0 = P.lpos[0] - L.x[0], pc1 = P.lpos[1] - L.x[1], pc2 = P.lpos[2] - L.x[2];
                const float t = fdiv(P.ln[0] * pc0 + P.ln[1] * pc1 + P.ln[2] * pc2, dn);
                if (t > 0.f && t < h.d) {
                    const float q0 = L.x[0] + t * L.w[0] - P.lpos[0];
                    const float q1 = L.x[1] + t * L.w[1] - P.lpos[1];
                    const float q2 = L.x[2] + t * L.w[2] - P.lpos[2];
                    const float a = (q0 * P.lu[0] + q1 * P.lu[1] + q2 * P.lu[2]) * P.lu_inv2;
                    const float b = (q0 * P.lv[0] + q1 * P.lv[1] + q2 * P.lv[2]) * P.lv_inv2;
                    if (a >= 0.f && a <= 1.f && b >= 0.f && b <= 1.f) {
                        h.d = t;
                        h.ev = EV_LIGHT;
                        h.idx = -1;
                    }
                }
            }
        }
        // sphere entries
        for (int s = 0; s < P.n_spheres; ++s) {
            const KSphere& sp = SP[s];
            const float o0 = L.x[0] - sp.c[0], o1 = L.x[1] - sp.c[1], o2 = L.x[2] - sp.c[2];
            const float b = o0 * L.w[0] + o1 * L.w[1] + o2 * L.w[2];
            if (!(b < 0.f)) continue;
            const float cc = o0 * o0 + o1 * o1 + o2 * o2 - sp.r2;
            const float disc = b * b - cc;
            if (!(disc > 0.f)) continue;
            const float t = fmaxf(-b - fsqrt(disc), 0.f);
            if (t < h.d) { h.d = t; h.ev = EV_ENTER; h.idx = s; }
        }
    }
    return h;
}

// A point that reached a planar boundary lies on it: set that coordinate exactly.
template <int GEOM>
DEV void snap_to_plane(const KParams& P, Lane& L, const Hit& h) {
    if constexpr (GEOM == FPT_GEOM_SLAB) {
        if (h.d < kInf) L.x[2] = L.w[2] < 0.f ? P.z0 : P.z1;
    } else if constexpr (GEOM == FPT_GEOM_HALFSPACE) {
        if (h.d < kInf) L.x[2] = P.z0;
    } else if constexpr (GEOM == FPT_GEOM_BOX) {
        if ((h.ev == EV_WALL || h.ev == EV_ESC) && h.idx >= 0) {
            const int ax = h.idx >> 1;
            const float v = (h.idx & 1) ? P.hi[ax] : P.lo[ax];
            if (ax == 0) L.x[0] = v;
            else if (ax == 1) L.x[1] = v;
            else L.x[2] = v;
        }
    }
}

// Smooth dielectric boundary of a body medium (index n, vacuum outside).
// Unpolarised reflectance (mean of the s and p Fresnel intensities) from index
// n1 into n2 at incidence cosine ci >= 0; 1 beyond the critical angle; ct gets
// the transmitted cosine.
DEV float fresnel(float ci, float n1, float n2, float& ct) {
    const float eta = fdiv(n1, n2);
    const float st2 = eta * eta * (1.f - ci * ci);
    if (st2 >= 1.f) {
        ct = 0.f;
        return 1.f;
    }
    const float c2 = fsqrt(1.f - st2);
    const float rs = fdiv(n1 * ci - n2 * c2, n1 * ci + n2 * c2);
    const float rp = fdiv(n1 * c2 - n2 * ci, n1 * c2 + n2 * ci);
    ct = c2;
    return 0.5f * (rs * rs + rp * rp);
}

// Outward normal of the body's boundary at x for a path moving along w (the
// slab face it is heading for).
template <int GEOM>
DEV void body_normal(const KParams& P, const float* x, const float* w, float* nb) {
    nb[0] = nb[1] = 0.f;
    if constexpr (GEOM == FPT_GEOM_SLAB) {
        nb[2] = w[2] > 0.f ? 1.f : -1.f;
    } else if constexpr (GEOM == FPT_GEOM_HALFSPACE) {
        nb[2] = -1.f;
    } else {
        const float d0 = x[0] - P.bc[0], d1 = x[1] - P.bc[1], d2 = x[2] - P.bc[2];
        const float s = __builtin_amdgcn_rsqf(d0 * d0 + d1 * d1 + d2 * d2);
        nb[0] = d0 * s;
        nb[1] = d1 * s;
        nb[2] = d2 * s;
    }
}

DEV void mirror(float* w, const float* nb) {
    const float d = 2.f * dot3(w, nb);
    w[0] -= d * nb[0];
    w[1] -= d * nb[1];
    w[2] -= d * nb[2];
}

// Length of the segment x + t wc, t in [0, dist], inside a sphere.  The
// half-chord squared is r^2 minus the squared distance of the line from the
// centre, taken from the perpendicular offset o - b wc: the textbook b^2 - |o|^2
// + r^2 cancels to fp32 noise when the line passes a distant sphere nearly
// tangentially, where the chord, going as its square root, is most sensitive.
DEV float chord_len(const KSphere& sp, const float* x, const float* wc, float dist) {
    const float o0 = x[0] - sp.c[0], o1 = x[1] - sp.c[1], o2 = x[2] - sp.c[2];
    const float b = o0 * wc[0] + o1 * wc[1] + o2 * wc[2];
    const float p0 = o0 - b * wc[0], p1 = o1 - b * wc[1], p2 = o2 - b * wc[2];
    const float disc = sp.r2 - (p0 * p0 + p1 * p1 + p2 * p2);
    const float sq = fsqrt(fmaxf(disc, 0.f));
    const float lo = fmaxf(-b - sq, 0.f), hi = fminf(-b + sq, dist);
    return disc > 0.f ? fmaxf(hi - lo, 0.f) : 0.f;
}


// -------------------------------------------------------------------------
// Launch parameters read from the running kernel's first argument in the
// kernarg segment.  The empty asm hides the address from the optimiser, so
// loads through it stay at each use: code that runs once per connection (the
// pinhole projection, visibility and light tests; the camera-side eye ray and
// light connection) then costs a few scalar loads, instead of its ~40 fields
// being loaded at kernel entry and held across the persistent loop, where the
// scalar registers run out and the spills come back through v_readlane.  That
// halved the box forward kernel's spills and took 10 % off the large scene.
// Valid only in kernels whose first parameter is `const KParams`: k_transport,
// k_splat_jobs, k_camera.
typedef const __attribute__((address_space(4))) KParams* KParamsArg;
DEV KParamsArg kernel_params() {
    KParamsArg p = (KParamsArg)__builtin_amdgcn_kernarg_segment_ptr();
    asm volatile("" : "+s"(p));
    return p;
}

// A medium vertex whose connection to the eye would cross an optical depth of
// at least P.tau_zero inside its own sphere alone deposits exactly 0 in fp32
// (at kTauZero its transmittance is 0; below that, at the run's path weight,
// the deposit's first product already rounds to 0), whatever the other
// spheres on the way add.  Where the host has shown that every point of that sphere passes the
// connection's geometric tests (P.sph_clear), its outcome is also known -- a
// hit of value 0, or a roulette kill when splat_rr > 0 -- so it is counted
// without being queued and evaluated (about a third of the large scene's
// connections, from deep inside its densest spheres).
// For x inside the (convex) sphere the exit distance along the eye direction
// w is at least L = P.tau_zero / sigma_t exactly when x + L w is inside too, so
// the test is one point-in-sphere check instead of a chord (no square root).
// inv_st = 1 / sigma_t of the vertex's medium and wavelength.
// Roundings written out, as in sphere_exit: every walk loop counts the same
// connections as opaque.
DEV bool opaque_to_eye(const float* x, int region, float inv_st, const float* sc, float sr2) {
#pragma clang fp contract(off)
    const auto& K = *kernel_params();
    if (region < 0 || !((K.sph_clear >> (uint32_t)region) & 1u)) return false;
    const float d0 = K.eye[0] - x[0], d1 = K.eye[1] - x[1], d2 = K.eye[2] - x[2];
    const float dd = __builtin_fmaf(d2, d2, __builtin_fmaf(d1, d1, d0 * d0));
    const float s = K.tau_zero * inv_st * __builtin_amdgcn_rsqf(dd);
    const float p0 = __builtin_fmaf(s, d0, x[0] - sc[0]), p1 = __builtin_fmaf(s, d1, x[1] - sc[1]),
                p2 = __builtin_fmaf(s, d2, x[2] - sc[2]);
    return __builtin_fmaf(p2, p2, __builtin_fmaf(p1, p1, p0 * p0)) <= sr2;
}

// The segment from a medium vertex x to the eye, shared by a deep round's
// opaque test and its in-place evaluation: d = eye - x, |d|^2 as the fma chain
// opaque_to_eye forms it, its reciprocal square root, and x minus the centre
// of the vertex's sphere.
struct EyeRay {
    float d[3], dist2, rdist, o[3];
};
DEV EyeRay eye_ray(const float* x, const float* sc) {
#pragma clang fp contract(off)
    const auto& K = *kernel_params();
    EyeRay r;
    r.d[0] = K.eye[0] - x[0];
    r.d[1] = K.eye[1] - x[1];
    r.d[2] = K.eye[2] - x[2];
    r.dist2 = __builtin_fmaf(r.d[2], r.d[2], __builtin_fmaf(r.d[1], r.d[1], r.d[0] * r.d[0]));
    r.rdist = __builtin_amdgcn_rsqf(r.dist2);
    r.o[0] = x[0] - sc[0];
    r.o[1] = x[1] - sc[1];
    r.o[2] = x[2] - sc[2];
    return r;
}
// opaque_to_eye from a precomputed ray (the same operations).
DEV bool opaque_to_eye(const EyeRay& r, int region, float inv_st, float sr2) {
#pragma clang fp contract(off)
    const auto& K = *kernel_params();
    if (region < 0 || !((K.sph_clear >> (uint32_t)region) & 1u)) return false;
    const float s = K.tau_zero * inv_st * r.rdist;
    const float p0 = __builtin_fmaf(s, r.d[0], r.o[0]), p1 = __builtin_fmaf(s, r.d[1], r.o[1]),
                p2 = __builtin_fmaf(s, r.d[2], r.o[2]);
    return __builtin_fmaf(p2, p2, __builtin_fmaf(p1, p1, p0 * p0)) <= sr2;
}

// -------------------------------------------------------------------------
// Pinhole splat at a realised vertex (eqs. 3-6).  Returns the deposited value
// (0 if rejected) and the film index.  f = 1/(4 pi) in a medium, cos/pi on a
// Lambertian surface.  CLEAR: a medium vertex inside a sphere of
// P.geo_clear, whose connection passes the geometric tests, which are then
// skipped, and whose transmittance is taken over the spheres of `smask`
// (P.sph_occl of its sphere) only: the others' chords are exactly 0, so the
// result is bit for bit the general one.
struct SplatOut {
    float v;
    long long idx;
    int status;  // 0 hit, 1 miss, 2 roulette kill
};

template <bool CLEAR = false>
DEV SplatOut splat_eval(const uint32_t* S, const KSphere* SP, const float* x, int lam, int comp,
                        uint32_t batch, int pend, const float* nrm, uint32_t rrb, float wgt = 1.f,
                        uint32_t smask = ~0u) {
    const auto& P = *kernel_params();
    // Every test is evaluated and folded into `ok`, so the lanes of a wave stay
    // together; a rejected connection deposits nothing.
    const float d[3] = {P.eye[0] - x[0], P.eye[1] - x[1], P.eye[2] - x[2]};
    const float dist2 = d[0] * d[0] + d[1] * d[1] + d[2] * d[2];
    const float rdist = __builtin_amdgcn_rsqf(dist2);
    const float dist = dist2 * rdist;
    const float wc[3] = {d[0] * rdist, d[1] * rdist, d[2] * rdist};
    const bool surf = pend != PEND_MEDIUM;
    const float cs = dot3(nrm, wc);
    const float f = surf ? cs * kInvPi : kInv4Pi;
    bool ok = !surf || cs > 0.f;
    // pinhole projection
    const float zc = -(d[0] * P.cf[0] + d[1] * P.cf[1] + d[2] * P.cf[2]);
    ok = ok && zc > 0.f;
    const float izc = __builtin_amdgcn_rcpf(zc);
    const float xi = -(d[0] * P.cr[0] + d[1] * P.cr[1] + d[2] * P.cr[2]) * izc * P.inv_tanx;
    const float yi = -(d[0] * P.cu[0] + d[1] * P.cu[1] + d[2] * P.cu[2]) * izc * P.inv_tany;
    const float fx = (xi + 1.f) * 0.5f * (float)P.W;
    const float fy = (1.f - yi) * 0.5f * (float)P.H;
    if (CLEAR) ok = true;
    ok = ok && (CLEAR || (fx >= 0.f && fx < (float)P.W && fy >= 0.f && fy < (float)P.H));
    // visibility: the segment from x (inside the box) to the eye (outside,
    // beyond the open face's plane) must cross that plane inside the face
    if constexpr (!CLEAR) {
        // one-hot axis vectors: the dot products pick coordinates exactly
        const auto& e = P.vis_e;
        const float xa = e[0][0] * x[0] + e[0][1] * x[1] + e[0][2] * x[2];
        const float da = e[0][0] * d[0] + e[0][1] * d[1] + e[0][2] * d[2];
        const float t = fdiv(P.vis_plane - xa, da);
        ok = ok && da != 0.f && t > 0.f && t < 1.f;
        const float q1 = e[1][0] * x[0] + e[1][1] * x[1] + e[1][2] * x[2] +
                         t * (e[1][0] * d[0] + e[1][1] * d[1] + e[1][2] * d[2]);
        const float q2 = e[2][0] * x[0] + e[2][1] * x[1] + e[2][2] * x[2] +
                         t * (e[2][0] * d[0] + e[2][1] * d[1] + e[2][2] * d[2]);
        ok = ok && q1 >= P.vis_lo1 && q1 <= P.vis_hi1 && q2 >= P.vis_lo2 && q2 <= P.vis_hi2;
    }
    // and must not pass through the (opaque) light quad, unless x is on it
    if (!CLEAR && pend != PEND_SOURCE) {
        const float dn = P.ln[0] * d[0] + P.ln[1] * d[1] + P.ln[2] * d[2];
        const float pc0 = P.lpos[0] - x[0], pc1 = P.lpos[1] - x[1], pc2 = P.lpos[2] - x[2];
        const float t = fdiv(P.ln[0] * pc0 + P.ln[1] * pc1 + P.ln[2] * pc2, dn);
        const float q0 = x[0] + t * d[0] - P.lpos[0];
        const float q1 = x[1] + t * d[1] - P.lpos[1];
        const float q2 = x[2] + t * d[2] - P.lpos[2];
        const float a = (q0 * P.lu[0] + q1 * P.lu[1] + q2 * P.lu[2]) * P.lu_inv2;
        const float b = (q0 * P.lv[0] + q1 * P.lv[1] + q2 * P.lv[2]) * P.lv_inv2;
        const bool blocked = dn != 0.f && t > 0.f && t < 1.f && a >= 0.f && a <= 1.f && b >= 0.f && b <= 1.f;
        ok = ok && !blocked;
    }
    // transmittance along the connection, through every sphere (eq. 6); past an
    // optical depth of kTauZero it is exactly 0 in fp32.  A sphere that no lane's
    // connection line meets adds nothing and is skipped by the whole wave.
    float tau = 0.f;
#pragma unroll
    for (int s = 0; s < FPT_MAX_SPHERES; ++s) {
        if (s >= P.n_spheres || !((smask >> s) & 1u)) continue;
        const float o0 = x[0] - SP[s].c[0], o1 = x[1] - SP[s].c[1], o2 = x[2] - SP[s].c[2];
        const float b = o0 * wc[0] + o1 * wc[1] + o2 * wc[2];
        const float p0 = o0 - b * wc[0], p1 = o1 - b * wc[1], p2 = o2 - b * wc[2];
        const float disc = SP[s].r2 - (p0 * p0 + p1 * p1 + p2 * p2);
        if (!__builtin_amdgcn_ballot_w64(disc > 0.f)) continue;
        const float sq = fsqrt(fmaxf(disc, 0.f));
        const float lo = fmaxf(-b - sq, 0.f), hi = fminf(-b + sq, dist);
        const float len = disc > 0.f ? fmaxf(hi - lo, 0.f) : 0.f;
        tau += wf(S, SP[s].st_row + 2 * lam) * len;
    }
    const float tr = tau < kTauZero ? __expf(-tau) : 0.f;
    const float cosc = zc * rdist;
    float v = P.wscale * f * tr * P.splat_norm * __builtin_amdgcn_rcpf(cosc * cosc * cosc * dist2) * wgt;
    SplatOut o;
    o.status = ok ? 0 : 1;
    if (ok && P.splat_rr > 0.f && tr < P.splat_rr) {
        const float q = tr * P.inv_splat_rr;
        const float u = (float)rrb * 5.9604644775390625e-08f;
        if (!(u < q)) o.status = 2;
        v = fdiv(v, q);
    }
    o.v = o.status == 0 ? v : 0.f;
    int px = min((int)(ok ? fx : 0.f), P.W - 1), py = min((int)(ok ? fy : 0.f), P.H - 1);
    if (CLEAR) {  // the host's margin keeps fx, fy inside the image; never index outside it
        px = max(px, 0);
        py = max(py, 0);
    }
    if (P.film_u32)  // the film's element count is below 2^32: 32-bit index arithmetic
        o.idx = (long long)((((uint32_t)batch * 2u + (uint32_t)comp) * (uint32_t)(P.H * P.W) +
                             (uint32_t)(py * P.W + px)) * (uint32_t)P.N + (uint32_t)lam);
    else
        o.idx = ((long long)((int)batch * 2 + comp) * (P.H * P.W) + (py * P.W + px)) * P.N + lam;
    return o;
}

// Per-block LDS tally of rare events (u32) and per-lane counters of frequent ones.
struct Counters {
    uint32_t vertices, scatters, splat_hit;
    uint32_t opaque;  // connections known to deposit exactly 0 (count_opaque)
};

DEV void lds_count(uint32_t* tally, int slot) { atomicAdd(&tally[slot], 1u); }

// Tallies of the lanes' connections known to deposit exactly 0
// (opaque_to_eye): the outcome splat_eval would give them, a hit or with
// splat_rr > 0 a roulette kill, and the count of such connections.  Called by
// the whole wave.
DEV void count_opaque(uint32_t* tally, Counters& cnt, bool opaque) {
    if (kernel_params()->splat_rr > 0.f) {  // roulette kills: rare runs, counted in LDS
        const uint64_t m = __ballot(opaque);
        if (m && lane_id() == (uint32_t)(__ffsll((unsigned long long)m) - 1)) {
            const uint32_t n = (uint32_t)__popcll(m);
            atomicAdd(&tally[FPT_T_SPLAT_OPAQUE], n);
            atomicAdd(&tally[FPT_T_SPLAT_RR_KILL], n);
        }
        return;
    }
    // hits: per-lane counters, summed when the wave ends
    cnt.opaque += opaque ? 1u : 0u;
    cnt.splat_hit += opaque ? 1u : 0u;
}

DEV void wave_sync() {
    __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
    __builtin_amdgcn_wave_barrier();
    __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
    asm volatile("" ::: "memory");
}

// -------------------------------------------------------------------------
// Deferred pinhole splats (forward renders).  A vertex that needs a camera
// connection is appended to its wave's LDS ring; whenever 64 are queued the
// wave evaluates them with every lane busy, instead of with only the lanes
// whose path happened to produce a vertex this step.  The film is a sum, so
// the order of the deposits is immaterial (up to fp32 rounding of the
// atomics, which is unordered anyway).  Entry: position, and two packed
// words: rr bits (24) | pend (2) << 24 | wall face (3) << 26 | component << 29,
// and wavelength bin | parity batch << 16.  head and count are wave-uniform.
constexpr int kSqCap = 128;             // entries per wave, a power of two >= 2 * 64
// LDS words of a wave's ring: structure of arrays of 5 words per entry, 6 with
// glossy walls (the weight word).  The sixth word is not reserved otherwise: at
// the large scene's table size it would cost a workgroup per CU.
__host__ __device__ inline int sq_words(const KParams& P) { return (P.glossy ? kEntryWords : kEntryWords - 1) * kSqCap; }

struct SplatQ {
    uint32_t* base;  // this wave's ring: [5][kSqCap] words
    uint32_t* agg;   // this wave's deposit-merging table: kAggWords words
    int held;        // its occupied slots
    int head, count;
    uint32_t* slice;  // this wave's slice of the deferred-connection buffer, or null
    int sj_n;         // entries written to it
};

// `face`: the wall face of a surface vertex, the sphere of a medium vertex.
DEV uint32_t sq_word_a(uint32_t rrb, int pend, int face, int comp) {
    return (rrb & 0xFFFFFFu) | ((uint32_t)pend << 24) | ((uint32_t)(face & 7) << 26) | ((uint32_t)comp << 29);
}

// Appends one entry per lane with `want`; at most 64, so count stays below
// kSqCap when it was below 64 before.  The weight word is written only where
// paths carry weights (WGT: scenes with glossy walls).
template <bool WGT>
DEV void sq_push(SplatQ& q, bool want, const float* x, uint32_t wa, uint32_t wb, float wgt) {
    const uint64_t m = __ballot(want);
    if (want) {
        const int k = (q.head + q.count + (int)mbcnt(m)) & (kSqCap - 1);
        q.base[k] = __float_as_uint(x[0]);
        q.base[kSqCap + k] = __float_as_uint(x[1]);
        q.base[2 * kSqCap + k] = __float_as_uint(x[2]);
        q.base[3 * kSqCap + k] = wa;
        q.base[4 * kSqCap + k] = wb;
        if constexpr (WGT) q.base[5 * kSqCap + k] = __float_as_uint(wgt);
    }
    q.count += __popcll(m);
}

// Film deposits of one wave, merged per film element before they go out.
// Consecutive vertices of a long path deep in a dense medium often project
// to the same pixel at the same wavelength, and a device atomic instruction
// whose lanes hit one address is executed lane by lane at the memory side;
// so the lanes first add their values into a small per-wave LDS hash table
// keyed by film index (linear probing; empty slots hold key kAggEmpty and
// value 0), and each occupied slot later issues one device atomic.  The table
// keeps its keys from batch to batch -- the next batches of a long path land
// mostly on the same elements -- and is written out once it holds more than
// kAggKeep keys before a batch (so it is never more than (kAggKeep + 64) /
// kAggSlots full) and when the wave ends.  Film indices must fit 32 bits below
// kAggEmpty (P.film_u32); larger films go out lane by lane.
constexpr int kAggSlots = 128;
constexpr int kAggWords = 2 * kAggSlots;  // keys, then values
constexpr uint32_t kAggEmpty = 0xFFFFFFFFu;
constexpr int kAggKeep = 32;

struct Deposit {
    bool has;
    long long idx;
    float v;
};

// One device atomic per occupied slot, leaving the table empty (whole wave).
DEV void agg_write_out(float* film, uint32_t* agg, uint32_t lane) {
    uint32_t* keys = agg;
    float* vals = reinterpret_cast<float*>(agg + kAggSlots);
    wave_sync();
#pragma unroll
    for (int j = 0; j < kAggSlots / 64; ++j) {
        const int sl = j * 64 + (int)lane;
        const uint32_t k = keys[sl];
        if (k != kAggEmpty) {
            unsafeAtomicAdd(&film[k], vals[sl]);
            keys[sl] = kAggEmpty;
            vals[sl] = 0.f;
        }
    }
    wave_sync();
}

// Adds the lanes' deposits to the table (whole wave); `held` is the
// wave-uniform count of its occupied slots.
DEV void film_add_merged(const KParams& P, float* film, uint32_t* agg, int& held, const Deposit& d,
                         uint32_t lane) {
    if (!P.film_u32) {
        if (d.has) unsafeAtomicAdd(&film[d.idx], d.v);
        return;
    }
    if (held > kAggKeep) {
        agg_write_out(film, agg, lane);
        held = 0;
    }
    uint32_t* keys = agg;
    float* vals = reinterpret_cast<float*>(agg + kAggSlots);
    bool fresh = false;  // this lane's key took an empty slot
    if (d.has) {
        const uint32_t key = (uint32_t)d.idx;
        uint32_t h = (key * 0x9E3779B1u) >> 25;  // 7 bits: kAggSlots = 128
        for (;;) {
            const uint32_t old = atomicCAS(&keys[h], kAggEmpty, key);
            fresh = old == kAggEmpty;
            if (fresh || old == key) break;
            h = (h + 1u) & (uint32_t)(kAggSlots - 1);
        }
        atomicAdd(&vals[h], d.v);
    }
    held += __popcll(__ballot(fresh));
    wave_sync();
}

// One queued connection: decode and evaluate; the deposit is returned.
template <bool CLEAR>
DEV Deposit splat_entry(const KParams& P, const uint32_t* T, const KSphere* SP, uint32_t* tally,
                        Counters& cnt, const float* x, uint32_t wa, uint32_t wb, float wgt, uint32_t smask) {
    // a CLEAR batch holds medium vertices only (splat_entries)
    const int pend = CLEAR ? PEND_MEDIUM : (int)((wa >> 24) & 3u), face = (int)((wa >> 26) & 7u);
    const int comp = (int)((wa >> 29) & 1u);
    // surface normal: the light's for its own vertex, a wall's inward normal otherwise
    const int ax = face >> 1;
    const float sg = (face & 1) ? -1.f : 1.f;
    float nrm[3];
    nrm[0] = pend == PEND_SOURCE ? P.ln[0] : (ax == 0 ? sg : 0.f);
    nrm[1] = pend == PEND_SOURCE ? P.ln[1] : (ax == 1 ? sg : 0.f);
    nrm[2] = pend == PEND_SOURCE ? P.ln[2] : (ax == 2 ? sg : 0.f);
    const SplatOut so = splat_eval<CLEAR>(T, SP, x, (int)(wb & 0xFFFFu), comp, wb >> 16, pend, nrm,
                                          wa & 0xFFFFFFu, wgt, smask);
    Deposit d;
    d.has = so.status == 0 && so.v != 0.f;  // +0 changes nothing
    d.idx = so.idx;
    d.v = so.v;
    if (so.status == 0) cnt.splat_hit++;
    else lds_count(tally, so.status == 2 ? FPT_T_SPLAT_RR_KILL : FPT_T_SPLAT_MISS);
    return d;
}

// The entries of the lanes with `valid`, evaluated together (called by the
// whole wave).  When every one is a medium vertex of the same sphere of
// P.geo_clear -- the usual case, the connections of one long path's wave
// rounds -- they take splat_eval's CLEAR form with that sphere's occluders.
DEV Deposit splat_entries(const KParams& P, const uint32_t* T, const KSphere* SP, uint32_t* tally,
                          Counters& cnt, bool valid, const float* x, uint32_t wa, uint32_t wb, float wgt) {
    const int pend = (int)((wa >> 24) & 3u), reg = (int)((wa >> 26) & 7u);
    const uint64_t act = __ballot(valid);
    Deposit d;
    d.has = false;
    d.idx = 0;
    d.v = 0.f;
    if (!act) return d;
    const int r0 = __builtin_amdgcn_readlane(reg, __ffsll((unsigned long long)act) - 1);
    const bool same = valid && pend == PEND_MEDIUM && reg == r0 && ((kernel_params()->geo_clear >> r0) & 1u);
    if (__ballot(same) == act) {
        const uint32_t smask = kernel_params()->sph_occl[r0];
        if (valid) d = splat_entry<true>(P, T, SP, tally, cnt, x, wa, wb, wgt, smask);
    } else if (valid) {
        d = splat_entry<false>(P, T, SP, tally, cnt, x, wa, wb, wgt, ~0u);
    }
    return d;
}

// Evaluates the oldest n <= 64 entries, lane i taking entry head + i.
DEV void sq_flush(const KParams& P, float* film, const uint32_t* T, const KSphere* SP, uint32_t* tally,
                  SplatQ& q, Counters& cnt, uint32_t lane, int n) {
    wave_sync();
    const bool valid = (int)lane < n;
    const int k = (q.head + (int)lane) & (kSqCap - 1);
    const float x[3] = {__uint_as_float(q.base[k]), __uint_as_float(q.base[kSqCap + k]),
                        __uint_as_float(q.base[2 * kSqCap + k])};
    const float wgt = P.glossy ? __uint_as_float(q.base[5 * kSqCap + k]) : 1.f;
    const Deposit d = splat_entries(P, T, SP, tally, cnt, valid, x, q.base[3 * kSqCap + k], q.base[4 * kSqCap + k],
                                    wgt);
    film_add_merged(P, film, q.agg, q.held, d, lane);
    q.head = (q.head + n) & (kSqCap - 1);
    q.count -= n;
    wave_sync();
}

// Once a wave's path queue is exhausted it only finishes the paths it holds,
// and the chip empties: from then on its connections go to the wave's own
// slice of a device buffer (same entry layout, structure of arrays of
// `sjob_slice` entries per wave; no atomics), which a separate launch
// evaluates with every lane busy, so the last long paths walk at the walk's
// own speed.  A full slice falls back to the LDS queue.
template <bool WGT>
DEV void splat_defer(const KBuffers& B, SplatQ& q, bool want, const float* x, uint32_t wa, uint32_t wb,
                     float wgt, bool exhausted) {
    const uint64_t m = __ballot(want);
    const int n = __popcll(m);
    if (exhausted && q.slice && q.sj_n + n <= (int)B.sjob_slice) {
        if (want) {
            const uint32_t S = B.sjob_slice;
            const uint32_t k = (uint32_t)q.sj_n + mbcnt(m);
            q.slice[k] = __float_as_uint(x[0]);
            q.slice[S + k] = __float_as_uint(x[1]);
            q.slice[2 * S + k] = __float_as_uint(x[2]);
            q.slice[3 * S + k] = wa;
            q.slice[4 * S + k] = wb;
            if constexpr (WGT) q.slice[5 * S + k] = __float_as_uint(wgt);
        }
        q.sj_n += n;
        return;
    }
    sq_push<WGT>(q, want, x, wa, wb, wgt);
}

// Full batches of 64 while there are any; with `all`, the remainder as well.
DEV void sq_drain(const KParams& P, float* film, const uint32_t* T, const KSphere* SP, uint32_t* tally,
                  SplatQ& q, Counters& cnt, uint32_t lane, bool all) {
    while (q.count >= 64 || (all && q.count > 0))
        sq_flush(P, film, T, SP, tally, q, cnt, lane, q.count < 64 ? q.count : 64);
}

// -------------------------------------------------------------------------
// Per-lane adjoint state lives in LDS: the running score S (d log p / d theta
// of the path prefix) and the chord part of the gradient, one slot per lane
// and parameter ([wave][param][lane], conflict free).
struct AdjView {
    float* S;   // + i*64
    float* Gx;  // + i*64
};

DEV void adj_add(float* base, int i, float v) { base[i * 64] += v; }

template <int MODE>
DEV void score_length(const KParams& P, const uint32_t* T, const Lane& L, AdjView& A, float len) {
    if constexpr (MODE == MODE_ADJ || MODE == MODE_REC_ADJ) {
        if (L.medium < 0 || !(len > 0.f)) return;
        const int b = P.off_med + L.medium * kMedWords;
        adj_add(A.S, wi(T, b + MW_PSS), -len);
        for (int j = 0; j < L.ndy; ++j)
            adj_add(A.S, wi(T, b + MW_PC + j),
                    -wf(T, P.off_kap + (L.medium * P.kap_stride + j) * P.N + L.lam) * len);
    }
}

// -------------------------------------------------------------------------
// Wave-cooperative walk of long paths.  Inside a homogeneous medium at a fixed
// wavelength the flight lengths, event choices and new directions of the next
// vertices depend only on their random counters, not on the position; so lane
// k of a segment draws vertex v+1+k of the segment's path, a segmented prefix
// sum of the segment vectors gives the positions, and a ballot finds the first
// vertex that leaves the medium or is not a scatter.  The scatter vertices
// before it are committed (and splat) in parallel; that vertex itself is left
// to the ordinary step.  A round serves one path with 64 lanes, two with 32 or
// four with 16.  Every width, and deep_round's 128-vertex rounds, give the
// same bits: a path walks the same way whichever lanes share its wave.
DEV float rl(float x, int j) { return __int_as_float(__builtin_amdgcn_readlane(__float_as_int(x), j)); }
// Cross-lane moves on the VALU (DPP) instead of through the LDS crossbar.
// row_shr:d takes the value of lane i-d within each row of 16 lanes; lanes
// with no source read +0 (bound_ctrl), which adds exactly (up to the sign of
// a zero sum), and with that fill the compiler folds the move into the add
// (one v_add_f32 with a DPP source instead of a fill, a move and an add).
// wave_shr:1 takes lane i-1 across the whole wave; lane 0 keeps `first`.
template <int D>
DEV float row_shr(float x) {
    return __int_as_float(__builtin_amdgcn_update_dpp(0, __float_as_int(x), 0x110 + D, 0xf, 0xf, true));
}
DEV float wave_shr1(float x, float first) {
    return __int_as_float(__builtin_amdgcn_update_dpp(__float_as_int(first), __float_as_int(x), 0x138, 0xf, 0xf,
                                                      false));
}
// Chains the rows of three prefix-summed values in place: row 0 (lanes 0..15)
// adds a base (ba, bb, bc), then row r adds lane 15 of row r-1, for r = 1, 2
// and 3 in turn (DPP with one row enabled at a time; the other rows keep
// their values).  Row r ends up with its own prefix sums plus the base and the
// totals of chunks 0..r-1 added one at a time.  Written in assembly because
// the compiler folds a DPP move into a float add only with every row enabled
// (a move, an add and a constant per step otherwise).  Each add reads its
// operand at least two instructions after writing it (the two wait states a
// DPP read needs after a VALU write); the leading s_nop covers the
// instructions before the block (five wait states, as after an EXEC write) and
// the trailing one those after it: the compiler's hazard checks do not see
// the block's writes as VALU results, so a DPP read of a result right after
// the block would otherwise get no wait states.  The whole wave must be
// active.
DEV void chain_rows3(float& a, float& b, float& c, float ba, float bb, float bc) {
    asm("s_nop 4\n\t"
        "v_add_f32_dpp %0, %3, %0 quad_perm:[0,1,2,3] row_mask:0x1 bank_mask:0xf\n\t"
        "v_add_f32_dpp %1, %4, %1 quad_perm:[0,1,2,3] row_mask:0x1 bank_mask:0xf\n\t"
        "v_add_f32_dpp %2, %5, %2 quad_perm:[0,1,2,3] row_mask:0x1 bank_mask:0xf\n\t"
        "v_add_f32_dpp %0, %0, %0 row_bcast:15 row_mask:0x2 bank_mask:0xf\n\t"
        "v_add_f32_dpp %1, %1, %1 row_bcast:15 row_mask:0x2 bank_mask:0xf\n\t"
        "v_add_f32_dpp %2, %2, %2 row_bcast:15 row_mask:0x2 bank_mask:0xf\n\t"
        "v_add_f32_dpp %0, %0, %0 row_bcast:15 row_mask:0x4 bank_mask:0xf\n\t"
        "v_add_f32_dpp %1, %1, %1 row_bcast:15 row_mask:0x4 bank_mask:0xf\n\t"
        "v_add_f32_dpp %2, %2, %2 row_bcast:15 row_mask:0x4 bank_mask:0xf\n\t"
        "v_add_f32_dpp %0, %0, %0 row_bcast:15 row_mask:0x8 bank_mask:0xf\n\t"
        "v_add_f32_dpp %1, %1, %1 row_bcast:15 row_mask:0x8 bank_mask:0xf\n\t"
        "v_add_f32_dpp %2, %2, %2 row_bcast:15 row_mask:0x8 bank_mask:0xf\n\t"
        "s_nop 1"
        : "+v"(a), "+v"(b), "+v"(c)
        : "v"(ba), "v"(bb), "v"(bc));
}
DEV int rli(int x, int j) { return __builtin_amdgcn_readlane(x, j); }
DEV uint32_t rlu(uint32_t x, int j) { return (uint32_t)__builtin_amdgcn_readlane((int)x, j); }

template <int GEOM>
DEV float medium_exit(const KParams& P, const float* x, const float* w, const float* sc, float sr2) {
    if constexpr (GEOM == FPT_GEOM_SLAB) {
        return w[2] != 0.f ? fmaxf(fdiv((w[2] > 0.f ? P.z1 : P.z0) - x[2], w[2]), 0.f) : kInf;
    } else if constexpr (GEOM == FPT_GEOM_HALFSPACE) {
        return w[2] < 0.f ? fmaxf(fdiv(P.z0 - x[2], w[2]), 0.f) : kInf;
    } else if constexpr (GEOM == FPT_GEOM_SPHERE) {
        return sphere_exit(x, w, P.bc, P.br2);
    } else if constexpr (GEOM == FPT_GEOM_INFINITE) {
        return kInf;
    } else {
        return sphere_exit(x, w, sc, sr2);
    }
}

template <int GEOM, int MODE, bool GLOSS>
DEV void block_walk(const KParams& P, const KBuffers& B, const uint32_t* T, const KSphere* SP,
                    uint32_t* tally, Lane& L, uint64_t& elig, uint32_t lane, bool pinhole,
                    Counters& cnt, float* Sw, float* Gxl, float* G, bool& full, bool& deep, SplatQ& q,
                    bool exhausted, uint64_t deepmask) {
    // the vertex arithmetic below must round exactly as deep_half's does
#pragma clang fp contract(off)
    constexpr bool ADJ = (MODE == MODE_ADJ || MODE == MODE_REC_ADJ);
    constexpr bool REC = (MODE == MODE_REC || MODE == MODE_REC_ADJ);
    // segment width: one path per 64 lanes, two per 32, or four per 16.  A
    // path whose last round ran its full width is deep in its medium and
    // likely to fill 64 lanes again: such paths go first, one per round.
    const uint64_t ed = elig & deepmask;
    uint64_t pick = ed ? ed : elig;
    const int ne = ed ? 1 : __popcll(elig);
    const int W = (ne >= 3 && P.max_segments >= 4) ? 16 : ((ne >= 2 && P.max_segments >= 2) ? 32 : 64);
    const int nseg = 64 / W;
    int own[4] = {-1, -1, -1, -1};
#pragma unroll
    for (int g = 0; g < 4; ++g) {
        if (g < nseg && pick) {
            own[g] = __ffsll((unsigned long long)pick) - 1;
            elig &= ~(1ull << own[g]);
            pick &= pick - 1ull;
        }
    }
    const int seg = (int)lane / W;
    const uint32_t pos = lane % (uint32_t)W;
    const int j = seg == 0 ? own[0] : (seg == 1 ? own[1] : (seg == 2 ? own[2] : own[3]));
    const bool active = j >= 0;
    const int js = active ? j : 0;
    // the segment owner's state: uniform (scalar) when one path takes the whole wave
    Lane Q;
    if (W == 64) {
#pragma unroll
        for (int c = 0; c < 3; ++c) {
            Q.x[c] = rl(L.x[c], js);
            Q.w[c] = rl(L.w[c], js);
            Q.sc[c] = rl(L.sc[c], js);
        }
        Q.sr2 = rl(L.sr2, js);
        Q.st = rl(L.st, js);
        Q.inv = rl(L.inv, js);
        Q.ss = rl(L.ss, js);
        Q.thr_bg = rl(L.thr_bg, js);
        Q.ndy = rli(L.ndy, js);
        Q.lam = rli(L.lam, js);
        Q.region = rli(L.region, js);
        Q.medium = rli(L.medium, js);
        Q.comp = rli(L.comp, js);
        Q.pid = rlu(L.pid, js);
        Q.v = rlu(L.v, js);
        Q.nsc = rlu(L.nsc, js);
        Q.nem = rlu(L.nem, js);
        Q.batch = rlu(L.batch, js);
        if constexpr (GLOSS) Q.wgt = rl(L.wgt, js);
    } else {
#pragma unroll
        for (int c = 0; c < 3; ++c) {
            Q.x[c] = __shfl(L.x[c], js);
            Q.w[c] = __shfl(L.w[c], js);
            Q.sc[c] = __shfl(L.sc[c], js);
        }
        Q.sr2 = __shfl(L.sr2, js);
        Q.st = __shfl(L.st, js);
        Q.inv = __shfl(L.inv, js);
        Q.ss = __shfl(L.ss, js);
        Q.thr_bg = __shfl(L.thr_bg, js);
        Q.ndy = __shfl(L.ndy, js);
        Q.lam = __shfl(L.lam, js);
        Q.region = __shfl(L.region, js);
        Q.medium = __shfl(L.medium, js);
        Q.comp = __shfl(L.comp, js);
        Q.pid = (uint32_t)__shfl((int)L.pid, js);
        Q.v = (uint32_t)__shfl((int)L.v, js);
        Q.nsc = (uint32_t)__shfl((int)L.nsc, js);
        Q.nem = (uint32_t)__shfl((int)L.nem, js);
        Q.batch = (uint32_t)__shfl((int)L.batch, js);
        if constexpr (GLOSS) Q.wgt = __shfl(L.wgt, js);
    }
    Q.splat_sum = 0.f;

    const uint32_t vk = Q.v + 1u + pos;
    const uint4 r = philox(Q.pid, vk, 0u, 0u, P.key0, P.key1);
    const float u0 = u24(r.x), u1 = u24(r.y), u2 = u24(r.z), u3 = u24(r.w);
    const float tk = neg_log1m(u0) * Q.inv;
    const bool scat = u1 * Q.st < Q.ss;
    float sp, cp;
    sincos_rev(u3, &sp, &cp);
    const float ct = __builtin_fmaf(-2.f, u2, 1.f), stt = 2.f * fsqrt(u2 * (1.f - u2));
    const float wn[3] = {stt * cp, stt * sp, ct};
    // incoming direction of segment k: the new direction of vertex k-1
    float win[3];
#pragma unroll
    for (int c = 0; c < 3; ++c) {
        const float up = wave_shr1(wn[c], Q.w[c]);
        win[c] = pos == 0 ? Q.w[c] : up;
    }
    const float seg3[3] = {tk * win[0], tk * win[1], tk * win[2]};
    // positions are built from 16-vertex chunks: an inclusive scan within the
    // chunk, then the chunk totals chained in order, exactly as consecutive
    // 16-wide rounds would add them, so every segment width gives the same bits
    float s0 = seg3[0], s1 = seg3[1], s2 = seg3[2], tt = tk;
#define FPT_SCAN_STEP(D) \
    s0 += row_shr<D>(s0); s1 += row_shr<D>(s1); s2 += row_shr<D>(s2); tt += row_shr<D>(tt);
    FPT_SCAN_STEP(1)
    FPT_SCAN_STEP(2)
    FPT_SCAN_STEP(4)
    FPT_SCAN_STEP(8)
#undef FPT_SCAN_STEP
    // chunk c of a segment adds the totals of the segment's chunks 0..c-1 in
    // order; they sit in lanes 15, 31, 47 (one 64-lane segment), 15 and 47
    // (two 32-lane segments; chunk 1 only) or nowhere (16-lane segments)
    float b0 = Q.x[0], b1 = Q.x[1], b2 = Q.x[2], bt = 0.f;
    const int chunk = (int)(pos >> 4);
    if (W >= 32) {
        const float a15[4] = {rl(s0, 15), rl(s1, 15), rl(s2, 15), rl(tt, 15)};
        const float a47[4] = {rl(s0, 47), rl(s1, 47), rl(s2, 47), rl(tt, 47)};
        const bool hi = W == 32 && seg == 1;
        if (chunk > 0) {
            b0 += hi ? a47[0] : a15[0];
            b1 += hi ? a47[1] : a15[1];
            b2 += hi ? a47[2] : a15[2];
            bt += hi ? a47[3] : a15[3];
        }
        if (W == 64) {
            const float a31[4] = {rl(s0, 31), rl(s1, 31), rl(s2, 31), rl(tt, 31)};
            if (chunk > 1) { b0 += a31[0]; b1 += a31[1]; b2 += a31[2]; bt += a31[3]; }
            if (chunk > 2) { b0 += a47[0]; b1 += a47[1]; b2 += a47[2]; bt += a47[3]; }
        }
    }
    tt += bt;
    // segment k ends at q_k if it stays in the medium, and starts where
    // segment k-1 ended (the segment's owner position for the first)
    const float qk[3] = {b0 + s0, b1 + s1, b2 + s2};
    float pk[3];
#pragma unroll
    for (int c = 0; c < 3; ++c) {
        const float up = wave_shr1(qk[c], Q.x[c]);
        pk[c] = pos == 0 ? Q.x[c] : up;
    }
    const float dif = medium_exit<GEOM>(P, pk, win, Q.sc, Q.sr2);
    bool stop = !active || !(tk < dif) || !scat || (Q.nsc + pos + 1u > P.max_scatter) ||
                (vk >= kMaxPathVertices);
    if (REC && P.max_vertices && vk >= P.max_vertices) stop = true;
    const uint64_t sm = __ballot(stop);
    const uint64_t segmask = W == 64 ? ~0ull : ((1ull << W) - 1ull);
    const uint64_t mybits = (sm >> (seg * W)) & segmask;
    const int kstar = mybits ? (__ffsll((unsigned long long)mybits) - 1) : W;
    const bool mine = active && (int)pos < kstar;
    Lane Lk = Q;
    Lk.x[0] = qk[0];
    Lk.x[1] = qk[1];
    Lk.x[2] = qk[2];
    float dep = 0.f;
    if (mine) {
        cnt.vertices++;
        cnt.scatters++;
    }
    // score of the path prefix up to vertex k (likelihood ratio of k+1 scatters)
    int pss = 0;
    float inv_ss = 0.f;
    if constexpr (ADJ) {
        const int mb = P.off_med + Q.medium * kMedWords;
        pss = wi(T, mb + MW_PSS);
        inv_ss = wf(T, mb + MW_INV_SS);
    }
    if constexpr (GEOM == FPT_GEOM_BOX && MODE == MODE_FWD) {
        if (pinhole) {
            bool want = mine && !(P.fluo_only && Q.comp == 0);
            const bool opq = want && opaque_to_eye(Lk.x, Q.region, Q.inv, Q.sc, Q.sr2);
            count_opaque(tally, cnt, opq);
            want = want && !opq;
            splat_defer<GLOSS>(B, q, want, Lk.x, sq_word_a(rr_bits(r), PEND_MEDIUM, Q.region, Q.comp),
                               (uint32_t)Q.lam | (Q.batch << 16), GLOSS ? Q.wgt : 1.f, exhausted);
        }
    } else if constexpr (GEOM == FPT_GEOM_BOX) {
        if (pinhole && mine && !(P.fluo_only && Q.comp == 0)) {
            const float zero3[3] = {0.f, 0.f, 0.f};
            const SplatOut so = splat_eval(T, SP, Lk.x, Q.lam, Q.comp, Q.batch, PEND_MEDIUM, zero3,
                                           rr_bits(r), GLOSS ? Q.wgt : 1.f);
            if (so.status == 0) {
                cnt.splat_hit++;
                dep = so.v;
                if constexpr (MODE == MODE_FWD)
                    if (so.v != 0.f) unsafeAtomicAdd(&B.film[so.idx], so.v);  // +0 changes nothing
                if constexpr (ADJ) {
                    const float gv = B.gfilm[so.idx] * so.v;
                    const int mb = P.off_med + Q.medium * kMedWords;
#pragma unroll
                    for (int i = 0; i < kMaxNP; ++i) {
                        if (i >= P.np) continue;
                        float Si = Sw[i * 64 + js];
                        if (i == pss) Si += (float)(pos + 1) * inv_ss - tt;
                        for (int q = 0; q < Q.ndy; ++q)
                            if (i == wi(T, mb + MW_PC + q))
                                Si -= wf(T, P.off_kap + (Q.medium * P.kap_stride + q) * P.N + Q.lam) * tt;
                        G[i] += gv * Si;
                    }
                    const float e0 = P.eye[0] - Lk.x[0], e1 = P.eye[1] - Lk.x[1], e2 = P.eye[2] - Lk.x[2];
                    const float dist = fsqrt(e0 * e0 + e1 * e1 + e2 * e2);
                    const float id = __builtin_amdgcn_rcpf(dist);
                    const float wc[3] = {e0 * id, e1 * id, e2 * id};
                    for (int s = 0; s < P.n_spheres; ++s) {
                        const float len = chord_len(SP[s], Lk.x, wc, dist);
                        if (!(len > 0.f)) continue;
                        const int m = SP[s].medium;
                        const int mbs = P.off_med + m * kMedWords;
                        const float c = -gv * len;
                        Gxl[wi(T, mbs + MW_PSS) * 64] += c;
                        const int nd = wi(T, mbs + MW_NDYES);
                        for (int q = 0; q < nd; ++q)
                            Gxl[wi(T, mbs + MW_PC + q) * 64] +=
                                c * wf(T, P.off_kap + (m * P.kap_stride + q) * P.N + Q.lam);
                    }
                }
            } else {
                lds_count(tally, so.status == 2 ? FPT_T_SPLAT_RR_KILL : FPT_T_SPLAT_MISS);
            }
        }
    }
    // every owner takes the state after its segment's vertex k*-1
    int myseg = -1;
#pragma unroll
    for (int g = 0; g < 4; ++g)
        if ((int)lane == own[g]) myseg = g;
    const int ks_of = [&] {
        // k* of segment `myseg`, from the uniform ballot
        if (myseg < 0) return 0;
        const uint64_t bits = (sm >> (myseg * W)) & segmask;
        return bits ? (__ffsll((unsigned long long)bits) - 1) : W;
    }();
    const int src = myseg < 0 ? 0 : myseg * W + (ks_of > 0 ? ks_of - 1 : 0);
    float nx0, nx1, nx2, nw0, nw1, nw2, tsum;
    if (W == 64) {
        // one owner: the source lane is uniform
        const int u = kstar > 0 ? kstar - 1 : 0;
        nx0 = rl(Lk.x[0], u); nx1 = rl(Lk.x[1], u); nx2 = rl(Lk.x[2], u);
        nw0 = rl(wn[0], u); nw1 = rl(wn[1], u); nw2 = rl(wn[2], u);
        tsum = rl(tt, u);
    } else {
        nx0 = __shfl(Lk.x[0], src); nx1 = __shfl(Lk.x[1], src); nx2 = __shfl(Lk.x[2], src);
        nw0 = __shfl(wn[0], src); nw1 = __shfl(wn[1], src); nw2 = __shfl(wn[2], src);
        tsum = __shfl(tt, src);
    }
    float dsum = 0.f;
    if constexpr (REC) {
        dsum = dep;
        for (int off = W >> 1; off > 0; off >>= 1) dsum += __shfl_xor(dsum, off, W);
        dsum = __shfl(dsum, myseg < 0 ? 0 : myseg * W);
    }
    // a path that committed the whole width without stopping continues with
    // another round instead of an ordinary step, whatever the width was
    if (myseg >= 0) {
        full = ks_of == W;
        // counted as deep after any full round, or only after a full round of the whole wave
        deep = full && (P.wide_rounds == 1 || W == 64);
    }
    if (myseg >= 0 && ks_of > 0) {
        L.x[0] = nx0; L.x[1] = nx1; L.x[2] = nx2;
        L.w[0] = nw0; L.w[1] = nw1; L.w[2] = nw2;
        L.v += (uint32_t)ks_of;
        L.nsc += (uint32_t)ks_of;
        if constexpr (REC) L.splat_sum += dsum;
        if constexpr (ADJ) {
            const int mb = P.off_med + L.medium * kMedWords;
            const int mpss = wi(T, mb + MW_PSS);
            Sw[mpss * 64 + lane] += (float)ks_of * wf(T, mb + MW_INV_SS) - tsum;
            for (int q = 0; q < L.ndy; ++q)
                Sw[wi(T, mb + MW_PC + q) * 64 + lane] -=
                    wf(T, P.off_kap + (L.medium * P.kap_stride + q) * P.N + L.lam) * tsum;
        }
    }
}

// A deep path in a forward render (its last round ran the whole wave) walks
// 128 vertices per round: lane k draws vertices v+1+k and, once the first 64
// are all committed, v+65+k.  The second half's positions chain from the
// first half's last vertex exactly as a following 64-lane round would, so
// the result is the same as two consecutive rounds.  (Drawing both halves
// together, for the overlap of their independent generator work, cost 1.4 %
// more on the large scene: the waves of a full chip hide that latency anyway,
// and a round that stops in its first half then wasted the second.)
template <int GEOM>
DEV void deep_half(const KParams& P, const Lane& Q, uint32_t v0, uint32_t lane, const float* wprev,
                   const float* xbase, float* wn, float* xk, float* pk, float* win, bool& stop_out) {
    // the vertex arithmetic rounds exactly as block_walk's does
#pragma clang fp contract(off)
    const uint32_t vk = v0 + 1u + lane;
    const uint4 r = philox(Q.pid, vk, 0u, 0u, P.key0, P.key1);
    const float u0 = u24(r.x), u1 = u24(r.y), u2 = u24(r.z), u3 = u24(r.w);
    const float tk = neg_log1m(u0) * Q.inv;
    const bool scat = u1 * Q.st < Q.ss;
    float sp, cp;
    sincos_rev(u3, &sp, &cp);
    const float ct = __builtin_fmaf(-2.f, u2, 1.f), stt = 2.f * fsqrt(u2 * (1.f - u2));
    wn[0] = stt * cp;
    wn[1] = stt * sp;
    wn[2] = ct;
#pragma unroll
    for (int c = 0; c < 3; ++c) win[c] = wave_shr1(wn[c], wprev[c]);
    const float seg3[3] = {tk * win[0], tk * win[1], tk * win[2]};
    float s0 = seg3[0], s1 = seg3[1], s2 = seg3[2];
#define FPT_SCAN3(D) s0 += row_shr<D>(s0); s1 += row_shr<D>(s1); s2 += row_shr<D>(s2);
    FPT_SCAN3(1)
    FPT_SCAN3(2)
    FPT_SCAN3(4)
    FPT_SCAN3(8)
#undef FPT_SCAN3
    // chunk 0 adds the base, then each chunk the position its predecessor
    // ended at: the chunk totals chained in order, exactly as block_walk's
    // readlane adds chain them (a + b rounds as b + a).  The DPP chain is
    // used by the box kernel only: in the smaller body-medium kernels its
    // operands in vector registers cost more registers (occupancy) than the
    // readlanes it saves (slab, 2^22 paths: 0.79 ms with readlanes, 0.87 ms
    // with the chain).
    if constexpr (GEOM == FPT_GEOM_BOX) {
        xk[0] = s0;
        xk[1] = s1;
        xk[2] = s2;
        chain_rows3(xk[0], xk[1], xk[2], xbase[0], xbase[1], xbase[2]);
    } else {
        float b0 = xbase[0], b1 = xbase[1], b2 = xbase[2];
        const int chunk = (int)(lane >> 4);
        const float a15[3] = {rl(s0, 15), rl(s1, 15), rl(s2, 15)};
        const float a31[3] = {rl(s0, 31), rl(s1, 31), rl(s2, 31)};
        const float a47[3] = {rl(s0, 47), rl(s1, 47), rl(s2, 47)};
        if (chunk > 0) { b0 += a15[0]; b1 += a15[1]; b2 += a15[2]; }
        if (chunk > 1) { b0 += a31[0]; b1 += a31[1]; b2 += a31[2]; }
        if (chunk > 2) { b0 += a47[0]; b1 += a47[1]; b2 += a47[2]; }
        xk[0] = b0 + s0;
        xk[1] = b1 + s1;
        xk[2] = b2 + s2;
    }
    // each segment starts where the one before it ended
#pragma unroll
    for (int c = 0; c < 3; ++c) pk[c] = wave_shr1(xk[c], xbase[c]);
    const float dif = medium_exit<GEOM>(P, pk, win, Q.sc, Q.sr2);
    stop_out = !(tk < dif) || !scat || (Q.nsc + (vk - Q.v) > P.max_scatter) || (vk >= kMaxPathVertices);
    // the rr bits of the vertex's own uniforms, for its camera connection
    xk[3] = __uint_as_float(rr_bits(r));
}

// splat_eval's CLEAR form for the usual case of a deep round's half: a
// medium vertex inside sphere sp, whose only possible occluder is sp itself,
// with the film's element count below 2^32.  The same operations in the same
// order (so the same deposit), written for that case: one chord, the medium's
// factor, 32-bit film indices.  `base` = ((batch * 2 + comp) * H * W) * N + lam,
// uniform over the half.  Roulette and its status as in splat_eval.
DEV SplatOut splat_own_sphere(const uint32_t* S, const KSphere& sp, const EyeRay& ray, int lam, uint32_t base,
                              uint32_t rrb, float wgt) {
    const auto& P = *kernel_params();
    const float* d = ray.d;
    const float dist2 = ray.dist2;
    const float rdist = ray.rdist;
    const float dist = dist2 * rdist;
    const float wc[3] = {d[0] * rdist, d[1] * rdist, d[2] * rdist};
    const float zc = -(d[0] * P.cf[0] + d[1] * P.cf[1] + d[2] * P.cf[2]);
    const float izc = __builtin_amdgcn_rcpf(zc);
    const float xi = -(d[0] * P.cr[0] + d[1] * P.cr[1] + d[2] * P.cr[2]) * izc * P.inv_tanx;
    const float yi = -(d[0] * P.cu[0] + d[1] * P.cu[1] + d[2] * P.cu[2]) * izc * P.inv_tany;
    const float fx = (xi + 1.f) * 0.5f * (float)P.W;
    const float fy = (1.f - yi) * 0.5f * (float)P.H;
    const float o0 = ray.o[0], o1 = ray.o[1], o2 = ray.o[2];
    const float b = o0 * wc[0] + o1 * wc[1] + o2 * wc[2];
    const float p0 = o0 - b * wc[0], p1 = o1 - b * wc[1], p2 = o2 - b * wc[2];
    const float disc = sp.r2 - (p0 * p0 + p1 * p1 + p2 * p2);
    const float sq = fsqrt(fmaxf(disc, 0.f));
    const float lo = fmaxf(-b - sq, 0.f), hi = fminf(-b + sq, dist);
    const float len = disc > 0.f ? fmaxf(hi - lo, 0.f) : 0.f;
    const float tau = 0.f + wf(S, sp.st_row + 2 * lam) * len;
    const float tr = tau < kTauZero ? __expf(-tau) : 0.f;
    const float cosc = zc * rdist;
    float v = P.wscale * kInv4Pi * tr * P.splat_norm * __builtin_amdgcn_rcpf(cosc * cosc * cosc * dist2) * wgt;
    SplatOut o;
    o.status = 0;
    if (P.splat_rr > 0.f && tr < P.splat_rr) {
        const float q = tr * P.inv_splat_rr;
        const float u = (float)rrb * 5.9604644775390625e-08f;
        if (!(u < q)) o.status = 2;
        v = fdiv(v, q);
    }
    o.v = o.status == 0 ? v : 0.f;
    const int px = max(min((int)fx, P.W - 1), 0), py = max(min((int)fy, P.H - 1), 0);
    o.idx = (long long)(base + (uint32_t)(py * P.W + px) * (uint32_t)P.N);
    return o;
}

// The camera connections of one half of a deep round, all of one path: one
// wavelength, component, parity slice and sphere.  When every committed
// vertex of the half connects (none was found opaque), its sphere passes the
// geometric tests (P.geo_clear) and the path queue is not yet exhausted, the
// half evaluates them in place, with as many lanes busy as a full ring batch
// and the path's values uniform; the ring's push, read-back and decode are
// saved.  Otherwise they join the ring.  `committed`: the half's committed
// lanes; x[3] holds the vertex's roulette bits.
template <bool GLOSS>
DEV void deep_connect(const KParams& P, const KBuffers& B, const uint32_t* T, const KSphere* SP, uint32_t* tally,
                      SplatQ& q, Counters& cnt, uint32_t lane, bool want, uint64_t committed, const float* x,
                      const EyeRay& ray, const Lane& Q, uint32_t wb, bool exhausted) {
    const uint64_t wm = __ballot(want);
    const auto& K = *kernel_params();
    if (wm && wm == committed && !exhausted && Q.region >= 0 && ((K.geo_clear >> (uint32_t)Q.region) & 1u)) {
        Deposit d;
        d.has = false;
        d.idx = 0;
        d.v = 0.f;
        const uint32_t occl = K.sph_occl[Q.region];
        const bool own = occl == (1u << (uint32_t)Q.region) && K.film_u32;
        const uint32_t base = (((uint32_t)Q.batch * 2u + (uint32_t)Q.comp) * (uint32_t)(K.H * K.W)) * (uint32_t)K.N +
                              (uint32_t)Q.lam;
        if (want) {
            const float zero3[3] = {0.f, 0.f, 0.f};
            const SplatOut so = own ? splat_own_sphere(T, SP[Q.region], ray, Q.lam, base, __float_as_uint(x[3]),
                                                       GLOSS ? Q.wgt : 1.f)
                                    : splat_eval<true>(T, SP, x, Q.lam, Q.comp, Q.batch, PEND_MEDIUM, zero3,
                                                       __float_as_uint(x[3]), GLOSS ? Q.wgt : 1.f, occl);
            d.has = so.status == 0 && so.v != 0.f;  // +0 changes nothing
            d.idx = so.idx;
            d.v = so.v;
            if (so.status == 0) cnt.splat_hit++;
            else lds_count(tally, so.status == 2 ? FPT_T_SPLAT_RR_KILL : FPT_T_SPLAT_MISS);
        }
        film_add_merged(P, B.film, q.agg, q.held, d, lane);
        return;
    }
    splat_defer<GLOSS>(B, q, want, x, sq_word_a(__float_as_uint(x[3]), PEND_MEDIUM, Q.region, Q.comp), wb,
                       GLOSS ? Q.wgt : 1.f, exhausted);
}

// Consecutive rounds of one path run in one call while each commits all 128
// vertices (at most kDeepRounds): the path's state stays uniform between them
// instead of being read back from its lane each round, and the rounds are the
// same as separate calls would walk.  Measured on the large scene: 4 rounds
// per call 58.8 ms, 16 57.8 ms, 32 or more 57.7 ms (2 rounds 60.3 ms).
constexpr int kDeepRounds = 1024;

template <int GEOM, bool GLOSS>
DEV void deep_round(const KParams& P, const KBuffers& B, const uint32_t* T, const KSphere* SP,
                    uint32_t* tally, Lane& L, int j, uint32_t lane, bool pinhole, Counters& cnt, bool& full,
                    SplatQ& q, bool exhausted) {
    Lane Q;
#pragma unroll
    for (int c = 0; c < 3; ++c) {
        Q.x[c] = rl(L.x[c], j);
        Q.w[c] = rl(L.w[c], j);
        Q.sc[c] = rl(L.sc[c], j);
    }
    Q.sr2 = rl(L.sr2, j);
    Q.st = rl(L.st, j);
    Q.inv = rl(L.inv, j);
    Q.ss = rl(L.ss, j);
    Q.lam = rli(L.lam, j);
    Q.region = rli(L.region, j);
    Q.comp = rli(L.comp, j);
    Q.pid = rlu(L.pid, j);
    Q.v = rlu(L.v, j);
    Q.nsc = rlu(L.nsc, j);
    Q.batch = rlu(L.batch, j);
    Q.wgt = GLOSS ? rl(L.wgt, j) : 1.f;
    const bool dep = !(P.fluo_only && Q.comp == 0);
    const uint32_t wb = (uint32_t)Q.lam | (Q.batch << 16);
    uint32_t walked = 0;
    for (int round = 0;; ++round) {
        float wn1[3], x1[4], p1[3], win1[3], wn2[3], x2[4], p2[3], win2[3];
        bool st1, st2;
        deep_half<GEOM>(P, Q, Q.v, lane, Q.w, Q.x, wn1, x1, p1, win1, st1);
        const uint64_t sm1 = __ballot(st1);
        const int k1 = sm1 ? (__ffsll((unsigned long long)sm1) - 1) : 64;
        int k2 = 0;
        x2[0] = x2[1] = x2[2] = x2[3] = 0.f;
        wn2[0] = wn2[1] = wn2[2] = 0.f;
        if (k1 == 64) {
            // the second half starts from the state after the first half's vertex 64
            const float w64[3] = {rl(wn1[0], 63), rl(wn1[1], 63), rl(wn1[2], 63)};
            const float x64[3] = {rl(x1[0], 63), rl(x1[1], 63), rl(x1[2], 63)};
            deep_half<GEOM>(P, Q, Q.v + 64u, lane, w64, x64, wn2, x2, p2, win2, st2);
            const uint64_t sm2 = __ballot(st2);
            k2 = sm2 ? (__ffsll((unsigned long long)sm2) - 1) : 64;
        }
        const bool m1 = (int)lane < k1, m2 = (int)lane < k2;
        cnt.vertices += (uint32_t)m1 + (uint32_t)m2;
        cnt.scatters += (uint32_t)m1 + (uint32_t)m2;
        if constexpr (GEOM == FPT_GEOM_BOX) {
            if (pinhole) {
                const EyeRay r1 = eye_ray(x1, Q.sc);
                const bool o1 = m1 && dep && opaque_to_eye(r1, Q.region, Q.inv, Q.sr2);
                count_opaque(tally, cnt, o1);
                const bool w1 = m1 && dep && !o1;
                const uint64_t c1 = k1 >= 64 ? ~0ull : ((1ull << k1) - 1ull);
                deep_connect<GLOSS>(P, B, T, SP, tally, q, cnt, lane, w1, c1, x1, r1, Q, wb, exhausted);
                sq_drain(P, B.film, T, SP, tally, q, cnt, lane, false);
                if (k2 > 0) {
                    const EyeRay r2 = eye_ray(x2, Q.sc);
                    const bool o2 = m2 && dep && opaque_to_eye(r2, Q.region, Q.inv, Q.sr2);
                    count_opaque(tally, cnt, o2);
                    const bool w2 = m2 && dep && !o2;
                    const uint64_t c2 = k2 >= 64 ? ~0ull : ((1ull << k2) - 1ull);
                    deep_connect<GLOSS>(P, B, T, SP, tally, q, cnt, lane, w2, c2, x2, r2, Q, wb, exhausted);
                }
            }
        }
        const int k = k1 + k2;
        full = k == 128;
        if (k > 0) {
            // the state after the last committed vertex (the source is uniform)
            const int u = (k2 > 0 ? k2 : k1) - 1;
            const bool h2 = k2 > 0;
#pragma unroll
            for (int c = 0; c < 3; ++c) {
                Q.x[c] = rl(h2 ? x2[c] : x1[c], u);
                Q.w[c] = rl(h2 ? wn2[c] : wn1[c], u);
            }
            Q.v += (uint32_t)k;
            Q.nsc += (uint32_t)k;
            walked += (uint32_t)k;
        }
        if (!full || round + 1 == kDeepRounds) break;
        // the ring holds fewer than 64 entries before the next round's appends
        if constexpr (GEOM == FPT_GEOM_BOX) {
            if (pinhole) sq_drain(P, B.film, T, SP, tally, q, cnt, lane, false);
        }
    }
    if (walked > 0 && (int)lane == j) {
        L.x[0] = Q.x[0]; L.x[1] = Q.x[1]; L.x[2] = Q.x[2];
        L.w[0] = Q.w[0]; L.w[1] = Q.w[1]; L.w[2] = Q.w[2];
        L.v += walked;
        L.nsc += walked;
    }
}

// -------------------------------------------------------------------------
// Glossy wall reflection: the normalised modified-Phong lobe of exponent n,
// rho (n+2)/(2 pi) cos^n(alpha), alpha measured from the mirror direction of
// the incoming direction w about the wall `face` (sec. 5: glossy Cornell box).
// The path survived the reflection test with probability rho, so its camera
// connection at this vertex is weighted by the lobe toward the eye over the
// Lambertian cos/pi the splat evaluates: (n+2)/2 cos^n(alpha_eye) (`lobe`).
// The new direction is drawn from the lobe: cos alpha = u2^(1/(n+1)), azimuth
// (sp, cp) = 2 pi u3, in the orthonormal basis of Duff et al. (2017) about the
// mirror direction.  Returns false when it falls below the wall (the path ends
// there), else sets w and the throughput factor (n+2)/(n+1) cos(theta_o).
DEV bool glossy_reflect(float n, int face, float u2, float sp, float cp, const float* x, float* w,
                        float* nrm, float& lobe, float& factor) {
    const auto& K = *kernel_params();
    const int ax = face >> 1;
    const float sg = (face & 1) ? -1.f : 1.f;
    nrm[0] = ax == 0 ? sg : 0.f;
    nrm[1] = ax == 1 ? sg : 0.f;
    nrm[2] = ax == 2 ? sg : 0.f;
    // mirror about an axis-aligned wall: negate the normal component
    const float r[3] = {ax == 0 ? -w[0] : w[0], ax == 1 ? -w[1] : w[1], ax == 2 ? -w[2] : w[2]};
    const float d0 = K.eye[0] - x[0], d1 = K.eye[1] - x[1], d2 = K.eye[2] - x[2];
    const float ce = (r[0] * d0 + r[1] * d1 + r[2] * d2) * __builtin_amdgcn_rsqf(d0 * d0 + d1 * d1 + d2 * d2);
    lobe = ce > 0.f ? (n + 2.f) * 0.5f * __builtin_amdgcn_exp2f(n * __builtin_amdgcn_logf(ce)) : 0.f;
    // cos alpha = u2^(1/(n+1)) = 2^y; sin^2 alpha = 1 - 2^(2y) = -expm1(2 y ln 2),
    // by its Taylor series where 2y ln 2 is small (a sharp lobe puts cos alpha
    // next to 1, where 1 - cos^2 would cancel), else directly
    const float y = u2 > 0.f ? __builtin_amdgcn_logf(u2) * __builtin_amdgcn_rcpf(n + 1.f) : -kInf;
    const float ca = __builtin_amdgcn_exp2f(y);
    const float e = 2.f * 0.693147180559945309f * y;
    float s2;
    if (e > -0.5f) {
        float t = 1.f + e * (1.f / 8.f);
        t = 1.f + e * (1.f / 7.f) * t;
        t = 1.f + e * (1.f / 6.f) * t;
        t = 1.f + e * (1.f / 5.f) * t;
        t = 1.f + e * (1.f / 4.f) * t;
        t = 1.f + e * (1.f / 3.f) * t;
        t = 1.f + e * (1.f / 2.f) * t;
        s2 = -e * t;
    } else {
        s2 = 1.f - ca * ca;
    }
    const float sa = fsqrt(fmaxf(0.f, s2));
    const float sz = r[2] >= 0.f ? 1.f : -1.f;
    const float a = -__builtin_amdgcn_rcpf(sz + r[2]);
    const float b = r[0] * r[1] * a;
    const float t1[3] = {1.f + sz * r[0] * r[0] * a, sz * b, -sz * r[0]};
    const float t2[3] = {b, sz + r[1] * r[1] * a, -r[1]};
    const float p = sa * cp, q = sa * sp;
    const float wo[3] = {p * t1[0] + q * t2[0] + ca * r[0], p * t1[1] + q * t2[1] + ca * r[1],
                         p * t1[2] + q * t2[2] + ca * r[2]};
    const float co = sg * (ax == 0 ? wo[0] : (ax == 1 ? wo[1] : wo[2]));
    if (!(co > 0.f)) {
        factor = 0.f;
        return false;
    }
    w[0] = wo[0];
    w[1] = wo[1];
    w[2] = wo[2];
    factor = (n + 2.f) * __builtin_amdgcn_rcpf(n + 1.f) * co;
    return true;
}

// -------------------------------------------------------------------------
// Per-wave context and per-lane walk state, shared by the single-scene and the
// batched persistent kernels.
struct WaveCtx {
    const uint32_t* T;   // table image (LDS)
    const KSphere* SP;   // sphere table (LDS)
    uint32_t* tally;     // u32[FPT_N_TALLIES] event counters (LDS)
    uint32_t* hist;      // escape histogram (LDS) when lds_hist
    bool lds_hist;
    bool pinhole;
    uint32_t lane;
};

struct WalkState {
    Lane L;
    bool alive, fresh;
    bool deep;  // the path's last wave-block round ran its full width
    int pend;
    int face;  // wall face of a pending surface splat (deferred splats)
    float nrm[3];
    uint32_t rrb;
    // glossy walls: the pending splat is a glossy reflection weighted by `sw`
    // (the path's weight times the lobe toward the eye), and the path ends
    // after it (its sampled direction fell below the wall)
    float sw;
    bool gspl, gdie;
    Counters cnt;
    SplatQ q;
};

// A dead lane takes path `pid`; its light vertex is drawn in the lane's next
// step, together with the vertices of the paths in flight.
DEV void assign_path(WalkState& W, uint32_t pid) {
    W.L.pid = pid;
    W.L.v = 0;
    W.alive = true;
    W.fresh = true;
    W.deep = false;
}

// One iteration of the walk for every live lane: wave-cooperative blocks for
// long paths, one segment of the walk, the convergent splat section and the
// bookkeeping of paths that ended.
// REFR: the body medium has a refracting boundary (index != 1).  A separate
// instantiation, because the Fresnel code costs registers (and with them
// occupancy) even in launches that never run it.
template <int GEOM, int MODE, bool REFR>
DEV void advance(const KParams& P, const KBuffers& B, const WaveCtx& C, WalkState& W, AdjView& A,
                 float* G, bool exhausted) {
    constexpr bool DEFER = (GEOM == FPT_GEOM_BOX && MODE == MODE_FWD);  // queued splats
    // in a box the refraction instantiation flag selects glossy walls instead
    // (per-path throughput weights)
    constexpr bool kGloss = REFR && GEOM == FPT_GEOM_BOX;
    constexpr bool ADJ = (MODE == MODE_ADJ || MODE == MODE_REC_ADJ);
    constexpr bool REC = (MODE == MODE_REC || MODE == MODE_REC_ADJ);
    (void)ADJ;
    (void)REC;
    Lane& L = W.L;
    bool& alive = W.alive;
    bool& fresh = W.fresh;
    int& pend = W.pend;
    float* nrm = W.nrm;
    uint32_t& rrb = W.rrb;
    Counters& cnt = W.cnt;
    const uint32_t* T = C.T;
    const KSphere* SP = C.SP;
    uint32_t* tally = C.tally;
    uint32_t* hist = C.hist;
    const bool lds_hist = C.lds_hist;
    const bool pinhole = C.pinhole;
    const uint32_t lane = C.lane;
    (void)SP;
    (void)hist;
    (void)lds_hist;
    (void)pinhole;
    (void)tally;
    (void)lane;
    // ---- long paths: wave-cooperative blocks of up to 64 vertices each
    bool full = false;
    bool deep = false;  // this iteration's last round of the path filled the whole wave
    const uint64_t dm = __ballot(W.deep);
    // a wave holding a deep path issues first on its SIMD while it walks blocks:
    // such paths set the end of the launch
    if (dm) __builtin_amdgcn_s_setprio(2);
    if constexpr (MODE != MODE_REC_ADJ) {
        // paths whose last block ran its full width without stopping go again,
        // up to kBlockPasses passes per iteration.  The box forward kernel takes
        // one: such a path skips its step and goes again in the next iteration.
        // There further passes kept loop-invariant lane masks live across its
        // large round code, spilled to VGPR lanes (four passes: the large scene
        // 0.8 % slower), while the slab and adjoint kernels gain from them
        // (one pass: 4 % and 1.5 % slower).
        constexpr int kPasses = (GEOM == FPT_GEOM_BOX && MODE == MODE_FWD) ? 1 : kBlockPasses;
        for (int pass = 0; pass < kPasses; ++pass) {
            uint64_t elig = __ballot(alive && !fresh && L.v >= P.block_min_v && L.medium >= 0 &&
                                     L.st > 0.f && (P.exc_scatter || L.nem > 0u) &&
                                     (pass == 0 || full));
            if (!elig) break;
            // paths whose round in this iteration filled the whole wave
            const uint64_t deepm = pass == 0 ? dm : __ballot(deep);
            while (elig) {  // each round takes up to four long paths off `elig`
                if constexpr (MODE == MODE_FWD) {
                    const uint64_t ed = P.wide_rounds ? (elig & deepm) : 0ull;
                    if (ed) {
                        const int j = __ffsll((unsigned long long)ed) - 1;
                        elig &= ~(1ull << j);
                        bool fj = false;
                        deep_round<GEOM, kGloss>(P, B, T, SP, tally, L, j, lane, pinhole, cnt, fj, W.q, exhausted);
                        if ((int)lane == j) {
                            full = fj;
                            deep = fj;
                        }
                        if constexpr (DEFER) sq_drain(P, B.film, T, SP, tally, W.q, cnt, lane, false);
                        continue;
                    }
                }
                block_walk<GEOM, MODE, kGloss>(P, B, T, SP, tally, L, elig, lane, pinhole, cnt,
                                       ADJ ? A.S - lane : nullptr, ADJ ? A.Gx : nullptr, G, full, deep, W.q,
                                       exhausted, deepm);
                if constexpr (DEFER) sq_drain(P, B.film, T, SP, tally, W.q, cnt, lane, false);
            }
        }
    }

    __builtin_amdgcn_s_setprio(0);
    W.deep = deep;
    // ---- one step for every live lane: the light vertex of a path assigned in
    // this iteration, or the next vertex of a path in flight.  Both draw their
    // uniforms from the same Philox calls (counter (pid, vertex, call, 0)), so a
    // new path costs no evaluation of the generator of its own.
    int ev = EV_NONE;
    int exit_code = -1;
    constexpr bool kBody = REFR && (GEOM == FPT_GEOM_SLAB || GEOM == FPT_GEOM_HALFSPACE || GEOM == FPT_GEOM_SPHERE);
    // escape through the body boundary or the open face: escape tally by side
    auto escape = [&]() {
        const int side = L.w[2] < 0.f ? 0 : 1;
        exit_code = side == 0 ? FPT_EXIT_ESC_R : FPT_EXIT_ESC_T;
        if (!pinhole && !(P.fluo_only && L.comp == 0)) {
            const int idx = ((L.batch * 2 + L.comp) * 2 + side) * P.N + L.lam;
            if constexpr (MODE == MODE_FWD) {
                if (lds_hist) atomicAdd(&hist[idx], 1u);
                else atomicAdd(&B.counts[idx], 1u);
            }
            L.splat_sum += P.wscale;
            if constexpr (ADJ) {
                const float g = B.gfilm[idx] * P.wscale;
#pragma unroll
                for (int i = 0; i < kMaxNP; ++i)
                    if (i < P.np) G[i] += g * A.S[i * 64];
            }
        }
    };
    // ---- vertex 0 of every path assigned in this iteration: the light (eq. 12;
    // counter (pid, 0): call 0 picks the excitation line and, on a quad, the
    // point, call 1 the direction).  Its camera connection is made at once and
    // the path takes its first flight in the same iteration, below, so a new
    // path costs no iteration of its own.
    if (alive && fresh) {
        cnt.vertices++;
        const uint4 r = philox(L.pid, 0u, 0u, 0u, P.key0, P.key1);
        const float u0 = u24(r.x), u1 = u24(r.y), u2 = u24(r.z);
        L.nsc = 0;
        L.nem = 0;
        L.comp = 0;
        if constexpr (kGloss) L.wgt = 1.f;
        L.batch = L.pid % P.batches;
        L.splat_sum = 0.f;
        int line = 0;
        for (; line < P.n_lines - 1; ++line)
            if (u0 < P.line_cum[line]) break;
        L.lam = P.line_bin[line];
        if constexpr (ADJ) {
#pragma unroll
            for (int i = 0; i < kMaxNP; ++i) A.S[i * 64] = 0.f;
        }
        bool reflected = false;  // off a refractive body on entry
        if (P.light == FPT_LIGHT_BEAM) {
            L.x[0] = P.lpos[0]; L.x[1] = P.lpos[1]; L.x[2] = P.lpos[2];
            L.w[0] = P.ldir[0]; L.w[1] = P.ldir[1]; L.w[2] = P.ldir[2];
            L.region = 0;
            if constexpr (kBody) {
                if (P.ior != 1.f) {
                    // entering a refractive body: Fresnel reflection (the path
                    // leaves at once) or refraction by Snell's law; u1 decides
                    float nb[3], ct;
                    const float ws[3] = {-L.w[0], -L.w[1], -L.w[2]};
                    body_normal<GEOM>(P, L.x, ws, nb);
                    const float ci = -dot3(L.w, nb);
                    if (u1 < fresnel(ci, 1.f, P.ior, ct)) {
                        mirror(L.w, nb);
                        lds_count(tally, FPT_T_WALL_REFLECT);
                        reflected = true;
                    } else {
                        const float eta = __builtin_amdgcn_rcpf(P.ior), k = eta * ci - ct;
                        float t3[3];
#pragma unroll
                        for (int i = 0; i < 3; ++i) t3[i] = eta * L.w[i] + k * nb[i];
                        const float s = __builtin_amdgcn_rsqf(dot3(t3, t3));
                        L.w[0] = t3[0] * s; L.w[1] = t3[1] * s; L.w[2] = t3[2] * s;
                    }
                }
            }
        } else {
            const uint4 r1 = philox(L.pid, 0u, 1u, 0u, P.key0, P.key1);
            const float ua = u24(r1.x), ub = u24(r1.y);
            float sp, cp;
            sincos_rev(ub, &sp, &cp);
            if (P.light == FPT_LIGHT_POINT) {
                L.x[0] = P.lpos[0]; L.x[1] = P.lpos[1]; L.x[2] = P.lpos[2];
                const float ct = 1.f - 2.f * ua;
                const float st = 2.f * fsqrt(ua * (1.f - ua));
                L.w[0] = st * cp; L.w[1] = st * sp; L.w[2] = ct;
                L.region = 0;
            } else {
                const float a = u1, b = u2;
                const float sr = fsqrt(ua), cz = fsqrt(1.f - ua);
                const float lx = sr * cp, ly = sr * sp;
#pragma unroll
                for (int i = 0; i < 3; ++i) {
                    L.x[i] = P.lpos[i] + a * P.lu[i] + b * P.lv[i];
                    L.w[i] = lx * P.lt1[i] + ly * P.lt2[i] + cz * P.ln[i];
                }
                L.region = -1;
            }
        }
        L.medium = (GEOM == FPT_GEOM_BOX) ? -1 : P.body_medium;
        L.sc[0] = L.sc[1] = L.sc[2] = 0.f;
        L.sr2 = 0.f;
        load_medium(P, T, L);
        if (reflected) escape();
        if (pinhole && P.light == FPT_LIGHT_QUAD) {
            pend = PEND_SOURCE;
            nrm[0] = P.ln[0]; nrm[1] = P.ln[1]; nrm[2] = P.ln[2];
            rrb = rr_bits(r);
        }
    }
    // ---- convergent splat section: the pending camera connection of every
    // lane (the light vertex's, then the step's).  `medium`: the vertex may be
    // a medium vertex (not for light vertices).
    auto connect = [&](const bool medium) {
        if constexpr (DEFER) {
            if (pinhole) {
                bool want = pend != PEND_NONE && alive && (exit_code < 0 || (kGloss && W.gdie)) &&
                            !(P.fluo_only && L.comp == 0);
                const bool opq = want && medium && pend == PEND_MEDIUM &&
                                 opaque_to_eye(L.x, L.region, L.inv, L.sc, L.sr2);
                count_opaque(tally, cnt, opq);
                want = want && !opq;
                float sw = 1.f;
                if constexpr (kGloss) sw = W.gspl ? W.sw : L.wgt;
                splat_defer<kGloss>(B, W.q, want, L.x,
                                    sq_word_a(rrb, pend, pend == PEND_MEDIUM ? L.region : W.face, L.comp),
                                    (uint32_t)L.lam | (L.batch << 16), sw, exhausted);
            }
        } else if constexpr (GEOM == FPT_GEOM_BOX) {
            if (pinhole && pend != PEND_NONE && alive && (exit_code < 0 || (kGloss && W.gdie))) {
                if (!(P.fluo_only && L.comp == 0)) {
                    float sw = 1.f;
                    if constexpr (kGloss) sw = W.gspl ? W.sw : L.wgt;
                    const SplatOut so = splat_eval(T, SP, L.x, L.lam, L.comp, L.batch, pend, nrm, rrb, sw);
                    if (so.status == 0) {
                        cnt.splat_hit++;
                        L.splat_sum += so.v;
                        if constexpr (MODE == MODE_FWD)
                        if (so.v != 0.f) unsafeAtomicAdd(&B.film[so.idx], so.v);  // +0 changes nothing
                        if constexpr (ADJ) {
                            const float g = B.gfilm[so.idx];
                            const float gv = g * so.v;
#pragma unroll
                            for (int i = 0; i < kMaxNP; ++i)
                                if (i < P.np) G[i] += gv * A.S[i * 64];
                            // d v / d theta = -v sum_s chord_s d sigma_t(m_s) / d theta
                            const float e0 = P.eye[0] - L.x[0], e1 = P.eye[1] - L.x[1], e2 = P.eye[2] - L.x[2];
                            const float dist = fsqrt(e0 * e0 + e1 * e1 + e2 * e2);
                            const float id = __builtin_amdgcn_rcpf(dist);
                            const float wc[3] = {e0 * id, e1 * id, e2 * id};
                            for (int s = 0; s < P.n_spheres; ++s) {
                                const float len = chord_len(SP[s], L.x, wc, dist);
                                if (!(len > 0.f)) continue;
                                const int m = SP[s].medium;
                                const int mb = P.off_med + m * kMedWords;
                                const float c = -gv * len;
                                adj_add(A.Gx, wi(T, mb + MW_PSS), c);
                                const int nd = wi(T, mb + MW_NDYES);
                                for (int j = 0; j < nd; ++j)
                                    adj_add(A.Gx, wi(T, mb + MW_PC + j),
                                            c * wf(T, P.off_kap + (m * P.kap_stride + j) * P.N + L.lam));
                            }
                        }
                    } else {
                        lds_count(tally, so.status == 2 ? FPT_T_SPLAT_RR_KILL : FPT_T_SPLAT_MISS);
                    }
                }
            }
        }
        pend = PEND_NONE;
        if constexpr (kGloss) {
            W.gspl = false;
            W.gdie = false;
        }
    };
    if (__ballot(pend != PEND_NONE)) {
        connect(false);
        // the ring holds fewer than 64 entries before each append
        if constexpr (DEFER) {
            if (pinhole) sq_drain(P, B.film, T, SP, tally, W.q, cnt, lane, false);
        }
    }
    // ---- one step for every live lane: the next vertex, from the counter
    // (pid, vertex) -- call 0 for the flight, the event and a new direction,
    // call 1 for a dye's quantum-yield test and emitted wavelength
    if (alive && !full && exit_code < 0) {
        L.v++;
        bool step = false;
        if (REC && P.max_vertices && L.v >= P.max_vertices) {
            exit_code = FPT_EXIT_TRUNC;
        } else if (L.v >= kMaxPathVertices) {
            exit_code = FPT_EXIT_SCAP;  // hard bound: every wave's loop terminates
        } else {
            step = true;
        }
        if (step) {
            cnt.vertices++;
            const uint4 r = philox(L.pid, L.v, 0u, 0u, P.key0, P.key1);
            const float u0 = u24(r.x), u1 = u24(r.y), u2 = u24(r.z), u3 = u24(r.w);
            float dir_sin = 0.f, dir_cos = 0.f;  // polar sine/cosine of a new direction
            int frame = -1;                      // -1 world axes, else wall face
            float gloss_n = 0.f;                 // Phong exponent of a glossy wall reflection
            bool need1 = false;                  // the vertex draws call 1 of its counter too
            int dye = 0;                         // the absorbing dye
            // eq. 6: free flight with density sigma_t exp(-sigma_t t)
            const float tf = (L.inv == kInf) ? kInf : neg_log1m(u0) * L.inv;
            const Hit h = next_surface<GEOM>(P, SP, L, GEOM == FPT_GEOM_BOX && L.v == 1u);
            const bool collide = tf < h.d;
            const float len = collide ? tf : h.d;
            if (len < kInf) {
                L.x[0] += len * L.w[0];
                L.x[1] += len * L.w[1];
                L.x[2] += len * L.w[2];
                score_length<MODE>(P, T, L, A, len);
            }
            if (!collide) snap_to_plane<GEOM>(P, L, h);
            if (collide) {
                const float s = u1 * L.st;
                if (s < L.ss) {
                    // elastic scattering, isotropic phase function (eq. 2)
                    ev = EV_SCATTER;
                    if constexpr (ADJ)
                        adj_add(A.S, wi(T, P.off_med + L.medium * kMedWords + MW_PSS),
                                wf(T, P.off_med + L.medium * kMedWords + MW_INV_SS));
                    L.nsc++;
                    cnt.scatters++;
                    if (!P.exc_scatter && L.nem == 0u) exit_code = FPT_EXIT_EXCSCAT;
                    else if (L.nsc > P.max_scatter) exit_code = FPT_EXIT_SCAP;
                    else {
                        dir_cos = 1.f - 2.f * u2;
                        dir_sin = 2.f * fsqrt(u2 * (1.f - u2));
                        pend = PEND_MEDIUM;
                    }
                } else if (s < L.thr_bg || L.ndy == 0) {
                    ev = EV_BG;
                    exit_code = FPT_EXIT_BG;
                } else {
                    // a fluorescent particle: which dye slot (sec. 4.1)
                    ev = EV_DYE;
                    int j = 0;
                    const int cb = P.off_cum + L.medium * P.cum_stride * P.N + L.lam;
                    for (; j < L.ndy - 1; ++j)
                        if (s < wf(T, cb + j * P.N)) break;
                    const int mb = P.off_med + L.medium * kMedWords;
                    if constexpr (ADJ) adj_add(A.S, wi(T, mb + MW_PC + j), wf(T, mb + MW_INV_C + j));
                    lds_count(tally, FPT_T_DYE_ABS);
                    if (L.nem >= P.max_emissions) {
                        exit_code = FPT_EXIT_KCAP;
                    } else {
                        dye = wi(T, mb + MW_DYE + j);
                        need1 = true;  // quantum-yield test and emitted wavelength
                    }
                }
            } else {
                ev = h.ev;
                bool refl = false;
                if constexpr (kBody) {
                    if (ev == EV_ESC && h.d < kInf && P.ior != 1.f) {
                        // the body's dielectric boundary: specular reflection with
                        // the Fresnel probability (total internal reflection beyond
                        // the critical angle), else the path crosses out; u1 decides
                        float nb[3], ct;
                        body_normal<GEOM>(P, L.x, L.w, nb);
                        if (u1 < fresnel(dot3(L.w, nb), P.ior, 1.f, ct)) {
                            mirror(L.w, nb);
                            lds_count(tally, FPT_T_WALL_REFLECT);
                            refl = true;
                        }
                    }
                }
                if (refl) {
                    // the path stays in the body with the mirrored direction
                } else if (ev == EV_ESC || ev == EV_INF) {
                    escape();
                } else if (ev == EV_LIGHT) {
                    exit_code = FPT_EXIT_LIGHT;
                } else if (ev == EV_WALL) {
                    const float rho = h.idx >= 0 ? wf(T, P.off_rho + h.idx * P.N + L.lam) : 0.f;
                    if (!(u1 < rho)) {
                        exit_code = FPT_EXIT_WALL;
                    } else {
                        lds_count(tally, FPT_T_WALL_REFLECT);
                        if (!P.exc_scatter && L.nem == 0u) {
                            // direct excitation only: an elastic event before the emission
                            exit_code = FPT_EXIT_EXCSCAT;
                        } else {
                            // Lambertian reflection about the wall's inward normal
                            // (or the glossy lobe, below)
                            dir_sin = fsqrt(u2);
                            dir_cos = fsqrt(1.f - u2);
                            frame = h.idx;
                            W.face = h.idx;
                            pend = PEND_SURFACE;
                            if constexpr (kGloss) gloss_n = wf(T, P.off_gloss + h.idx);
                        }
                    }
                } else {
                    // index-matched interface: change medium, keep direction
                    lds_count(tally, FPT_T_CROSSINGS);
                    if constexpr (GEOM == FPT_GEOM_BOX) {
                        L.region = (ev == EV_ENTER) ? h.idx : -1;
                        L.medium = -1;
                        if (L.region >= 0) {
                            const KSphere& sp = SP[L.region];
                            L.sc[0] = sp.c[0];
                            L.sc[1] = sp.c[1];
                            L.sc[2] = sp.c[2];
                            L.sr2 = sp.r2;
                            L.medium = sp.medium;
                        }
                        load_medium(P, T, L);
                    }
                }
            }
            uint4 r1 = make_uint4(0u, 0u, 0u, 0u);
            if (need1) r1 = philox(L.pid, L.v, 1u, 0u, P.key0, P.key1);
            if (need1) {
                const int db = P.off_dye + dye * kDyeWords;
                const float uq = u24(r1.x);
                if (!(uq < wf(T, db + DW_QY))) {
                    if constexpr (ADJ) adj_add(A.S, wi(T, db + DW_PQ), -wf(T, db + DW_INV_1MQY));
                    exit_code = FPT_EXIT_NONRAD;
                } else {
                    if constexpr (ADJ) adj_add(A.S, wi(T, db + DW_PQ), wf(T, db + DW_INV_QY));
                    // eq. 10: emitted wavelength from the emission CDF,
                    // independent of the excitation wavelength (sec. 2.1)
                    const float ul = u24(r1.y);
                    const uint32_t* cdf = T + P.off_cdf + dye * P.N;
                    int lo = 0, hi = P.N - 1;
                    while (lo < hi) {
                        const int mid = (lo + hi) >> 1;
                        if (ul < __uint_as_float(cdf[mid])) hi = mid;
                        else lo = mid + 1;
                    }
                    L.lam = lo;
                    load_sigma(P, T, L);
                    L.nem++;
                    L.comp = 1;
                    lds_count(tally, FPT_T_EMISSIONS);
                    dir_cos = 1.f - 2.f * u2;
                    dir_sin = 2.f * fsqrt(u2 * (1.f - u2));
                    pend = PEND_MEDIUM;
                }
            }
            if (pend != PEND_NONE && exit_code < 0) {
                float sp, cp;
                sincos_rev(u3, &sp, &cp);
                const float a = dir_sin * cp, b = dir_sin * sp;
                if (kGloss && gloss_n > 0.f) {
                    float lobe = 0.f, fac = 0.f;
                    const bool on = glossy_reflect(gloss_n, frame, u2, sp, cp, L.x, L.w, nrm, lobe, fac);
                    W.sw = L.wgt * lobe;
                    W.gspl = true;
                    if (on) {
                        L.wgt *= fac;
                    } else {
                        exit_code = FPT_EXIT_WALL;
                        W.gdie = true;
                    }
                } else if (frame < 0) {
                    L.w[0] = a; L.w[1] = b; L.w[2] = dir_cos;
                } else {
                    // wall frame: normal n = sg e_ax, tangents e_(ax+1), sg e_(ax+2)
                    const int ax = frame >> 1;
                    const float sg = (frame & 1) ? -1.f : 1.f;
                    const float c = sg * dir_cos, bb = sg * b;
                    L.w[0] = ax == 0 ? c : (ax == 1 ? bb : a);
                    L.w[1] = ax == 0 ? a : (ax == 1 ? c : bb);
                    L.w[2] = ax == 0 ? bb : (ax == 1 ? a : c);
                    nrm[0] = ax == 0 ? sg : 0.f;
                    nrm[1] = ax == 1 ? sg : 0.f;
                    nrm[2] = ax == 2 ? sg : 0.f;
                }
                rrb = rr_bits(r);
            } else {
                pend = PEND_NONE;
            }
        }
    }
    connect(true);

    // ---- path end
    if (alive && exit_code >= 0) {
        alive = false;
        lds_count(tally, FPT_T_EXIT0 + exit_code);
        if constexpr (REC) {
            fpt_path_record rc;
            rc.n_vertices = L.v + (exit_code == FPT_EXIT_TRUNC ? 0u : 1u);
            rc.n_scatter = L.nsc;
            rc.n_emit = L.nem;
            rc.exit_code = (uint32_t)exit_code;
            rc.lambda = L.lam;
            rc.comp = L.comp;
            rc.region = L.region;
            rc.pad = 0;
            rc.pos[0] = L.x[0]; rc.pos[1] = L.x[1]; rc.pos[2] = L.x[2];
            rc.dir[0] = L.w[0]; rc.dir[1] = L.w[1]; rc.dir[2] = L.w[2];
            rc.splat_sum = L.splat_sum;
            rc.pad2 = 0.f;
            const uint32_t k = L.pid - P.path_begin;
            B.rec[k] = rc;
            if constexpr (ADJ) {
                if (B.rec_grad) {
#pragma unroll
                    for (int i = 0; i < kMaxNP; ++i)
                        if (i < P.np) B.rec_grad[(size_t)k * P.np + i] = G[i] + A.Gx[i * 64];
                }
#pragma unroll
                for (int i = 0; i < kMaxNP; ++i) {
                    G[i] = 0.f;
                    A.Gx[i * 64] = 0.f;
                }
            }
        }
    }
    // ---- evaluate queued splats: full batches, and everything once the wave is done
    if constexpr (DEFER) {
        if (pinhole)
            sq_drain(P, B.film, T, SP, tally, W.q, cnt, lane, exhausted && __ballot(alive) == 0ull);
    }
}

// -------------------------------------------------------------------------
// The persistent transport kernel.
template <int GEOM, int MODE, bool REFR>
__global__ void __launch_bounds__(256) k_transport(const KParams P, const KBuffers B) {
    constexpr bool ADJ = (MODE == MODE_ADJ || MODE == MODE_REC_ADJ);
    constexpr bool REC = (MODE == MODE_REC || MODE == MODE_REC_ADJ);
    extern __shared__ uint32_t smem[];
    uint32_t* tally = smem;                                          // FPT_N_TALLIES u32
    KSphere* SPw = reinterpret_cast<KSphere*>(smem + kLdsSpheres);  // sphere table
    const KSphere* SP = SPw;
    const uint32_t* T = smem + kLdsTable;                            // table image
    // the image up to the d sigma_a / d conc rows, which only the adjoint reads
    const int staged = ADJ ? P.off_src : P.off_kap;
    const int tw = (staged + 63) & ~63;
    // escape histogram in LDS (FWD, escape sensor, small films), flushed once per block
    uint32_t* hist = smem + kLdsTable + tw;
    const bool lds_hist = MODE == MODE_FWD && P.hist_words > 0;
    for (int i = threadIdx.x; i < FPT_N_TALLIES; i += blockDim.x) tally[i] = 0u;
    for (int i = threadIdx.x; i < staged; i += blockDim.x) smem[kLdsTable + i] = B.tables[i];
    for (int i = threadIdx.x; i < P.n_spheres; i += blockDim.x) SPw[i] = P.spheres[i];
    if (lds_hist)
        for (int i = threadIdx.x; i < P.hist_words; i += blockDim.x) hist[i] = 0u;
    const int wave = threadIdx.x >> 6;
    const uint32_t lane = lane_id();
    AdjView A;
    float G[ADJ ? kMaxNP : 1];
    if constexpr (ADJ) {
        float* base = reinterpret_cast<float*>(smem + kLdsTable + tw + P.hist_words) +
                      wave * (2 * kMaxNP * 64) + lane;
        A.S = base;
        A.Gx = base + kMaxNP * 64;
#pragma unroll
        for (int i = 0; i < kMaxNP; ++i) {
            A.S[i * 64] = 0.f;
            A.Gx[i * 64] = 0.f;
            G[i] = 0.f;
        }
    }
    __syncthreads();

    WaveCtx C;
    C.T = T;
    C.SP = SP;
    C.tally = tally;
    C.hist = hist;
    C.lds_hist = lds_hist;
    C.pinhole = (GEOM == FPT_GEOM_BOX) && P.sensor == FPT_SENSOR_PINHOLE;
    C.lane = lane;
    WalkState W;
    W.cnt = {0u, 0u, 0u, 0u};
    W.L.pid = 0;
    W.alive = false;
    W.deep = false;
    W.pend = PEND_NONE;
    W.face = 0;
    W.nrm[0] = W.nrm[1] = W.nrm[2] = 0.f;
    W.rrb = 0;
    W.sw = 1.f;
    W.gspl = false;
    W.gdie = false;
    W.L.wgt = 1.f;
    constexpr bool DEFER = (GEOM == FPT_GEOM_BOX && MODE == MODE_FWD);
    W.q.base = smem + kLdsTable + tw + P.hist_words + wave * (sq_words(P) + kAggWords);  // DEFER only
    W.q.agg = W.q.base + sq_words(P);
    if constexpr (DEFER) {
        for (int i = (int)lane; i < kAggSlots; i += 64) {
            W.q.agg[i] = kAggEmpty;
            W.q.agg[kAggSlots + i] = 0u;
        }
    }
    W.q.head = 0;
    W.q.count = 0;
    W.q.held = 0;
    const uint32_t gwave = blockIdx.x * (blockDim.x >> 6) + (uint32_t)__builtin_amdgcn_readfirstlane(wave);
    W.q.slice = (DEFER && B.sjobs) ? B.sjobs + (size_t)gwave * kEntryWords * B.sjob_slice : nullptr;
    W.q.sj_n = 0;
    bool exhausted = false;
    // the path queue is split into kQueueShards contiguous ranges with a head
    // each (a single head serialises every wave's claim at the memory-side
    // atomic unit); a wave starts on shard gwave mod kQueueShards and moves on
    // to the next shard only once its own is used up
    int shard = (int)(gwave % (uint32_t)kQueueShards);
    int moves = 0;

    for (;;) {
        // ---- refill dead lanes from the path queue (one atomic per wave)
        W.fresh = false;
        if (!exhausted) {
            const uint64_t dead = __ballot(!W.alive);
            const int ndead = __popcll(dead);
            if (ndead >= P.refill_lanes || ndead == 64) {
                for (;;) {  // at most kQueueShards iterations over the wave's life
                    const unsigned long long lo = (unsigned long long)shard * P.path_count / kQueueShards;
                    const unsigned long long hi = (unsigned long long)(shard + 1) * P.path_count / kQueueShards;
                    unsigned long long off = 0;
                    if (lane == 0) off = atomicAdd(&B.counter[shard * kShardStride], (unsigned long long)ndead);
                    off = ((unsigned long long)(uint32_t)__builtin_amdgcn_readfirstlane((int)(off >> 32)) << 32) |
                          (uint32_t)__builtin_amdgcn_readfirstlane((int)(uint32_t)off);
                    const unsigned long long base = lo + off;
                    if (base < hi) {
                        if (!W.alive) {
                            const unsigned long long idx = base + mbcnt(dead);
                            if (idx < hi) assign_path(W, P.path_begin + (uint32_t)idx);
                        }
                        if (base + (unsigned long long)ndead < hi) break;
                        // this claim used the shard up: count it
                        if (lane == 0) atomicAdd(&B.counter[kQueueShards * kShardStride], 1ull);
                    }
                    // this shard is used up: the end of the queue once every
                    // shard is, else the next shard
                    unsigned long long used = 0;
                    if (lane == 0)
                        used = __hip_atomic_load(&B.counter[kQueueShards * kShardStride], __ATOMIC_RELAXED,
                                                 __HIP_MEMORY_SCOPE_AGENT);
                    used = (unsigned long long)(uint32_t)__builtin_amdgcn_readfirstlane((int)(uint32_t)used);
                    if (++moves == kQueueShards || used >= (unsigned long long)kQueueShards) {
                        exhausted = true;
                        break;
                    }
                    shard = shard + 1 == kQueueShards ? 0 : shard + 1;
                    if (base < hi) break;  // the lanes got paths; claim from the next shard later
                }
            }
        }
        if (__ballot(W.alive) == 0ull && !exhausted) continue;
        // with every lane done and the queue exhausted this only drains the splats
        advance<GEOM, MODE, REFR>(P, B, C, W, A, G, exhausted);
        if (exhausted && __ballot(W.alive) == 0ull) break;
    }

    if constexpr (DEFER) {
        if (W.q.held > 0) agg_write_out(B.film, W.q.agg, lane);  // the deposits still merging
    }
    if (DEFER && W.q.slice && lane == 0) B.sjob_counts[gwave] = (uint32_t)W.q.sj_n;
    // ---- flush counters: per-lane -> wave -> block LDS -> global
    {
        uint32_t a = W.cnt.vertices, b = W.cnt.scatters, c = W.cnt.splat_hit, o = W.cnt.opaque;
        for (int off = 32; off > 0; off >>= 1) {
            a += __shfl_xor(a, off);
            b += __shfl_xor(b, off);
            c += __shfl_xor(c, off);
            o += __shfl_xor(o, off);
        }
        if (lane == 0) {
            atomicAdd(&tally[FPT_T_VERTICES], a);
            atomicAdd(&tally[FPT_T_SCATTERS], b);
            atomicAdd(&tally[FPT_T_SPLAT_HIT], c);
            if (o) atomicAdd(&tally[FPT_T_SPLAT_OPAQUE], o);
        }
    }
    if constexpr (ADJ && !REC) {
        // block reduction of the gradient: lanes -> wave (shuffle) -> block (LDS)
        float* red = reinterpret_cast<float*>(smem + kLdsTable + tw + P.hist_words) +
                     (blockDim.x >> 6) * (2 * kMaxNP * 64);
#pragma unroll
        for (int i = 0; i < kMaxNP; ++i) {
            float g = G[i] + A.Gx[i * 64];
            for (int off = 32; off > 0; off >>= 1) g += __shfl_xor(g, off);
            if (lane == 0) red[wave * kMaxNP + i] = g;
        }
        __syncthreads();
        if (threadIdx.x < kMaxNP) {
            float g = 0.f;
            for (int w = 0; w < (int)(blockDim.x >> 6); ++w) g += red[w * kMaxNP + threadIdx.x];
            B.partials[blockIdx.x * kMaxNP + threadIdx.x] = g;
        }
    }
    __syncthreads();
    if (lds_hist)
        for (int i = threadIdx.x; i < P.hist_words; i += blockDim.x)
            if (hist[i]) atomicAdd(&B.counts[i], hist[i]);
    if (threadIdx.x < FPT_N_TALLIES && B.tallies) {
        uint32_t v = tally[threadIdx.x];
        if (threadIdx.x == FPT_T_PATHS) {
            v = 0u;
            for (int e = 0; e < 10; ++e) v += tally[FPT_T_EXIT0 + e];
        }
        if (v) atomicAdd(&B.tallies[threadIdx.x], (unsigned long long)v);
    }
}

// -------------------------------------------------------------------------
// Batched form: many independent escape-sensor instances in one persistent
// launch.  Each wave owns an LDS slot holding its current instance's event
// tally, escape histogram and tables; it claims (instance, path range) items
// from a device queue, prefetching the next item so that ranges of the same
// instance merge without draining the lanes; a new instance is staged only once
// every lane has finished, and the slot's histogram and tally are flushed to
// that instance's global counters.  The instance's launch parameters are read
// from device memory through a constant-address-space pointer with a
// wave-uniform index, so they arrive by scalar loads in scalar registers (read
// from an LDS copy they took a VGPR each: 149 VGPRs against 118, one wave less
// per SIMD, 7 % of the batched form).

DEV void batch_flush(const KBatch& Bt, int inst, uint32_t* tally, uint32_t* hist, Counters& cnt,
                     uint32_t lane) {
    uint32_t a = cnt.vertices, b = cnt.scatters, c = cnt.splat_hit;
    for (int off = 32; off > 0; off >>= 1) {
        a += __shfl_xor(a, off);
        b += __shfl_xor(b, off);
        c += __shfl_xor(c, off);
    }
    cnt = {0u, 0u, 0u, 0u};
    if (lane == 0) {
        tally[FPT_T_VERTICES] += a;
        tally[FPT_T_SCATTERS] += b;
        tally[FPT_T_SPLAT_HIT] += c;
    }
    wave_sync();
    uint32_t* dst = Bt.counts + (size_t)inst * Bt.hist_words;
    for (int i = lane; i < Bt.hist_words; i += 64)
        if (hist[i]) atomicAdd(&dst[i], hist[i]);
    if (Bt.tallies && lane < FPT_N_TALLIES) {
        uint32_t v = tally[lane];
        if (lane == FPT_T_PATHS) {
            v = 0u;
            for (int e = 0; e < 10; ++e) v += tally[FPT_T_EXIT0 + e];
        }
        if (v) atomicAdd(&Bt.tallies[(size_t)inst * FPT_N_TALLIES + lane], (unsigned long long)v);
    }
    wave_sync();
}

template <bool REFR>
__global__ void __launch_bounds__(256) k_batch(const KBatch Bt) {
    extern __shared__ uint32_t smem[];
    const int wave = threadIdx.x >> 6;
    const uint32_t lane = lane_id();
    uint32_t* slot = smem + (size_t)wave * Bt.slot_words;
    uint32_t* tally = slot;
    uint32_t* hist = tally + 32;
    uint32_t* table = hist + ((Bt.hist_words + 3) & ~3);
    WaveCtx C;
    C.T = table;
    C.SP = nullptr;
    C.tally = tally;
    C.hist = hist;
    C.lds_hist = true;
    C.pinhole = false;
    C.lane = lane;
    WalkState W;
    W.cnt = {0u, 0u, 0u, 0u};
    W.L.pid = 0;
    W.alive = false;
    W.deep = false;
    W.pend = PEND_NONE;
    W.face = 0;
    W.nrm[0] = W.nrm[1] = W.nrm[2] = 0.f;
    W.rrb = 0;
    W.sw = 1.f;
    W.gspl = false;
    W.gdie = false;
    W.L.wgt = 1.f;
    W.q.base = nullptr;
    W.q.agg = nullptr;
    W.q.head = 0;
    W.q.count = 0;
    W.q.held = 0;
    W.q.slice = nullptr;
    W.q.sj_n = 0;
    AdjView A;
    A.S = nullptr;
    A.Gx = nullptr;
    float G[1] = {0.f};
    KBuffers Bd;
    Bd.tables = nullptr;
    Bd.film = nullptr;
    Bd.counts = nullptr;
    Bd.tallies = nullptr;
    Bd.counter = nullptr;
    Bd.gfilm = nullptr;
    Bd.partials = nullptr;
    Bd.rec = nullptr;
    Bd.rec_grad = nullptr;
    int cur = -1, pending = -1;
    bool done = false;
    uint32_t lo = 0, hi = 0;
    for (;;) {
        if (lo >= hi) {
            if (pending < 0 && !done) {
                unsigned long long it = 0;
                if (lane == 0) it = atomicAdd(Bt.item_counter, 1ull);
                it = __shfl(it, 0);
                if (it < (unsigned long long)Bt.n_items) pending = (int)it;
                else done = true;
            }
            if (pending >= 0) {
                const KWorkItem item = Bt.items[pending];
                if ((int)item.instance == cur) {
                    lo = item.path_lo;
                    hi = item.path_hi;
                    pending = -1;
                } else if (__ballot(W.alive) == 0ull) {
                    if (cur >= 0) batch_flush(Bt, cur, tally, hist, W.cnt, lane);
                    // stage the new instance: zeroed counters, tables
                    for (int i = lane; i < 32; i += 64) tally[i] = 0u;
                    for (int i = lane; i < Bt.hist_words; i += 64) hist[i] = 0u;
                    const uint32_t* tsrc = Bt.tables + Bt.table_off[item.instance];
                    const int tw = Bt.params[item.instance].off_kap;  // forward: no d sigma_a rows
                    for (int i = lane; i < tw; i += 64) table[i] = tsrc[i];
                    wave_sync();
                    cur = (int)item.instance;
                    lo = item.path_lo;
                    hi = item.path_hi;
                    pending = -1;
                }
            }
        }
        // the current instance's parameters (instance 0 stands in before the first)
        typedef const __attribute__((address_space(4))) KParams* KParamsC;
        const KParams& P = *(const KParams*)((KParamsC)Bt.params + __builtin_amdgcn_readfirstlane(max(cur, 0)));
        W.fresh = false;
        if (lo < hi) {
            const uint64_t dead = __ballot(!W.alive);
            const int ndead = __popcll(dead);
            if (ndead >= P.refill_lanes || ndead == 64) {
                const uint32_t base = lo;
                lo = min(hi, lo + (uint32_t)ndead);
                if (!W.alive) {
                    const uint32_t idx = base + mbcnt(dead);
                    if (idx < hi) assign_path(W, P.path_begin + idx);
                }
            }
        }
        if (__ballot(W.alive) == 0ull) {
            if (done && pending < 0 && lo >= hi) break;
            continue;
        }
        if (P.geometry == FPT_GEOM_SLAB) advance<FPT_GEOM_SLAB, MODE_FWD, REFR>(P, Bd, C, W, A, G, false);
        else advance<FPT_GEOM_SPHERE, MODE_FWD, REFR>(P, Bd, C, W, A, G, false);
    }
    if (cur >= 0) batch_flush(Bt, cur, tally, hist, W.cnt, lane);
}

// Connections deferred to the device buffer by the transport kernel: block b
// evaluates the slice of transport wave b.
__global__ void __launch_bounds__(256) k_splat_jobs(const KParams P, const KBuffers B) {
    extern __shared__ uint32_t smem[];
    uint32_t* tally = smem;
    KSphere* SPw = reinterpret_cast<KSphere*>(smem + kLdsSpheres);
    const uint32_t* T = smem + kLdsTable;
    const uint32_t n = B.sjob_counts[blockIdx.x];
    if (n == 0) return;  // uniform across the block
    for (int i = threadIdx.x; i < FPT_N_TALLIES; i += blockDim.x) tally[i] = 0u;
    for (int i = threadIdx.x; i < P.off_kap; i += blockDim.x) smem[kLdsTable + i] = B.tables[i];
    for (int i = threadIdx.x; i < P.n_spheres; i += blockDim.x) SPw[i] = P.spheres[i];
    __syncthreads();
    const uint32_t S = B.sjob_slice;
    const uint32_t* sl = B.sjobs + (size_t)blockIdx.x * kEntryWords * S;
    const uint32_t lane = lane_id();
    const uint32_t wv = threadIdx.x >> 6;
    uint32_t* agg = smem + kLdsTable + ((P.off_kap + 63) & ~63) + wv * kAggWords;
    for (int i = (int)lane; i < kAggSlots; i += 64) {
        agg[i] = kAggEmpty;
        agg[kAggSlots + i] = 0u;
    }
    Counters cnt = {0u, 0u, 0u, 0u};
    int held = 0;
    for (uint32_t b0 = wv * 64; b0 < n; b0 += blockDim.x) {  // uniform per wave
        const uint32_t i = b0 + lane;
        const bool valid = i < n;
        const uint32_t j = valid ? i : 0u;
        const float x[3] = {__uint_as_float(sl[j]), __uint_as_float(sl[S + j]), __uint_as_float(sl[2 * S + j])};
        const float wgt = P.glossy ? __uint_as_float(sl[5 * S + j]) : 1.f;
        const Deposit d = splat_entries(P, T, SPw, tally, cnt, valid, x, sl[3 * S + j], sl[4 * S + j], wgt);
        film_add_merged(P, B.film, agg, held, d, lane);
    }
    if (held > 0) agg_write_out(B.film, agg, lane);
    uint32_t h = cnt.splat_hit;
    for (int off = 32; off > 0; off >>= 1) h += __shfl_xor(h, off);
    if (lane_id() == 0 && h) atomicAdd(&tally[FPT_T_SPLAT_HIT], h);
    __syncthreads();
    if (threadIdx.x < FPT_N_TALLIES && B.tallies && tally[threadIdx.x])
        atomicAdd(&B.tallies[threadIdx.x], (unsigned long long)tally[threadIdx.x]);
}

size_t splat_jobs_lds_bytes(const KParams& P) {
    return (size_t)(kLdsTable + ((P.off_kap + 63) & ~63) + 4 * kAggWords) * 4;
}

hipError_t launch_splat_jobs(const KParams& P, const KBuffers& B, int grid, hipStream_t s) {
    hipLaunchKernelGGL(k_splat_jobs, dim3(grid), dim3(256), splat_jobs_lds_bytes(P), s, P, B);
    return hipGetLastError();
}

// films[i] += counts[i] * wscale[instance of i]
__global__ void k_finalize_batch(const uint32_t* counts, float* films, const float* wscale,
                                 int hist_words, size_t n) {
    for (size_t i = blockIdx.x * (size_t)blockDim.x + threadIdx.x; i < n; i += (size_t)gridDim.x * blockDim.x) {
        const uint32_t c = counts[i];
        if (c) films[i] += (float)c * wscale[i / hist_words];
    }
}

size_t batch_lds_bytes(const KBatch& Bt, int block) { return (size_t)(block / 64) * Bt.slot_words * 4; }

int batch_slot_words(int hist_words, int max_table_words) {
    return 32 + ((hist_words + 3) & ~3) + ((max_table_words + 3) & ~3);
}

hipError_t batch_occupancy(const KBatch& Bt, int block, int* n) {
    const void* f = Bt.refractive ? reinterpret_cast<const void*>(&k_batch<true>)
                                  : reinterpret_cast<const void*>(&k_batch<false>);
    return hipOccupancyMaxActiveBlocksPerMultiprocessor(n, f, block, batch_lds_bytes(Bt, block));
}

hipError_t launch_batch(const KBatch& Bt, int grid, int block, hipStream_t s) {
    if (Bt.refractive)
        hipLaunchKernelGGL((k_batch<true>), dim3(grid), dim3(block), batch_lds_bytes(Bt, block), s, Bt);
    else
        hipLaunchKernelGGL((k_batch<false>), dim3(grid), dim3(block), batch_lds_bytes(Bt, block), s, Bt);
    return hipGetLastError();
}

hipError_t launch_finalize_batch(const uint32_t* counts, float* films, const float* wscale,
                                 int hist_words, size_t n, hipStream_t s) {
    if (!n) return hipSuccess;
    const int grid = (int)std::min<size_t>((n + 255) / 256, 4096);
    hipLaunchKernelGGL(k_finalize_batch, dim3(grid), dim3(256), 0, s, counts, films, wscale, hist_words, n);
    return hipGetLastError();
}

// -------------------------------------------------------------------------
// Small helper kernels (graph-safe replacements for memset and reductions).
__global__ void k_zero_u32(uint32_t* p, size_t n) {
    for (size_t i = blockIdx.x * (size_t)blockDim.x + threadIdx.x; i < n; i += (size_t)gridDim.x * blockDim.x)
        p[i] = 0u;
}

__global__ void k_zero_u64(unsigned long long* p, size_t n) {
    for (size_t i = blockIdx.x * (size_t)blockDim.x + threadIdx.x; i < n; i += (size_t)gridDim.x * blockDim.x)
        p[i] = 0ull;
}

// film[i] += counts[i] * scale (integer escape tallies -> fractions of photons)
__global__ void k_finalize_counts(const uint32_t* counts, float* film, size_t n, float scale) {
    for (size_t i = blockIdx.x * (size_t)blockDim.x + threadIdx.x; i < n; i += (size_t)gridDim.x * blockDim.x) {
        const uint32_t c = counts[i];
        if (c) film[i] += (float)c * scale;
    }
}

// grad[i] += sum over blocks of partials[b][i] (fp64 sum)
__global__ void k_reduce_partials(const float* partials, int nblocks, int np, float* grad) {
    __shared__ double acc[256];
    for (int i = 0; i < np; ++i) {
        double s = 0.0;
        for (int b = threadIdx.x; b < nblocks; b += blockDim.x) s += (double)partials[b * kMaxNP + i];
        acc[threadIdx.x] = s;
        __syncthreads();
        for (int o = blockDim.x / 2; o > 0; o >>= 1) {
            if ((int)threadIdx.x < o) acc[threadIdx.x] += acc[threadIdx.x + o];
            __syncthreads();
        }
        if (threadIdx.x == 0) grad[i] += (float)acc[0];
        __syncthreads();
    }
}

// -------------------------------------------------------------------------
// Camera-side estimator (sec. 4.1: paths leave the camera at the emission
// wavelength and sample the light only where an emission is realised; sec.
// 4.3, eq. 12).  Path p = ((s H + py) W + px) N + k walks analogously at bin
// k from the eye through a uniform point of pixel (px, py).  At every
// collision in a dye medium the light is connected directly: a uniform point
// on the quad, the transmittance at each of its lines through every sphere,
// the emitter cosine and 1/r^2; the fluorescence source over sigma_t(k) is
// added to the path's sum, which goes to film component 1 once, when the path
// ends.  Any absorption ends the walk (a dye absorbing at the emission
// wavelength would be a second emission: K = 1), as do the light quad and the
// open face.  One lane per path.  A wave claims chunks of kCamChunk
// consecutive paths (one pixel's bins, neighbouring pixels) from a global
// counter and hands them to its finished lanes once refill_lanes of them are
// free.  The whole table image, camera rows included, sits in LDS.

// New direction from its polar cosine/sine about +z (frame < 0) or about the
// inward normal of wall `frame`, azimuth 2 pi u3.
DEV void turn(float* w, float c, float sn, int frame, float u3) {
    float sp, cp;
    sincos_rev(u3, &sp, &cp);
    const float a = sn * cp, b = sn * sp;
    if (frame < 0) {
        w[0] = a; w[1] = b; w[2] = c;
        return;
    }
    // wall frame: normal n = sg e_ax, tangents e_(ax+1), sg e_(ax+2)
    const int ax = frame >> 1;
    const float sg = (frame & 1) ? -1.f : 1.f;
    const float cc = sg * c, bb = sg * b;
    w[0] = ax == 0 ? cc : (ax == 1 ? bb : a);
    w[1] = ax == 0 ? a : (ax == 1 ? cc : bb);
    w[2] = ax == 0 ? bb : (ax == 1 ? a : cc);
}

// Fluorescence source at the lane's collision from the light point (ua, ub):
// sum_l src[m][k][l] T_l cos_n / r^2, or 0 with hit = false when the point's
// emitting side faces away.
DEV float cam_source(const uint32_t* S, const KSphere* SP, const Lane& L, float ua, float ub,
                     bool& hit) {
    const auto& P = *kernel_params();
    const float d0 = P.lpos[0] + ua * P.lu[0] + ub * P.lv[0] - L.x[0];
    const float d1 = P.lpos[1] + ua * P.lu[1] + ub * P.lv[1] - L.x[1];
    const float d2 = P.lpos[2] + ua * P.lu[2] + ub * P.lv[2] - L.x[2];
    const float r2 = d0 * d0 + d1 * d1 + d2 * d2;
    const float rinv = __builtin_amdgcn_rsqf(r2);
    const float cos_n = -(P.ln[0] * d0 + P.ln[1] * d1 + P.ln[2] * d2) * rinv;
    hit = cos_n > 0.f;
    if (!hit) return 0.f;
    const float wc[3] = {d0 * rinv, d1 * rinv, d2 * rinv};
    const float r = r2 * rinv;
    float len[FPT_MAX_SPHERES];
#pragma unroll
    for (int s = 0; s < FPT_MAX_SPHERES; ++s)
        len[s] = s < P.n_spheres ? chord_len(SP[s], L.x, wc, r) : 0.f;
    const int row = P.off_src + (L.medium * P.N + L.lam) * P.n_lines;
    float sum = 0.f;
#pragma unroll
    for (int l = 0; l < FPT_MAX_LINES; ++l) {
        if (l >= P.n_lines) break;
        float tau = 0.f;
#pragma unroll
        for (int s = 0; s < FPT_MAX_SPHERES; ++s)
            if (s < P.n_spheres) tau += wf(S, P.off_csig + s * P.n_lines + l) * len[s];
        sum += wf(S, row + l) * (tau < kTauZero ? __expf(-tau) : 0.f);
    }
    return sum * cos_n * (rinv * rinv);
}

struct CamLane {
    Lane L;
    float acc;       // the path's deposit so far
    long long fidx;  // its film element
};

// Vertex 0: the eye ray through a uniform point of the pixel enters the box
// through the open face (the last of the three slab entries), else the path
// ends at once (exit ESC_T).  Returns the exit code or -1.
DEV int cam_start(const KParams& P, const uint32_t* S, CamLane& C, uint32_t pid) {
    const auto& K = *kernel_params();  // camera and box fields
    Lane& L = C.L;
    const uint32_t npix = (uint32_t)K.W * (uint32_t)K.H;
    const uint32_t k = pid % (uint32_t)P.N, rest = pid / (uint32_t)P.N;
    const uint32_t pix = rest % npix, smp = rest / npix;
    const uint32_t px = pix % (uint32_t)K.W, py = pix / (uint32_t)K.W;
    L.pid = pid;
    L.v = 0u;
    L.nsc = 0u;
    L.nem = 0u;
    L.lam = (int)k;
    L.comp = 1;
    L.batch = smp % P.batches;
    L.region = -1;
    L.medium = -1;
    L.splat_sum = 0.f;
    load_medium(P, S, L);
    C.acc = 0.f;
    C.fidx = (((long long)L.batch * 2 + 1) * npix + pix) * P.N + k;
    const uint4 r = philox(pid, 0u, 0u, 0u, P.key0, P.key1);
    const float xi = fdiv(2.f * ((float)px + u24(r.x)), (float)K.W) - 1.f;
    const float yi = 1.f - fdiv(2.f * ((float)py + u24(r.y)), (float)K.H);
    float w[3];
#pragma unroll
    for (int a = 0; a < 3; ++a) w[a] = K.cf[a] + xi * K.tanx * K.cr[a] + yi * K.tany * K.cu[a];
    const float wn = __builtin_amdgcn_rsqf(w[0] * w[0] + w[1] * w[1] + w[2] * w[2]);
    float t_in = -kInf, t_out = kInf;
    int face = -1;
    bool inside = true;
#pragma unroll
    for (int a = 0; a < 3; ++a) {
        w[a] *= wn;
        L.w[a] = w[a];
        if (w[a] == 0.f) {
            if (K.eye[a] < K.lo[a] || K.eye[a] > K.hi[a]) inside = false;
            continue;
        }
        const float t0 = fdiv(K.lo[a] - K.eye[a], w[a]), t1 = fdiv(K.hi[a] - K.eye[a], w[a]);
        const float tn = w[a] > 0.f ? t0 : t1, tf = w[a] > 0.f ? t1 : t0;
        if (tn > t_in) {
            t_in = tn;
            face = w[a] > 0.f ? 2 * a : 2 * a + 1;
        }
        t_out = fminf(t_out, tf);
    }
    if (!(inside && face == K.open_face && t_in > 0.f && t_in < t_out)) return FPT_EXIT_ESC_T;
    const int oa = K.open_face >> 1;
#pragma unroll
    for (int a = 0; a < 3; ++a) L.x[a] = a == oa ? K.vis_plane : K.eye[a] + t_in * w[a];
    return -1;
}

// One vertex of a live camera path.  Returns the exit code or -1.
DEV int cam_step(const KParams& P, const uint32_t* S, const KSphere* SP, uint32_t* tally,
                 Counters& cnt, CamLane& C) {
    Lane& L = C.L;
    L.v += 1u;
    if (P.max_vertices && L.v >= P.max_vertices) return FPT_EXIT_TRUNC;
    if (L.v >= kMaxPathVertices) return FPT_EXIT_SCAP;
    cnt.vertices++;
    const uint4 r = philox(L.pid, L.v, 0u, 0u, P.key0, P.key1);
    const float u0 = u24(r.x), u1 = u24(r.y), u2 = u24(r.z), u3 = u24(r.w);
    // eq. 6: free flight at the emission wavelength
    const float tf = (L.inv == kInf) ? kInf : neg_log1m(u0) * L.inv;
    const Hit h = next_surface<FPT_GEOM_BOX>(P, SP, L, false);
    const bool collide = tf < h.d;
    const float len = collide ? tf : h.d;
    if (len < kInf) {
        L.x[0] += len * L.w[0];
        L.x[1] += len * L.w[1];
        L.x[2] += len * L.w[2];
    }
    if (collide) {
        if (L.ndy > 0) {
            // a candidate emission vertex: connect to the light
            const uint4 r1 = philox(L.pid, L.v, 1u, 0u, P.key0, P.key1);
            bool hit;
            const float q = cam_source(S, SP, L, u24(r1.x), u24(r1.y), hit);
            if (hit) {
                cnt.splat_hit++;
                C.acc += P.wscale * q * L.inv;
            } else {
                lds_count(tally, FPT_T_SPLAT_MISS);
            }
        }
        const float sv = u1 * L.st;
        if (sv < L.ss) {
            // elastic scattering, isotropic phase function (eq. 2)
            L.nsc++;
            cnt.scatters++;
            if (L.nsc > P.max_scatter) return FPT_EXIT_SCAP;
            turn(L.w, 1.f - 2.f * u2, 2.f * fsqrt(u2 * (1.f - u2)), -1, u3);
            return -1;
        }
        if (sv < L.thr_bg || L.ndy == 0) return FPT_EXIT_BG;
        lds_count(tally, FPT_T_DYE_ABS);
        return FPT_EXIT_KCAP;
    }
    snap_to_plane<FPT_GEOM_BOX>(P, L, h);
    if (h.ev == EV_ESC || h.ev == EV_INF) return FPT_EXIT_ESC_R;
    if (h.ev == EV_LIGHT) return FPT_EXIT_LIGHT;
    if (h.ev == EV_WALL) {
        const float rho = h.idx >= 0 ? wf(S, P.off_rho + h.idx * P.N + L.lam) : 0.f;
        if (!(u1 < rho)) return FPT_EXIT_WALL;
        lds_count(tally, FPT_T_WALL_REFLECT);
        turn(L.w, fsqrt(1.f - u2), fsqrt(u2), h.idx, u3);
        return -1;
    }
    // index-matched interface: change medium, keep direction
    lds_count(tally, FPT_T_CROSSINGS);
    L.region = (h.ev == EV_ENTER) ? h.idx : -1;
    L.medium = -1;
    if (L.region >= 0) {
        const KSphere& sp = SP[L.region];
        L.sc[0] = sp.c[0];
        L.sc[1] = sp.c[1];
        L.sc[2] = sp.c[2];
        L.sr2 = sp.r2;
        L.medium = sp.medium;
    }
    load_medium(P, S, L);
    return -1;
}

template <bool REC>
DEV void cam_finish(const KParams& P, const KBuffers& B, uint32_t* tally, const CamLane& C,
                    int exit_code) {
    lds_count(tally, FPT_T_EXIT0 + exit_code);
    if (C.acc != 0.f && B.film) atomicAdd(&B.film[C.fidx], C.acc);
    if constexpr (REC) {
        const Lane& L = C.L;
        fpt_path_record rc;
        rc.n_vertices = L.v + (exit_code == FPT_EXIT_TRUNC ? 0u : 1u);
        rc.n_scatter = L.nsc;
        rc.n_emit = 0u;
        rc.exit_code = (uint32_t)exit_code;
        rc.lambda = L.lam;
        rc.comp = 1;
        rc.region = L.region;
        rc.pad = 0;
        rc.pos[0] = L.x[0]; rc.pos[1] = L.x[1]; rc.pos[2] = L.x[2];
        rc.dir[0] = L.w[0]; rc.dir[1] = L.w[1]; rc.dir[2] = L.w[2];
        rc.splat_sum = C.acc;
        rc.pad2 = 0.f;
        B.rec[L.pid - P.path_begin] = rc;
    }
}

// Paths per claim: 128 consecutive paths (a pixel's bins and part of the next).
// Measured on the 128x128x101x8 job: 512 took 3.88 ms, 256 2.83, 192 2.55,
// 160 2.50, 128 2.46, 96 2.59, 64 3.27 (more claims on the one counter); the
// last chunks of larger claims left a few waves with hundreds of paths to walk
// while the rest of the chip had run out.
constexpr uint32_t kCamChunk = 128;
constexpr uint32_t kCamBlockMinV = 24;  // paths in a sphere from this vertex on walk in wave rounds
constexpr int kCamRounds = 8;           // wave rounds per iteration

// One wave round of camera path j inside its sphere: lane k draws vertex
// v+1+k (the forward's whole-wave round: free flight, scatter test, new
// direction, positions from the canonical 16-vertex chunk scan), the vertices
// before the first stop (sphere boundary reached, absorption, a cap) are
// committed as scatters and each makes its light connection in its own lane;
// the deposits are summed over the wave.  The stop vertex itself is left to
// the path's next sequential step.  Returns the number committed.
DEV int cam_round(const KParams& P, const uint32_t* S, const KSphere* SP, uint32_t* tally,
                  Counters& cnt, CamLane& C, int j, uint32_t lane) {
    Lane Q;
#pragma unroll
    for (int c = 0; c < 3; ++c) {
        Q.x[c] = rl(C.L.x[c], j);
        Q.w[c] = rl(C.L.w[c], j);
        Q.sc[c] = rl(C.L.sc[c], j);
    }
    Q.sr2 = rl(C.L.sr2, j);
    Q.st = rl(C.L.st, j);
    Q.inv = rl(C.L.inv, j);
    Q.ss = rl(C.L.ss, j);
    Q.ndy = rli(C.L.ndy, j);
    Q.lam = rli(C.L.lam, j);
    Q.medium = rli(C.L.medium, j);
    Q.region = rli(C.L.region, j);
    Q.pid = rlu(C.L.pid, j);
    Q.v = rlu(C.L.v, j);
    Q.nsc = rlu(C.L.nsc, j);
    float wn[3], xk[4], pk[3], win[3];
    bool stop;
    deep_half<FPT_GEOM_BOX>(P, Q, Q.v, lane, Q.w, Q.x, wn, xk, pk, win, stop);
    const uint32_t vk = Q.v + 1u + lane;
    if (P.max_vertices && vk >= P.max_vertices) stop = true;
    const uint64_t sm = __ballot(stop);
    const int kstar = sm ? __ffsll((unsigned long long)sm) - 1 : 64;
    float dep = 0.f;
    if ((int)lane < kstar) {
        cnt.vertices++;
        cnt.scatters++;
        if (Q.ndy > 0) {
            const uint4 r1 = philox(Q.pid, vk, 1u, 0u, P.key0, P.key1);
            Lane Lk = Q;
            Lk.x[0] = xk[0];
            Lk.x[1] = xk[1];
            Lk.x[2] = xk[2];
            bool hit;
            const float q = cam_source(S, SP, Lk, u24(r1.x), u24(r1.y), hit);
            if (hit) {
                cnt.splat_hit++;
                dep = P.wscale * q * Q.inv;
            } else {
                lds_count(tally, FPT_T_SPLAT_MISS);
            }
        }
    }
    for (int off = 32; off > 0; off >>= 1) dep += __shfl_xor(dep, off);
    if (kstar > 0) {
        const int u = kstar - 1;
        const float nx0 = rl(xk[0], u), nx1 = rl(xk[1], u), nx2 = rl(xk[2], u);
        const float nw0 = rl(wn[0], u), nw1 = rl(wn[1], u), nw2 = rl(wn[2], u);
        if ((int)lane == j) {
            C.L.x[0] = nx0; C.L.x[1] = nx1; C.L.x[2] = nx2;
            C.L.w[0] = nw0; C.L.w[1] = nw1; C.L.w[2] = nw2;
            C.L.v += (uint32_t)kstar;
            C.L.nsc += (uint32_t)kstar;
            C.acc += dep;
        }
    }
    return kstar;
}

template <bool REC>
__global__ void __launch_bounds__(256) k_camera(const KParams P, const KBuffers B) {
    extern __shared__ uint32_t smem[];
    uint32_t* tally = smem;
    KSphere* SPw = reinterpret_cast<KSphere*>(smem + kLdsSpheres);
    const KSphere* SP = SPw;
    const uint32_t* T = smem + kLdsTable;
    for (int i = threadIdx.x; i < FPT_N_TALLIES; i += blockDim.x) tally[i] = 0u;
    for (int i = threadIdx.x; i < P.table_words; i += blockDim.x) smem[kLdsTable + i] = B.tables[i];
    for (int i = threadIdx.x; i < P.n_spheres; i += blockDim.x) SPw[i] = P.spheres[i];
    __syncthreads();
    const uint32_t lane = lane_id();
    CamLane C;
    C.acc = 0.f;
    C.fidx = 0;
    C.L.pid = 0u;
    C.L.v = 0u;
    Counters cnt = {0u, 0u, 0u, 0u};
    bool alive = false, exhausted = false;
    bool seq_next = false;  // the lane's last wave round stopped short of 64 vertices
    uint32_t q_next = 0u, q_end = 0u;  // the wave's current chunk of path indices (uniform)
    for (;;) {
        const uint64_t idle = __ballot(!alive);
        if (exhausted && idle == ~0ull) break;
        if (!exhausted && __popcll(idle) >= (uint32_t)P.refill_lanes) {
            const uint32_t need = (uint32_t)__popcll(idle);
            const uint32_t rank = mbcnt(idle);  // among the idle lanes
            uint32_t mine = ~0u;
            uint32_t took = min(need, q_end - q_next);
            if (rank < took) mine = q_next + rank;
            q_next += took;
            if (took < need) {
                // the chunk ran dry: claim the next one for the remaining lanes
                unsigned long long base = 0ull;
                if (lane == 0u) base = atomicAdd(B.counter, (unsigned long long)kCamChunk);
                const uint32_t hi = __builtin_amdgcn_readfirstlane((uint32_t)(base >> 32));
                const uint32_t lo = __builtin_amdgcn_readfirstlane((uint32_t)base);
                if (hi != 0u || lo >= P.path_count) {
                    exhausted = true;
                } else {
                    q_next = lo;
                    q_end = min(P.path_count, lo + min(kCamChunk, P.path_count - lo));
                    const uint32_t more = min(need - took, q_end - q_next);
                    if (rank >= took && rank - took < more) mine = q_next + (rank - took);
                    q_next += more;
                }
            }
            if (!alive && mine != ~0u) {
                cnt.vertices++;
                const int e = cam_start(P, T, C, P.path_begin + mine);
                if (e >= 0) cam_finish<REC>(P, B, tally, C, e);
                else alive = true;
            }
        }
        // paths deep in a sphere walk in wave rounds, up to kCamRounds per
        // iteration; one whose round stopped short resolves the stop vertex
        // with a sequential step, one still waiting for a round skips its step
        uint64_t wait = __ballot(alive && !seq_next && C.L.region >= 0 && C.L.v >= kCamBlockMinV);
        for (int rd = 0; rd < kCamRounds && wait; ++rd) {
            const int j = __ffsll((unsigned long long)wait) - 1;
            if (cam_round(P, T, SP, tally, cnt, C, j, lane) < 64) {
                wait &= ~(1ull << j);
                if ((int)lane == j) seq_next = true;
            }
        }
        if (alive && !((wait >> lane) & 1ull)) {
            seq_next = false;
            const int e = cam_step(P, T, SP, tally, cnt, C);
            if (e >= 0) {
                cam_finish<REC>(P, B, tally, C, e);
                alive = false;
            }
        }
    }
    {
        uint32_t a = cnt.vertices, b = cnt.scatters, c = cnt.splat_hit;
        for (int off = 32; off > 0; off >>= 1) {
            a += __shfl_xor(a, off);
            b += __shfl_xor(b, off);
            c += __shfl_xor(c, off);
        }
        if (lane == 0u) {
            atomicAdd(&tally[FPT_T_VERTICES], a);
            atomicAdd(&tally[FPT_T_SCATTERS], b);
            atomicAdd(&tally[FPT_T_SPLAT_HIT], c);
        }
    }
    __syncthreads();
    if (threadIdx.x < FPT_N_TALLIES && B.tallies) {
        uint32_t v = tally[threadIdx.x];
        if (threadIdx.x == FPT_T_PATHS) {
            v = 0u;
            for (int e = 0; e < 10; ++e) v += tally[FPT_T_EXIT0 + e];
        }
        if (v) atomicAdd(&B.tallies[threadIdx.x], (unsigned long long)v);
    }
}

// -------------------------------------------------------------------------
// Host-side launchers (called by the C-ABI implementation).
size_t queue_words() { return (size_t)(kQueueShards + 1) * kShardStride; }  // heads, used-up count

size_t transport_lds_bytes(const KParams& P, int block_threads, int mode) {
    const int staged = (mode == MODE_ADJ || mode == MODE_REC_ADJ) ? P.off_src : P.off_kap;
    size_t words = kLdsTable + ((staged + 63) & ~63) + P.hist_words;
    if (mode == MODE_FWD && P.geometry == FPT_GEOM_BOX)  // deferred splat rings and merging tables
        words += (size_t)(block_threads / 64) * (sq_words(P) + kAggWords);
    if (mode == MODE_ADJ || mode == MODE_REC_ADJ)
        words += (size_t)(block_threads / 64) * 2 * kMaxNP * 64 + (size_t)(block_threads / 64) * kMaxNP;
    return words * 4;
}

template <int GEOM, int MODE>
static hipError_t launch_t(const KParams& P, const KBuffers& B, int grid, int block, size_t lds,
                           hipStream_t s) {
    if (P.ior != 1.f)
        hipLaunchKernelGGL((k_transport<GEOM, MODE, true>), dim3(grid), dim3(block), lds, s, P, B);
    else
        hipLaunchKernelGGL((k_transport<GEOM, MODE, false>), dim3(grid), dim3(block), lds, s, P, B);
    return hipGetLastError();
}

template <int MODE>
static hipError_t launch_m(const KParams& P, const KBuffers& B, int grid, int block, size_t lds,
                           hipStream_t s) {
    switch (P.geometry) {
    case FPT_GEOM_SLAB: return launch_t<FPT_GEOM_SLAB, MODE>(P, B, grid, block, lds, s);
    case FPT_GEOM_HALFSPACE: return launch_t<FPT_GEOM_HALFSPACE, MODE>(P, B, grid, block, lds, s);
    case FPT_GEOM_SPHERE: return launch_t<FPT_GEOM_SPHERE, MODE>(P, B, grid, block, lds, s);
    case FPT_GEOM_INFINITE:
        hipLaunchKernelGGL((k_transport<FPT_GEOM_INFINITE, MODE, false>), dim3(grid), dim3(block), lds, s, P, B);
        return hipGetLastError();
    default:  // the box: the second instantiation carries glossy walls
        if (P.glossy)
            hipLaunchKernelGGL((k_transport<FPT_GEOM_BOX, MODE, true>), dim3(grid), dim3(block), lds, s, P, B);
        else
            hipLaunchKernelGGL((k_transport<FPT_GEOM_BOX, MODE, false>), dim3(grid), dim3(block), lds, s, P, B);
        return hipGetLastError();
    }
}

template <int GEOM, int MODE, bool REFR>
static hipError_t occ_t(const KParams& P, int block, int* n) {
    return hipOccupancyMaxActiveBlocksPerMultiprocessor(n, reinterpret_cast<const void*>(&k_transport<GEOM, MODE, REFR>),
                                                        block, transport_lds_bytes(P, block, MODE));
}

template <int MODE>
static hipError_t occ_m(const KParams& P, int block, int* n) {
    const bool r = P.ior != 1.f;
    switch (P.geometry) {
    case FPT_GEOM_SLAB: return r ? occ_t<FPT_GEOM_SLAB, MODE, true>(P, block, n) : occ_t<FPT_GEOM_SLAB, MODE, false>(P, block, n);
    case FPT_GEOM_HALFSPACE:
        return r ? occ_t<FPT_GEOM_HALFSPACE, MODE, true>(P, block, n) : occ_t<FPT_GEOM_HALFSPACE, MODE, false>(P, block, n);
    case FPT_GEOM_SPHERE: return r ? occ_t<FPT_GEOM_SPHERE, MODE, true>(P, block, n) : occ_t<FPT_GEOM_SPHERE, MODE, false>(P, block, n);
    case FPT_GEOM_INFINITE: return occ_t<FPT_GEOM_INFINITE, MODE, false>(P, block, n);
    default: return P.glossy ? occ_t<FPT_GEOM_BOX, MODE, true>(P, block, n) : occ_t<FPT_GEOM_BOX, MODE, false>(P, block, n);
    }
}

hipError_t transport_occupancy(const KParams& P, int mode, int block, int* blocks_per_cu) {
    switch (mode) {
    case MODE_FWD: return occ_m<MODE_FWD>(P, block, blocks_per_cu);
    case MODE_ADJ: return occ_m<MODE_ADJ>(P, block, blocks_per_cu);
    case MODE_REC: return occ_m<MODE_REC>(P, block, blocks_per_cu);
    default: return occ_m<MODE_REC_ADJ>(P, block, blocks_per_cu);
    }
}

hipError_t launch_transport(const KParams& P, const KBuffers& B, int mode, int grid, int block,
                            hipStream_t s) {
    const size_t lds = transport_lds_bytes(P, block, mode);
    switch (mode) {
    case MODE_FWD: return launch_m<MODE_FWD>(P, B, grid, block, lds, s);
    case MODE_ADJ: return launch_m<MODE_ADJ>(P, B, grid, block, lds, s);
    case MODE_REC: return launch_m<MODE_REC>(P, B, grid, block, lds, s);
    default: return launch_m<MODE_REC_ADJ>(P, B, grid, block, lds, s);
    }
}

size_t camera_lds_bytes(const KParams& P) { return (size_t)(kLdsTable + P.table_words) * 4; }

hipError_t camera_occupancy(const KParams& P, bool rec, int block, int* blocks_per_cu) {
    const void* f = rec ? reinterpret_cast<const void*>(&k_camera<true>)
                        : reinterpret_cast<const void*>(&k_camera<false>);
    return hipOccupancyMaxActiveBlocksPerMultiprocessor(blocks_per_cu, f, block, camera_lds_bytes(P));
}

hipError_t launch_camera(const KParams& P, const KBuffers& B, bool rec, int grid, int block,
                         hipStream_t s) {
    const size_t lds = camera_lds_bytes(P);
    if (rec) hipLaunchKernelGGL((k_camera<true>), dim3(grid), dim3(block), lds, s, P, B);
    else hipLaunchKernelGGL((k_camera<false>), dim3(grid), dim3(block), lds, s, P, B);
    return hipGetLastError();
}

hipError_t launch_zero_u32(uint32_t* p, size_t n, hipStream_t s) {
    if (!n) return hipSuccess;
    const int grid = (int)std::min<size_t>((n + 255) / 256, 4096);
    hipLaunchKernelGGL(k_zero_u32, dim3(grid), dim3(256), 0, s, p, n);
    return hipGetLastError();
}

hipError_t launch_zero_u64(unsigned long long* p, size_t n, hipStream_t s) {
    if (!n) return hipSuccess;
    const int grid = (int)std::min<size_t>((n + 255) / 256, 4096);
    hipLaunchKernelGGL(k_zero_u64, dim3(grid), dim3(256), 0, s, p, n);
    return hipGetLastError();
}

hipError_t launch_finalize_counts(const uint32_t* counts, float* film, size_t n, float scale,
                                  hipStream_t s) {
    if (!n) return hipSuccess;
    const int grid = (int)std::min<size_t>((n + 255) / 256, 4096);
    hipLaunchKernelGGL(k_finalize_counts, dim3(grid), dim3(256), 0, s, counts, film, n, scale);
    return hipGetLastError();
}

hipError_t launch_reduce_partials(const float* partials, int nblocks, int np, float* grad,
                                  hipStream_t s) {
    hipLaunchKernelGGL(k_reduce_partials, dim3(1), dim3(256), 0, s, partials, nblocks, np, grad);
    return hipGetLastError();
}

// -------------------------------------------------------------------------
// Device scratch of the allocation-free forward render (fpt_render_noalloc):
// path-queue heads, escape counters and deferred-connection slices live in
// this file-scope array instead of buffers the scene allocates.  Every device
// the library runs on holds its own copy until the process ends; its name is
// a host-side stand-in, so host code only ever uses the address
// hipGetSymbolAddress returns on each device (looked up once per device, with
// that device current, and kept).
constexpr size_t kStaticScratchBytes = (size_t)24 << 20;
static __device__ __align__(256) uint32_t scratch[kStaticScratchBytes / 4];

hipError_t static_scratch(void** ptr, size_t* bytes) {
    constexpr int kMaxDevices = 64;
    static std::mutex mu;
    static void* addr[kMaxDevices] = {};
    int dev = 0;
    hipError_t e = hipGetDevice(&dev);
    if (e != hipSuccess) return e;
    if (dev < 0 || dev >= kMaxDevices) return hipErrorInvalidDevice;
    std::lock_guard<std::mutex> lock(mu);
    if (!addr[dev]) {
        void* p = nullptr;
        e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
        if (e != hipSuccess) return e;
        addr[dev] = p;
    }
    *ptr = addr[dev];
    *bytes = kStaticScratchBytes;
    return hipSuccess;
}

}  // namespace fpt
