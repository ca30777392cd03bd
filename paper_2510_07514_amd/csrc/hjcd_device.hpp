// Device-side math of the batched HJCD-IK solve for gfx950 (CDNA4).
//
// One seed per lane.  The joint vector, the joint frames and the 6 x 6 LM
// system live in VGPRs; robot and obstacle tables are read with wave-uniform
// indices so they come through the scalar data cache (s_load); nothing of a
// seed's state touches memory between its first read and its last write.
// Arrays are sized by the compile-time bucket NM >= n (n is wave-uniform and
// every per-joint loop is unrolled to NM with a uniform `j < n` guard).
//
// Citations refer to arXiv 2510.07514.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

#include "hjcd_launch.hpp"
#include "hjcd_tables.hpp"

namespace hjcd {

// ----------------------------------------------------------------------------
// small vector / quaternion helpers
// ----------------------------------------------------------------------------
struct V3 {
    float x, y, z;
};
// Robot tables are read-only in every kernel.  PJ-IK reads them through the
// constant address space: loads at uniform addresses (every joint constant)
// then go to the scalar unit, into SGPRs, instead of through the vector memory
// path into one VGPR per lane.  That matters where a kernel runs one wave per
// SIMD (20 joints: nothing else hides the vector-load latency of each FK
// step); PO-CCD keeps the generic pointer (measured faster there).
using RobotRef = const __attribute__((address_space(4))) DevRobot*;
__device__ __forceinline__ RobotRef robot_ref(const DevRobot* p) { return (RobotRef)p; }

__device__ __forceinline__ V3 mk(float x, float y, float z) { return V3{x, y, z}; }
__device__ __forceinline__ V3 operator+(V3 a, V3 b) { return mk(a.x + b.x, a.y + b.y, a.z + b.z); }
__device__ __forceinline__ V3 operator-(V3 a, V3 b) { return mk(a.x - b.x, a.y - b.y, a.z - b.z); }
__device__ __forceinline__ V3 operator*(float s, V3 a) { return mk(s * a.x, s * a.y, s * a.z); }
__device__ __forceinline__ float dot(V3 a, V3 b) { return a.x * b.x + a.y * b.y + a.z * b.z; }
__device__ __forceinline__ V3 cross(V3 a, V3 b) {
    return mk(a.y * b.z - a.z * b.y, a.z * b.x - a.x * b.z, a.x * b.y - a.y * b.x);
}
// a + s b
__device__ __forceinline__ V3 axpy(float s, V3 b, V3 a) {
    return mk(fmaf(s, b.x, a.x), fmaf(s, b.y, a.y), fmaf(s, b.z, a.z));
}

struct Quat {
    float w, x, y, z;
};

// Hamilton product (a0, a)(b0, b) = (a0 b0 - a.b, a0 b + b0 a + a x b)
__device__ __forceinline__ Quat qmul(Quat a, Quat b) {
    Quat r;
    r.w = a.w * b.w - a.x * b.x - a.y * b.y - a.z * b.z;
    r.x = a.w * b.x + b.w * a.x + a.y * b.z - a.z * b.y;
    r.y = a.w * b.y + b.w * a.y + a.z * b.x - a.x * b.z;
    r.z = a.w * b.z + b.w * a.z + a.x * b.y - a.y * b.x;
    return r;
}

// Rigid frame: rotation columns X, Y, Z and origin p.
struct Frame {
    V3 X, Y, Z, p;
};

__device__ __forceinline__ Frame identity_frame() {
    return Frame{mk(1, 0, 0), mk(0, 1, 0), mk(0, 0, 1), mk(0, 0, 0)};
}

__device__ __forceinline__ float clampf(float x, float lo, float hi) { return fminf(fmaxf(x, lo), hi); }

// sin and cos of x for |x| <= 4096 (every angle here: joint values are
// clipped to limits the library bounds by 1000 rad, steps are below pi).
// Cody and Waite's reduction (Software Manual for the Elementary Functions,
// 1980): k = rint(2x/pi), r = x - k pi/2 with pi/2 split into three floats
// (each product exact inside an FMA), then the Taylor series of sin to r^9
// and of cos to r^10 on |r| <= pi/4 and the quadrant k mod 4.  Error about
// 1.5 ulp, 7e-8 absolute.
__device__ __forceinline__ void sincos_cw(float x, float* sn, float* cs) {
    const float k = rintf(x * 0.63661975f);
    float r = fmaf(-k, 1.57079637f, x);
    r = fmaf(-k, -4.37113883e-08f, r);
    r = fmaf(-k, -1.71512451e-15f, r);
    const float r2 = r * r;
    float ps = fmaf(2.75573192e-06f, r2, -1.98412698e-04f);
    ps = fmaf(ps, r2, 8.33333333e-03f);
    ps = fmaf(ps, r2, -1.66666667e-01f);
    const float sr = fmaf(r * r2, ps, r);
    float pc = fmaf(-2.75573192e-07f, r2, 2.48015873e-05f);
    pc = fmaf(pc, r2, -1.38888889e-03f);
    pc = fmaf(pc, r2, 4.16666667e-02f);
    pc = fmaf(pc, r2, -0.5f);
    const float cr = fmaf(r2, pc, 1.f);
    const int q = (int)k;
    const bool swap = (q & 1) != 0;
    const float a = swap ? cr : sr, b = swap ? sr : cr;
    *sn = (q & 2) ? -a : a;
    *cs = ((q + 1) & 2) ? -b : b;
}

// ----------------------------------------------------------------------------
// Forward kinematics (eq. fk): joint origins P_i and axes Z_i (STORE), and the
// end-effector frame.  Column updates of R * Rx(alpha) * Rz(theta):
//   modified DH: p += R (a, -d sin alpha, d cos alpha); R <- R Rx(alpha) Rz(theta);
//                joint i = frame i
//   standard DH: joint i = frame i-1; p += a (R Rz(theta)).X + d R.Z;
//                R <- R Rz(theta) Rx(alpha)
// ----------------------------------------------------------------------------
template <int NM, bool STORE, typename RB>
__device__ __forceinline__ void fk_chain(RB rb, int n, const float* th,
                                         V3* P, V3* Z, Frame& ee) {
    Frame T = identity_frame();
    if (rb->conv == 0) {
#pragma unroll
        for (int i = 0; i < NM; ++i) {
            if (i < n) {
                float s, c;
                sincos_cw(th[i] + rb->off[i], &s, &c);
                const float ca = rb->ca[i], sa = rb->sa[i];
                T.p = axpy(rb->pz[i], T.Z, axpy(rb->py[i], T.Y, axpy(rb->px[i], T.X, T.p)));
                V3 Yb = axpy(sa, T.Z, ca * T.Y);
                V3 Zb = axpy(-sa, T.Y, ca * T.Z);
                V3 Xn = axpy(s, Yb, c * T.X);
                V3 Yn = axpy(-s, T.X, c * Yb);
                T.X = Xn;
                T.Y = Yn;
                T.Z = Zb;
                if (STORE) {
                    P[i] = T.p;
                    Z[i] = T.Z;
                }
            }
        }
    } else {
#pragma unroll
        for (int i = 0; i < NM; ++i) {
            if (i < n) {
                if (STORE) {
                    P[i] = T.p;
                    Z[i] = T.Z;
                }
                float s, c;
                sincos_cw(th[i] + rb->off[i], &s, &c);
                const float ca = rb->ca[i], sa = rb->sa[i];
                V3 Xb = axpy(s, T.Y, c * T.X);
                V3 Yb = axpy(-s, T.X, c * T.Y);
                T.p = axpy(rb->d[i], T.Z, axpy(rb->a[i], Xb, T.p));
                V3 Yn = axpy(sa, T.Z, ca * Yb);
                V3 Zn = axpy(-sa, Yb, ca * T.Z);
                T.X = Xb;
                T.Y = Yn;
                T.Z = Zn;
            }
        }
    }
    // end effector = T_0n * tool
    const auto* tl = rb->tool;
    ee.p = axpy(tl[11], T.Z, axpy(tl[7], T.Y, axpy(tl[3], T.X, T.p)));
    if (rb->tool_rot) {
        ee.X = axpy(tl[8], T.Z, axpy(tl[4], T.Y, tl[0] * T.X));
        ee.Y = axpy(tl[9], T.Z, axpy(tl[5], T.Y, tl[1] * T.X));
        ee.Z = axpy(tl[10], T.Z, axpy(tl[6], T.Y, tl[2] * T.X));
    } else {
        ee.X = T.X;
        ee.Y = T.Y;
        ee.Z = T.Z;
    }
}

// One link-frame step of the chain (used by the collision pass, which needs
// every link frame).  Advances T from frame i-1 to frame i.
__device__ __forceinline__ void chain_step(const DevRobot* __restrict__ rb, int i, float theta,
                                           Frame& T) {
    float s, c;
    sincos_cw(theta + rb->off[i], &s, &c);
    const float ca = rb->ca[i], sa = rb->sa[i];
    if (rb->conv == 0) {
        T.p = axpy(rb->pz[i], T.Z, axpy(rb->py[i], T.Y, axpy(rb->px[i], T.X, T.p)));
        V3 Yb = axpy(sa, T.Z, ca * T.Y);
        V3 Zb = axpy(-sa, T.Y, ca * T.Z);
        V3 Xn = axpy(s, Yb, c * T.X);
        V3 Yn = axpy(-s, T.X, c * Yb);
        T.X = Xn;
        T.Y = Yn;
        T.Z = Zb;
    } else {
        V3 Xb = axpy(s, T.Y, c * T.X);
        V3 Yb = axpy(-s, T.X, c * T.Y);
        T.p = axpy(rb->d[i], T.Z, axpy(rb->a[i], Xb, T.p));
        V3 Yn = axpy(sa, T.Z, ca * Yb);
        V3 Zn = axpy(-sa, Yb, ca * T.Z);
        T.X = Xb;
        T.Y = Yn;
        T.Z = Zn;
    }
}

// a / b for finite b of moderate size (|b| in [2^-100, 2^100]): the hardware
// reciprocal estimate (1 ulp), the quotient, and one correction with the
// exact FMA residual a - q b (Markstein, IA-64 and Elementary Functions,
// 2000), which leaves the quotient within about half an ulp.
__device__ __forceinline__ float div_corr(float a, float b) {
    const float r = __builtin_amdgcn_rcpf(b);
    const float q = a * r;
    return fmaf(fmaf(-q, b, a), r, q);
}

// Rotation -> unit quaternion, Shepperd's method (largest of trace and the
// diagonal decides the divisor), w >= 0; the divisor 4 max(w^2, x^2, y^2,
// z^2) lies in [1, 4].  FAST: hardware square root and reciprocal (1 ulp),
// for the collision pass's compressed link frames.  A residual fed to the
// solver's decisions keeps the correctly rounded square root and the
// corrected quotient (half an ulp): a 2-4 ulp residual moved one sensitive
// PJ-IK trajectory out of the 1e-4 band.
// CANON = false skips the final sign choice (q and -q are the same rotation);
// the cost of a trial only needs |w| and |v| of the error quaternion, which do
// not depend on that sign.
template <bool FAST = false, bool CANON = true>
__device__ __forceinline__ Quat quat_of(const Frame& F) {
    const float R00 = F.X.x, R10 = F.X.y, R20 = F.X.z;
    const float R01 = F.Y.x, R11 = F.Y.y, R21 = F.Y.z;
    const float R02 = F.Z.x, R12 = F.Z.y, R22 = F.Z.z;
    const float tr = R00 + R11 + R22;
    const bool c0 = tr >= R00 && tr >= R11 && tr >= R22;
    const bool c1 = !c0 && R00 >= R11 && R00 >= R22;
    const bool c2 = !c0 && !c1 && R11 >= R22;
    const float big = c0 ? 1.f + tr : c1 ? 1.f + R00 - R11 - R22 : c2 ? 1.f - R00 + R11 - R22
                                                                       : 1.f - R00 - R11 + R22;
    const float r = FAST ? __builtin_amdgcn_sqrtf(big) : sqrtf(big);
    const float qb = 0.5f * r;
    const float k = FAST ? 0.5f * __builtin_amdgcn_rcpf(r) : div_corr(0.5f, r);
    const float d21 = (R21 - R12) * k, d02 = (R02 - R20) * k, d10 = (R10 - R01) * k;
    const float s01 = (R01 + R10) * k, s02 = (R02 + R20) * k, s12 = (R12 + R21) * k;
    Quat q;
    q.w = c0 ? qb : c1 ? d21 : c2 ? d02 : d10;
    q.x = c0 ? d21 : c1 ? qb : c2 ? s01 : s02;
    q.y = c0 ? d02 : c1 ? s01 : c2 ? qb : s12;
    q.z = c0 ? d10 : c1 ? s02 : c2 ? s12 : qb;
    if (CANON && q.w < 0.f) {
        q.w = -q.w;
        q.x = -q.x;
        q.y = -q.y;
        q.z = -q.z;
    }
    return q;
}

// Task residual (eq. task_residual, eq. quat_diff): r_p = P_t - P_ee and the
// error quaternion q_err = q_t (x) q_e^-1 taken with w >= 0 (short rotation);
// phi = 2 atan2(|v|, w) in [0, pi].
struct Err {
    V3 rp;
    Quat q;     // canonical error quaternion
    float s;    // |v|
    float phi;  // rotation angle
    float ep2;  // |r_p|^2
};

struct Target {
    V3 p;
    Quat q;
};

__device__ __forceinline__ Err residual(const Frame& ee, const Target& tg) {
    Err e;
    e.rp = tg.p - ee.p;
    e.ep2 = dot(e.rp, e.rp);
    Quat qe = quat_of(ee);
    qe.x = -qe.x;
    qe.y = -qe.y;
    qe.z = -qe.z;
    Quat q = qmul(tg.q, qe);
    if (q.w < 0.f) {
        q.w = -q.w;
        q.x = -q.x;
        q.y = -q.y;
        q.z = -q.z;
    }
    e.q = q;
    e.s = sqrtf(q.x * q.x + q.y * q.y + q.z * q.z);
    e.phi = 2.f * atan2f(e.s, q.w);
    return e;
}

// omega of eq. (quat_diff): (phi / |v|) v, or 2 v / w when |v| vanishes.
__device__ __forceinline__ V3 omega_of(const Err& e) {
    const float f = e.s > 1e-20f ? e.phi / e.s : 2.f / e.q.w;
    return mk(f * e.q.x, f * e.q.y, f * e.q.z);
}

__device__ __forceinline__ float cost_of(const Err& e) { return 0.5f * (e.ep2 + e.phi * e.phi); }

__device__ __forceinline__ Target load_target(const float* __restrict__ tg, int64_t T, int64_t t) {
    Target g;
    g.p = mk(tg[t], tg[T + t], tg[2 * T + t]);
    float w = tg[3 * T + t], x = tg[4 * T + t], y = tg[5 * T + t], z = tg[6 * T + t];
    float inv = 1.f / sqrtf(w * w + x * x + y * y + z * z);
    g.q = Quat{w * inv, x * inv, y * inv, z * inv};
    return g;
}

// ----------------------------------------------------------------------------
// Philox4x32-10 (Salmon, Moraes, Dror, Shaw, SC'11) and the draws built on it
// ----------------------------------------------------------------------------
struct U4 {
    uint32_t a, b, c, d;
};

__device__ __forceinline__ U4 philox(U4 ctr, uint32_t k0, uint32_t k1) {
#pragma unroll
    for (int r = 0; r < 10; ++r) {
        if (r > 0) {
            k0 += 0x9E3779B9u;
            k1 += 0xBB67AE85u;
        }
        const uint32_t lo0 = 0xD2511F53u * ctr.a, hi0 = __umulhi(0xD2511F53u, ctr.a);
        const uint32_t lo1 = 0xCD9E8D57u * ctr.c, hi1 = __umulhi(0xCD9E8D57u, ctr.c);
        ctr = U4{hi1 ^ ctr.b ^ k0, lo1, hi0 ^ ctr.d ^ k1, lo0};
    }
    return ctr;
}

enum { STAGE_INIT = 0, STAGE_CD = 1, STAGE_RESAMPLE = 2, STAGE_POLISH = 3, STAGE_WARM = 4 };

// Uniform in (0, 1) from the top 24 bits: exact in single precision.
__device__ __forceinline__ float uni24(uint32_t x) {
    return ((float)(x >> 8) + 0.5f) * (1.0f / 16777216.0f);
}

__device__ __forceinline__ U4 draw(uint64_t seed, uint32_t m, uint32_t tkey, uint32_t stage,
                                   uint32_t iter, uint32_t block) {
    return philox(U4{m, tkey, (stage << 24) | (iter & 0xFFFFFFu), block}, (uint32_t)seed,
                  (uint32_t)(seed >> 32));
}

// theta <- clip(theta + mu + sigma z), z ~ N(0, I) by Box-Muller: joint j takes
// word pair (2p, 2p+1), p = (j % 4) / 2, of block j / 4; cos for even j, sin
// for odd j.
template <int NM, typename RB>
__device__ __forceinline__ void perturb(RB rb, int n, float* th,
                                        uint64_t seed, uint32_t m, uint32_t tkey, uint32_t stage,
                                        uint32_t iter, float mu, float sigma) {
#pragma unroll
    for (int b = 0; b < (NM + 3) / 4; ++b) {
        if (4 * b < n) {
            U4 x = draw(seed, m, tkey, stage, iter, (uint32_t)b);
            const uint32_t w[4] = {x.a, x.b, x.c, x.d};
#pragma unroll
            for (int p = 0; p < 2; ++p) {
                const float rad = sqrtf(-2.f * logf(uni24(w[2 * p])));
                float sn, cs;
                sincospif(2.f * uni24(w[2 * p + 1]), &sn, &cs);
#pragma unroll
                for (int h = 0; h < 2; ++h) {
                    const int j = 4 * b + 2 * p + h;
                    if (j < NM && j < n) {
                        const float z = h == 0 ? rad * cs : rad * sn;
                        th[j] = clampf(th[j] + mu + sigma * z, rb->lo[j], rb->hi[j]);
                    }
                }
            }
        }
    }
}

// Order this wave's LDS accesses (in-order execution within a wave; this
// keeps the compiler from moving loads and stores across it).
__device__ __forceinline__ void wave_lds_sync() {
    __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
    __builtin_amdgcn_wave_barrier();
    __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
}

// LDS floats per wave of perturb_spread.
template <int NM>
__host__ __device__ constexpr int perturb_wave_floats() {
    return (NM + 3) * 64;
}

// The same perturbation for the lanes with `want`, its draws spread over the
// wave: each such lane writes its seed index, target key and iteration to
// slot r (its rank) of the wave's LDS rows; task t = q nneed + r draws the
// Box-Muller pair q (joints 2q, 2q + 1: block q / 2, words 2 (q % 2) and
// 2 (q % 2) + 1) of slot r and stores the normals at [2q][r], [2q + 1][r];
// each lane then applies its n normals as perturb does.  The draws and
// updates are perturb's, so the results are the same; the wave runs
// ceil(lanes x ceil(n / 2) / 64) passes of one pair each instead of every
// pair of the lanes that perturb.  Called by the whole wave (uniform control
// flow); `ws` holds perturb_wave_floats<NM>() floats of this wave's LDS.
template <int NM, typename RB>
__device__ __forceinline__ void perturb_spread(RB rb, int n, float* th, bool want, uint64_t seed, uint32_t m,
                                               uint32_t tkey, uint32_t stage, uint32_t iter, float mu, float sigma,
                                               float* __restrict__ ws) {
    const uint64_t need = __ballot(want);
    if (need == 0ull) return;
    const int lane = (int)(threadIdx.x & 63u);
    const int nneed = __popcll(need);
    const int npair = (n + 1) >> 1;
    const int ntask = nneed * npair;
    const int myrank = __popcll(need & ((1ull << lane) - 1ull));
    float* __restrict__ wz = ws;                           // [NM][64] normals by rank
    uint32_t* __restrict__ wk = (uint32_t*)(ws + NM * 64);  // [3][64] m, tkey, iter by rank
    if (want) {
        wk[0 * 64 + myrank] = m;
        wk[1 * 64 + myrank] = tkey;
        wk[2 * 64 + myrank] = iter;
    }
    wave_lds_sync();
    // (t + 1/2) / nneed is at least 1 / 128 away from an integer and t < 1024:
    // its FP32 product with the hardware reciprocal (within 1 ulp) floors exactly
    const float inv_need = __builtin_amdgcn_rcpf((float)nneed);
    for (int base = 0; base < ntask; base += 64) {
        const int t = base + lane;
        if (t < ntask) {
            const int q = (int)(((float)t + 0.5f) * inv_need);  // pair index
            const int r = t - q * nneed;
            const U4 x = draw(seed, wk[0 * 64 + r], wk[1 * 64 + r], stage, wk[2 * 64 + r], (uint32_t)(q >> 1));
            const bool hi = (q & 1) != 0;
            const uint32_t w0 = hi ? x.c : x.a, w1 = hi ? x.d : x.b;
            const float rad = sqrtf(-2.f * logf(uni24(w0)));
            float sn, cs;
            sincospif(2.f * uni24(w1), &sn, &cs);
            wz[(2 * q) * 64 + r] = rad * cs;
            if (2 * q + 1 < n) wz[(2 * q + 1) * 64 + r] = rad * sn;
        }
    }
    wave_lds_sync();
    if (want) {
#pragma unroll
        for (int j = 0; j < NM; ++j) {
            if (j < n) {
                const float z = wz[j * 64 + myrank];
                th[j] = clampf(th[j] + mu + sigma * z, rb->lo[j], rb->hi[j]);
            }
        }
    }
    wave_lds_sync();  // the rows are free for the next writes
}

template <int NM>
__device__ __forceinline__ void uniform_seed(const DevRobot* __restrict__ rb, int n, float* th,
                                             uint64_t seed, uint32_t m, uint32_t tkey) {
#pragma unroll
    for (int b = 0; b < (NM + 3) / 4; ++b) {
        if (4 * b < n) {
            U4 x = draw(seed, m, tkey, STAGE_INIT, 0, (uint32_t)b);
            const uint32_t w[4] = {x.a, x.b, x.c, x.d};
#pragma unroll
            for (int h = 0; h < 4; ++h) {
                const int j = 4 * b + h;
                if (j < NM && j < n) th[j] = fmaf(rb->hi[j] - rb->lo[j], uni24(w[h]), rb->lo[j]);
            }
        }
    }
}

// Rodrigues rotation of w about unit axis z by the angle whose half-angle
// cosine / sine are (ch, sh).
__device__ __forceinline__ V3 rot_half(V3 z, float ch, float sh, V3 w) {
    const float s = 2.f * sh * ch;
    const float omc = 2.f * sh * sh;  // 1 - cos
    return axpy(omc * dot(z, w), z, axpy(s, cross(z, w), axpy(-omc, w, w)));
}

// q (x) conj(q_z(angle)) with q_z(angle) = (ch, sh z)
__device__ __forceinline__ Quat qmul_conj_axis(Quat q, V3 z, float ch, float sh) {
    Quat r;
    const float vz = q.x * z.x + q.y * z.y + q.z * z.z;
    r.w = q.w * ch + sh * vz;
    // ch v - w sh z - sh (v x z)
    const V3 v = mk(q.x, q.y, q.z);
    const V3 vxz = cross(v, z);
    r.x = ch * v.x - q.w * sh * z.x - sh * vxz.x;
    r.y = ch * v.y - q.w * sh * z.y - sh * vxz.y;
    r.z = ch * v.z - q.w * sh * z.z - sh * vxz.z;
    return r;
}

// ----------------------------------------------------------------------------
// Per-lane counters of executed work (summed per wave, then atomically)
// ----------------------------------------------------------------------------
struct Counters {
    uint32_t cd_iters = 0, cd_perturb = 0, pol_iters = 0, pol_trials = 0, pol_dogleg = 0,
             pol_single = 0, pol_perturb = 0, coll_coarse = 0, coll_fine = 0;
};

__device__ __forceinline__ uint32_t wave_sum(uint32_t v) {
#pragma unroll
    for (int o = 32; o > 0; o >>= 1) v += __shfl_xor(v, o, 64);
    return v;
}

__device__ __forceinline__ void flush_counters(const Counters& c, unsigned long long* __restrict__ out,
                                               bool enabled) {
    if (!enabled) return;
    const uint32_t v[9] = {c.cd_iters, c.cd_perturb, c.pol_iters, c.pol_trials, c.pol_dogleg,
                           c.pol_single, c.pol_perturb, c.coll_coarse, c.coll_fine};
#pragma unroll
    for (int i = 0; i < 9; ++i) {
        const uint32_t s = wave_sum(v[i]);
        if ((threadIdx.x & 63) == 0 && s) atomicAdd(out + i, (unsigned long long)s);
    }
}

__device__ __forceinline__ bool wave_all(bool p) {
    return __ballot(!p) == 0ull;
}

__device__ __forceinline__ bool wave_any(bool p) { return __ballot(p) != 0ull; }

// ----------------------------------------------------------------------------
// Parameters as the kernels read them (KernelParams of hjcd_launch.hpp)
// ----------------------------------------------------------------------------
using KParams = KernelParams;

// ----------------------------------------------------------------------------
// Trajectory row: theta, |r_p|, phi of every seed, [rows][n+2][S].
template <int NM>
__device__ __forceinline__ void write_traj(float* __restrict__ traj, int n, int64_t S, int64_t s,
                                           int row, const float* th, float ep, float phi) {
    if (!traj) return;
    float* base = traj + (int64_t)row * (n + 2) * S + s;
#pragma unroll
    for (int j = 0; j < NM; ++j)
        if (j < n) base[(int64_t)j * S] = th[j];
    base[(int64_t)n * S] = ep;
    base[(int64_t)(n + 1) * S] = phi;
}

// ----------------------------------------------------------------------------
// The two PO-CCD candidates of one joint (origin P, axis z, value tj, limits
// lo..hi) at the pose ee with residual e (Sec. III, Sec. IV-A):
//  - position, eq. (vec_proj) / (theta_proj) signed about z, clipped: step dp,
//    score sp = |r_p|^2 after the move (rigid rotation of the EE about z);
//  - orientation, eq. (ori_update) delta(k) sgn(a_hat . z) phi, clipped: step
//    dor, ranked by (oV, oW) = (|v'|^2, w'^2) of the moved error quaternion,
//    which orders like tan^2(phi'/2).
// (shu, chu): half-angle sine / cosine of the unclipped move dk * phi.
// ----------------------------------------------------------------------------
__device__ __forceinline__ void cd_candidate(V3 P, V3 z, float tj, float lo, float hi, const Frame& ee, const Err& e,
                                             const Target& tg, const KParams& kp, float dk, float shu, float chu,
                                             float& sp, float& dp, float& oV, float& oW, float& dor_out) {
    const V3 u = ee.p - P;
    const V3 v = tg.p - P;
    const float uz = dot(u, z), vz = dot(v, z);
    const V3 up = axpy(-uz, z, u);
    const V3 vp = axpy(-vz, z, v);
    const float du2 = dot(up, up), dv2 = dot(vp, vp);
    const bool valid = du2 >= kp.proj_eps2 && dv2 >= kp.proj_eps2;
    // eq. (vec_proj) / (theta_proj), signed about z
    const float C = dot(up, vp);
    const float Sg = dot(z, cross(up, vp));
    const float d = valid ? atan2f(Sg, C) : 0.f;
    const bool clp = (tj + d > hi) || (tj + d < lo);
    dp = clp ? clampf(tj + d, lo, hi) - tj : d;
    const float az = vz - uz;
    if (!valid) {
        sp = e.ep2;
    } else if (!clp) {
        // the move aligns up with vp: |v - R u|^2 = az^2 + (|vp| - |up|)^2
        const float dd = sqrtf(dv2) - sqrtf(du2);
        sp = fmaf(az, az, dd * dd);
    } else {
        float sh, ch;
        sincos_cw(0.5f * dp, &sh, &ch);
        const float c2 = 1.f - 2.f * sh * sh, s2 = 2.f * sh * ch;
        const V3 rw = axpy(s2, cross(z, up), c2 * up);
        const V3 df = vp - rw;
        sp = fmaf(az, az, dot(df, df));
    }
    // eq. (ori_update): delta(k) sgn(a_hat . z) phi
    const float vzq = e.q.x * z.x + e.q.y * z.y + e.q.z * z.z;
    const float sg = vzq > 0.f ? 1.f : (vzq < 0.f ? -1.f : 0.f);
    const float dor = dk * sg * e.phi;
    const bool clo = (tj + dor > hi) || (tj + dor < lo);
    float ch = chu, sh = sg * shu;
    float doc = dor;
    if (clo) {
        doc = clampf(tj + dor, lo, hi) - tj;
        sincos_cw(0.5f * doc, &sh, &ch);
    }
    const Quat qn = qmul_conj_axis(e.q, z, ch, sh);
    oV = qn.x * qn.x + qn.y * qn.y + qn.z * qn.z;
    oW = qn.w * qn.w;
    dor_out = doc;
}

// ----------------------------------------------------------------------------
// PO-CCD (Alg. PO-CCD, Sec. III, Sec. IV-A) on one seed, iterations
// [k0, k1).  `live` is false for padding lanes; they run the uniform control
// flow with no effect.  `frozen` carries the exit state across calls (a
// fresh seed starts with frozen = !live).  out_err is the residual at the
// configuration the last iteration produced.
// ----------------------------------------------------------------------------
// PSPREAD: the perturbations of rejected moves run through perturb_spread
// on the wave's LDS rows `pws` (same results).
template <int NM, bool PSPREAD = false>
__device__ __forceinline__ void po_ccd(const DevRobot* __restrict__ rb, int n, const Target& tg, const KParams& kp,
                                       uint32_t m, uint32_t tkey, float* th, bool live, bool& frozen,
                                       Counters& cnt, float* __restrict__ traj, int64_t S, int64_t s, int k0,
                                       int k1, Err& out_err, float* __restrict__ pws = nullptr) {
    float last_ep = 0.f, last_phi = 0.f;
    V3 P[NM], Z[NM];
    float delta = kp.delta0 * powf(kp.delta_decay, (float)k0);
    for (int k = k0; k < k1; ++k) {
        if (wave_all(frozen) && !traj) break;
        bool pert = false;  // this iteration's move was rejected
        if (!frozen) {
            Frame ee;
            fk_chain<NM, true>(rb, n, th, P, Z, ee);
            const Err e = residual(ee, tg);
            last_ep = sqrtf(e.ep2);
            last_phi = e.phi;
            // exit test on the configuration the previous iteration produced
            if (e.ep2 < kp.eps_cd2 && e.phi < kp.nu_cd) frozen = true;
            if (live) write_traj<NM>(traj, n, S, s, k, th, last_ep, last_phi);
            if (!frozen) {
                ++cnt.cd_iters;
                const float dk = fmaxf(kp.delta_min, delta);
                // half-angle of the unclamped orientation move |delta(k) phi|
                float shu, chu;
                sincos_cw(0.5f * dk * e.phi, &shu, &chu);
                // --- per-joint candidates ---------------------------------
                // Position candidates are ranked by their squared residual sp;
                // orientation candidates by phi' = 2 atan2(|v'|, |w'|) through
                // the pair (v'^2, w'^2), which orders like tan^2(phi'/2).  Only
                // the best of each needs its score in m / rad (for the
                // tie-tolerant pick below).
                float sPq[NM], dP[NM], oV[NM], oW[NM], dO[NM];
                float spmin = 3.4e38f;
                float bv = 1.f, bw = 0.f;  // (v'^2, w'^2) of the best orientation candidate (phi' = pi)
#pragma unroll
                for (int j = 0; j < NM; ++j) {
                    sPq[j] = 3.4e38f;
                    oV[j] = 1.f;
                    oW[j] = 0.f;
                    dP[j] = 0.f;
                    dO[j] = 0.f;
                    if (j < n) {
                        cd_candidate(P[j], Z[j], th[j], rb->lo[j], rb->hi[j], ee, e, tg, kp, dk, shu, chu, sPq[j],
                                     dP[j], oV[j], oW[j], dO[j]);
                        spmin = fminf(spmin, sPq[j]);
                        // tan^2(phi'_j / 2) < tan^2(phi'_best / 2), cross-multiplied
                        if (oV[j] * bw < bv * oW[j]) {
                            bv = oV[j];
                            bw = oW[j];
                        }
                    }
                }
                // greedy picks: the lowest joint whose score lies within tie_eps
                // of the best: sqrt(sp_j) <= sqrt(sp_min) + tie_eps, and
                // phi'_j <= phi'_min + tie_eps, i.e. tan^2(phi'_j/2) <=
                // tan^2(h) with h = (phi'_min + tie_eps) / 2 (every candidate
                // passes when h >= pi/2)
                const float dlim = sqrtf(spmin) + kp.tie_eps;
                const float plim = dlim * dlim;
                const float hlim = 0.5f * (2.f * atan2f(sqrtf(bv), sqrtf(bw)) + kp.tie_eps);
                const bool oall = hlim >= 1.5707963f;
                float sT, cT;
                sincos_cw(oall ? 0.f : hlim, &sT, &cT);
                const float sT2 = sT * sT, cT2 = cT * cT;
                int jp = -1, jo = -1;
                float dpb = 0.f, dob = 0.f;
#pragma unroll
                for (int j = 0; j < NM; ++j) {
                    if (j < n) {
                        if (jp < 0 && sPq[j] <= plim) {
                            jp = j;
                            dpb = dP[j];
                        }
                        if (jo < 0 && (oall || oV[j] * cT2 <= oW[j] * sT2)) {
                            jo = j;
                            dob = dO[j];
                        }
                    }
                }
                // --- combine (Sec. IV-A): both moves, or the larger on one joint
                int ja = jp, jb = jo;
                float da = dpb, db = dob;
                if (jp == jo) {
                    if (fabsf(dpb) >= fabsf(dob)) {
                        db = 0.f;
                    } else {
                        da = 0.f;
                    }
                    jb = ja;
                    da = da + db;  // one of them is 0
                    db = 0.f;
                } else if (jo < jp) {
                    ja = jo;
                    jb = jp;
                    da = dob;
                    db = dpb;
                }
                // rigid update of the EE pose: distal move (jb) first, both axes
                // taken at theta; ja <= jb.
                V3 Pa = P[0], Za = Z[0], Pb = P[0], Zb = Z[0];
#pragma unroll
                for (int j = 0; j < NM; ++j) {
                    if (j == ja) {
                        Pa = P[j];
                        Za = Z[j];
                    }
                    if (j == jb) {
                        Pb = P[j];
                        Zb = Z[j];
                    }
                }
                float sha, cha, shb, chb;
                sincos_cw(0.5f * da, &sha, &cha);
                sincos_cw(0.5f * db, &shb, &chb);
                V3 ph = Pb + rot_half(Zb, chb, shb, ee.p - Pb);
                ph = Pa + rot_half(Za, cha, sha, ph - Pa);
                Quat qh = qmul_conj_axis(qmul_conj_axis(e.q, Zb, chb, shb), Za, cha, sha);
                const V3 rph = tg.p - ph;
                const float h2p = dot(rph, rph);
                const float hs = sqrtf(qh.x * qh.x + qh.y * qh.y + qh.z * qh.z);
                const float hphi = 2.f * atan2f(hs, fabsf(qh.w));
                const bool acc = (e.ep2 - h2p > kp.gamma) || (e.phi * e.phi - hphi * hphi > kp.gamma);
                if (acc) {
#pragma unroll
                    for (int j = 0; j < NM; ++j) {
                        if (j == ja) th[j] += da;
                        if (j == jb) th[j] += db;
                    }
                } else {
                    pert = true;
                    ++cnt.cd_perturb;
                }
            }
        } else if (live) {
            write_traj<NM>(traj, n, S, s, k, th, last_ep, last_phi);
        }
        // rejected: random perturbation
        if (PSPREAD)
            perturb_spread<NM>(rb, n, th, pert, kp.seed, m, tkey, STAGE_CD, (uint32_t)k, kp.mu, kp.sigma, pws);
        else if (pert)
            perturb<NM>(rb, n, th, kp.seed, m, tkey, STAGE_CD, (uint32_t)k, kp.mu, kp.sigma);
        delta *= kp.delta_decay;
    }
    Frame ee;
    V3 Pd[1], Zd[1];
    fk_chain<NM, false>(rb, n, th, Pd, Zd, ee);
    out_err = residual(ee, tg);
    if (live) write_traj<NM>(traj, n, S, s, k1, th, sqrtf(out_err.ep2), out_err.phi);
}

// ----------------------------------------------------------------------------
// PO-CCD with two lanes per seed (lane pairs 2i, 2i+1 of a wave), for long
// chains: both lanes hold the joint vector and walk the whole chain, the even
// lane keeps the frames and candidates of joints [0, NM/2), the odd lane
// those of [NM/2, NM), so the per-joint state of a lane is half that of
// po_ccd.  The picks are combined across the pair by shuffles in the same
// order po_ccd scans the joints (lowest joint first), so both lanes take the
// same steps, draws and decisions as po_ccd.
// ----------------------------------------------------------------------------
// FK (eq. fk) keeping the joint origins and axes of this lane's half:
// P0[k], Z0[k] = joint k (even lane) or joint k + NM/2 (odd lane).
template <int NM, typename RB>
__device__ __forceinline__ void fk_chain_half(RB rb, int n, const float* th, bool odd, V3* P0, V3* Z0, Frame& ee) {
    constexpr int H = NM / 2;
    Frame T = identity_frame();
    auto keep = [&](int i, const Frame& F) {
        if (i < H) {
            if (!odd) {
                P0[i] = F.p;
                Z0[i] = F.Z;
            }
        } else {
            if (odd) {
                P0[i - H] = F.p;
                Z0[i - H] = F.Z;
            }
        }
    };
    if (rb->conv == 0) {
#pragma unroll
        for (int i = 0; i < NM; ++i) {
            if (i < n) {
                float s, c;
                sincos_cw(th[i] + rb->off[i], &s, &c);
                const float ca = rb->ca[i], sa = rb->sa[i];
                T.p = axpy(rb->pz[i], T.Z, axpy(rb->py[i], T.Y, axpy(rb->px[i], T.X, T.p)));
                V3 Yb = axpy(sa, T.Z, ca * T.Y);
                V3 Zb = axpy(-sa, T.Y, ca * T.Z);
                V3 Xn = axpy(s, Yb, c * T.X);
                V3 Yn = axpy(-s, T.X, c * Yb);
                T.X = Xn;
                T.Y = Yn;
                T.Z = Zb;
                keep(i, T);
            }
        }
    } else {
#pragma unroll
        for (int i = 0; i < NM; ++i) {
            if (i < n) {
                keep(i, T);
                float s, c;
                sincos_cw(th[i] + rb->off[i], &s, &c);
                const float ca = rb->ca[i], sa = rb->sa[i];
                V3 Xb = axpy(s, T.Y, c * T.X);
                V3 Yb = axpy(-s, T.X, c * T.Y);
                T.p = axpy(rb->d[i], T.Z, axpy(rb->a[i], Xb, T.p));
                V3 Yn = axpy(sa, T.Z, ca * Yb);
                V3 Zn = axpy(-sa, Yb, ca * T.Z);
                T.X = Xb;
                T.Y = Yn;
                T.Z = Zn;
            }
        }
    }
    const auto* tl = rb->tool;
    ee.p = axpy(tl[11], T.Z, axpy(tl[7], T.Y, axpy(tl[3], T.X, T.p)));
    if (rb->tool_rot) {
        ee.X = axpy(tl[8], T.Z, axpy(tl[4], T.Y, tl[0] * T.X));
        ee.Y = axpy(tl[9], T.Z, axpy(tl[5], T.Y, tl[1] * T.X));
        ee.Z = axpy(tl[10], T.Z, axpy(tl[6], T.Y, tl[2] * T.X));
    } else {
        ee.X = T.X;
        ee.Y = T.Y;
        ee.Z = T.Z;
    }
}

__device__ __forceinline__ V3 shfl_pair(V3 v) {
    return mk(__shfl_xor(v.x, 1, 64), __shfl_xor(v.y, 1, 64), __shfl_xor(v.z, 1, 64));
}

template <int NM>
__device__ __forceinline__ void po_ccd_pair(const DevRobot* __restrict__ rb, int n, const Target& tg, const KParams& kp,
                                            uint32_t m, uint32_t tkey, float* th, bool live, bool& frozen,
                                            Counters& cnt, float* __restrict__ traj, int64_t S, int64_t s, int k0,
                                            int k1, Err& out_err) {
    static_assert(NM % 2 == 0, "lane pairs split an even joint bucket");
    constexpr int H = NM / 2;
    const bool odd = (threadIdx.x & 1u) != 0;
    const int base = odd ? H : 0;  // first joint of this lane's half
    float last_ep = 0.f, last_phi = 0.f;
    V3 P0[H], Z0[H];
    float delta = kp.delta0 * powf(kp.delta_decay, (float)k0);
    for (int k = k0; k < k1; ++k) {
        if (wave_all(frozen) && !traj) break;
        if (!frozen) {
            Frame ee;
            fk_chain_half<NM>(rb, n, th, odd, P0, Z0, ee);
            const Err e = residual(ee, tg);
            last_ep = sqrtf(e.ep2);
            last_phi = e.phi;
            if (e.ep2 < kp.eps_cd2 && e.phi < kp.nu_cd) frozen = true;
            if (live && !odd) write_traj<NM>(traj, n, S, s, k, th, last_ep, last_phi);
            if (!frozen) {
                if (!odd) ++cnt.cd_iters;
                const float dk = fmaxf(kp.delta_min, delta);
                float shu, chu;
                sincos_cw(0.5f * dk * e.phi, &shu, &chu);
                float sPq[H], dP[H], oV[H], oW[H], dO[H];
                float spmin = 3.4e38f;
                float bv = 1.f, bw = 0.f;
#pragma unroll
                for (int i = 0; i < H; ++i) {
                    const int j = base + i;
                    sPq[i] = 3.4e38f;
                    oV[i] = 1.f;
                    oW[i] = 0.f;
                    dP[i] = 0.f;
                    dO[i] = 0.f;
                    if (j < n) {
                        const float tj = odd ? th[i + H] : th[i];
                        const float lo = odd ? rb->lo[i + H] : rb->lo[i];
                        const float hi = odd ? rb->hi[i + H] : rb->hi[i];
                        cd_candidate(P0[i], Z0[i], tj, lo, hi, ee, e, tg, kp, dk, shu, chu, sPq[i], dP[i], oV[i],
                                     oW[i], dO[i]);
                        spmin = fminf(spmin, sPq[i]);
                        if (oV[i] * bw < bv * oW[i]) {
                            bv = oV[i];
                            bw = oW[i];
                        }
                    }
                }
                // pair: the smallest position score, and the best orientation
                // candidate of the lower half unless the upper half's is
                // strictly better (the joint order of a single scan)
                spmin = fminf(spmin, __shfl_xor(spmin, 1, 64));
                {
                    const float pv = __shfl_xor(bv, 1, 64), pw = __shfl_xor(bw, 1, 64);
                    const float ve = odd ? pv : bv, we = odd ? pw : bw;
                    const float vo = odd ? bv : pv, wo = odd ? bw : pw;
                    const bool up = vo * we < ve * wo;
                    bv = up ? vo : ve;
                    bw = up ? wo : we;
                }
                const float dlim = sqrtf(spmin) + kp.tie_eps;
                const float plim = dlim * dlim;
                const float hlim = 0.5f * (2.f * atan2f(sqrtf(bv), sqrtf(bw)) + kp.tie_eps);
                const bool oall = hlim >= 1.5707963f;
                float sT, cT;
                sincos_cw(oall ? 0.f : hlim, &sT, &cT);
                const float sT2 = sT * sT, cT2 = cT * cT;
                int jp = -1, jo = -1;
                float dpb = 0.f, dob = 0.f;
#pragma unroll
                for (int i = 0; i < H; ++i) {
                    if (base + i < n) {
                        if (jp < 0 && sPq[i] <= plim) {
                            jp = base + i;
                            dpb = dP[i];
                        }
                        if (jo < 0 && (oall || oV[i] * cT2 <= oW[i] * sT2)) {
                            jo = base + i;
                            dob = dO[i];
                        }
                    }
                }
                // the lowest pick of the pair
                {
                    const int pjp = __shfl_xor(jp, 1, 64), pjo = __shfl_xor(jo, 1, 64);
                    const float pdp = __shfl_xor(dpb, 1, 64), pdo = __shfl_xor(dob, 1, 64);
                    const int ejp = odd ? pjp : jp, ojp = odd ? jp : pjp;
                    const float edp = odd ? pdp : dpb, odp = odd ? dpb : pdp;
                    const int ejo = odd ? pjo : jo, ojo = odd ? jo : pjo;
                    const float edo = odd ? pdo : dob, odo = odd ? dob : pdo;
                    jp = ejp >= 0 ? ejp : ojp;
                    dpb = ejp >= 0 ? edp : odp;
                    jo = ejo >= 0 ? ejo : ojo;
                    dob = ejo >= 0 ? edo : odo;
                }
                int ja = jp, jb = jo;
                float da = dpb, db = dob;
                if (jp == jo) {
                    if (fabsf(dpb) >= fabsf(dob)) {
                        db = 0.f;
                    } else {
                        da = 0.f;
                    }
                    jb = ja;
                    da = da + db;
                    db = 0.f;
                } else if (jo < jp) {
                    ja = jo;
                    jb = jp;
                    da = dob;
                    db = dpb;
                }
                // origins and axes of the moved joints from the lane that keeps them
                V3 Pa = P0[0], Za = Z0[0], Pb = P0[0], Zb = Z0[0];
#pragma unroll
                for (int i = 0; i < H; ++i) {
                    if (base + i == ja) {
                        Pa = P0[i];
                        Za = Z0[i];
                    }
                    if (base + i == jb) {
                        Pb = P0[i];
                        Zb = Z0[i];
                    }
                }
                {
                    const bool own_a = odd == (ja >= H), own_b = odd == (jb >= H);
                    const V3 qPa = shfl_pair(Pa), qZa = shfl_pair(Za), qPb = shfl_pair(Pb), qZb = shfl_pair(Zb);
                    if (!own_a) {
                        Pa = qPa;
                        Za = qZa;
                    }
                    if (!own_b) {
                        Pb = qPb;
                        Zb = qZb;
                    }
                }
                float sha, cha, shb, chb;
                sincos_cw(0.5f * da, &sha, &cha);
                sincos_cw(0.5f * db, &shb, &chb);
                V3 ph = Pb + rot_half(Zb, chb, shb, ee.p - Pb);
                ph = Pa + rot_half(Za, cha, sha, ph - Pa);
                Quat qh = qmul_conj_axis(qmul_conj_axis(e.q, Zb, chb, shb), Za, cha, sha);
                const V3 rph = tg.p - ph;
                const float h2p = dot(rph, rph);
                const float hs = sqrtf(qh.x * qh.x + qh.y * qh.y + qh.z * qh.z);
                const float hphi = 2.f * atan2f(hs, fabsf(qh.w));
                const bool acc = (e.ep2 - h2p > kp.gamma) || (e.phi * e.phi - hphi * hphi > kp.gamma);
                if (acc) {
#pragma unroll
                    for (int j = 0; j < NM; ++j) {
                        if (j == ja) th[j] += da;
                        if (j == jb) th[j] += db;
                    }
                } else {
                    perturb<NM>(rb, n, th, kp.seed, m, tkey, STAGE_CD, (uint32_t)k, kp.mu, kp.sigma);
                    if (!odd) ++cnt.cd_perturb;
                }
            }
        } else if (live && !odd) {
            write_traj<NM>(traj, n, S, s, k, th, last_ep, last_phi);
        }
        delta *= kp.delta_decay;
    }
    Frame ee;
    V3 Pd[1], Zd[1];
    fk_chain<NM, false>(rb, n, th, Pd, Zd, ee);
    out_err = residual(ee, tg);
    if (live && !odd) write_traj<NM>(traj, n, S, s, k1, th, sqrtf(out_err.ep2), out_err.phi);
}

// ----------------------------------------------------------------------------
// 6 x 6 Cholesky in registers (packed lower triangle, 21 entries)
// ----------------------------------------------------------------------------
__device__ __forceinline__ int tri(int i, int j) { return i * (i + 1) / 2 + j; }  // i >= j

// The 6 x 6 systems are assembled and factored in double precision: near
// singular J their condition number (up to ~|J|^2 / lambda) is beyond what
// single precision resolves, and double FMAs issue at the same per-lane rate
// as unpacked single ones on CDNA4.
//
// 1/sqrt(s) and 1/d in double precision from the single-precision hardware
// estimates (relative error ~2^-22) and two Newton steps each (quadratic
// convergence: ~2^-44, then rounding-limited), a few FMAs instead of the
// library's division and square-root sequences.  Arguments are the positive
// pivots and column norms of the 6 x 6 systems (>= lambda > 0).
__device__ __forceinline__ double rsqrt_nr(double s) {
    double r = (double)rsqrtf((float)fmax(s, 1e-30));
    const double hs = 0.5 * s;
    r = r * fma(-hs * r, r, 1.5);
    r = r * fma(-hs * r, r, 1.5);
    return r;
}

__device__ __forceinline__ double rcp_nr(double d) {
    double r = (double)__builtin_amdgcn_rcpf((float)d);
    r = r * fma(-d, r, 2.0);
    r = r * fma(-d, r, 2.0);
    return r;
}

// In place: A (lower, packed) -> L with A = L L^T, and the reciprocals of
// L's diagonal in inv.  Returns false if a pivot is not positive.
__device__ __forceinline__ bool chol6(double* A, double* inv) {
    bool ok = true;
#pragma unroll
    for (int j = 0; j < 6; ++j) {
        double s = A[tri(j, j)];
#pragma unroll
        for (int k = 0; k < j; ++k) s = fma(-A[tri(j, k)], A[tri(j, k)], s);
        ok = ok && (s > 0.0);
        const double il = rsqrt_nr(fmax(s, 1e-300));
        A[tri(j, j)] = s * il;
        inv[j] = il;
#pragma unroll
        for (int i = j + 1; i < 6; ++i) {
            double t = A[tri(i, j)];
#pragma unroll
            for (int k = 0; k < j; ++k) t = fma(-A[tri(i, k)], A[tri(j, k)], t);
            A[tri(i, j)] = t * il;
        }
    }
    return ok;
}

__device__ __forceinline__ void chol6_solve(const double* L, const double* inv, const double* b, double* x) {
    double y[6];
#pragma unroll
    for (int i = 0; i < 6; ++i) {
        double t = b[i];
#pragma unroll
        for (int k = 0; k < i; ++k) t = fma(-L[tri(i, k)], y[k], t);
        y[i] = t * inv[i];
    }
#pragma unroll
    for (int i = 5; i >= 0; --i) {
        double t = y[i];
#pragma unroll
        for (int k = i + 1; k < 6; ++k) t = fma(-L[tri(k, i)], x[k], t);
        x[i] = t * inv[i];
    }
}

// Column j of J (eq. jacobian) with J stored as Jp[j] = z_j x (P_ee - P_j), Z[j].
__device__ __forceinline__ void jcol(const V3* Jp, const V3* Z, int j, float* c) {
    c[0] = Jp[j].x;
    c[1] = Jp[j].y;
    c[2] = Jp[j].z;
    c[3] = Z[j].x;
    c[4] = Z[j].y;
    c[5] = Z[j].z;
}

// Cost 0.5 (|r_p|^2 + phi^2) of a trial configuration: the residual's
// arithmetic without the sign choices of the quaternions (phi = 2 atan2(|v|,
// |w|) is the same for q and -q), so the value equals cost_of(residual(...)).
template <int NM>
__device__ __forceinline__ float trial_cost(RobotRef rb, int n, const Target& tg,
                                            const float* tt) {
    Frame ee;
    V3 Pd[1], Zd[1];
    fk_chain<NM, false>(rb, n, tt, Pd, Zd, ee);
    const V3 rp = tg.p - ee.p;
    const float ep2 = dot(rp, rp);
    Quat qe = quat_of<false, false>(ee);
    qe.x = -qe.x;
    qe.y = -qe.y;
    qe.z = -qe.z;
    const Quat q = qmul(tg.q, qe);
    const float sv = sqrtf(q.x * q.x + q.y * q.y + q.z * q.z);
    const float phi = 2.f * atan2f(sv, fabsf(q.w));
    return 0.5f * (ep2 + phi * phi);
}

// ----------------------------------------------------------------------------
// PJ-IK line search with the later trials spread over the wave.
//
// The first trial (alpha = 1) runs on every lane that still searches.  The
// lanes it did not satisfy need alpha = 1/beta, ..., 1/beta^A in order and
// take the first that lowers the cost.  Those trials are independent, so they
// are evaluated all at once as (lane, alpha) tasks dealt to every lane of the
// wave (converged and satisfied lanes included), 64 tasks per pass; each
// searching lane then takes its first decreasing alpha.  The trial values and
// costs are the ones the sequential search computes, so the choice is the
// same; the wave runs ceil(searching lanes x A / 64) passes instead of A.
// Counters record the trials the sequential search would run.
// ----------------------------------------------------------------------------
constexpr int kLsSpread = 8;  // largest A handled this way

// Lane index of the r-th set bit of m (r < popcount(m)): binary descent
// over halves of the 64-bit mask.
__device__ __forceinline__ int nth_set_bit(uint64_t m, int r) {
    int pos = 0;
#pragma unroll
    for (int w = 32; w >= 1; w >>= 1) {
        const uint64_t low = m & ((1ull << w) - 1ull);
        const int c = __popcll(low);
        const bool up = r >= c;
        r = up ? r - c : r;
        m = up ? (m >> w) : low;
        pos += up ? w : 0;
    }
    return pos;
}

template <int NM>
__device__ __forceinline__ void line_search_spread(RobotRef rb, int n, const Target& tg,
                                                   const KParams& kp, float* th, const float* dth, float* tt,
                                                   float c0, bool& done, Counters& cnt) {
    // alpha = 1 on the searching lanes
    if (!wave_all(done)) {
        if (!done) {
#pragma unroll
            for (int j = 0; j < NM; ++j)
                if (j < n) tt[j] = clampf(fmaf(1.f, dth[j], th[j]), rb->lo[j], rb->hi[j]);
            const float c1 = trial_cost<NM>(rb, n, tg, tt);
            ++cnt.pol_trials;
            if (c1 < c0) {
#pragma unroll
                for (int j = 0; j < NM; ++j)
                    if (j < n) th[j] = tt[j];
                done = true;
            }
        }
    }
    const int A = kp.ls_A;
    const uint64_t need = __ballot(!done);
    if (A == 0 || need == 0ull) return;
    const int lane = (int)(threadIdx.x & 63u);
    const int ntask = __popcll(need) * A;
    const int myrank = __popcll(need & ((1ull << lane) - 1ull));
    uint32_t lower = 0u;  // bit k: trial k + 1 lowers this lane's cost
    for (int base = 0; base < ntask; base += 64) {
        const int t = base + lane;
        const bool has = t < ntask;
        const int r = has ? t / A : 0;
        const int i = has ? 1 + t - r * A : 1;  // trial index 1..A
        const int L = nth_set_bit(need, r);
        // alpha_i as the sequential search forms it: i products by 1/beta
        float a = 1.f;
#pragma unroll
        for (int k = 1; k <= kLsSpread; ++k)
            if (k <= i) a *= kp.inv_beta;
#pragma unroll
        for (int j = 0; j < NM; ++j) {
            const float thL = __shfl(th[j], L, 64);
            const float dL = __shfl(dth[j], L, 64);
            if (j < n) tt[j] = clampf(fmaf(a, dL, thL), rb->lo[j], rb->hi[j]);
        }
        Target tgL;
        tgL.p = mk(__shfl(tg.p.x, L, 64), __shfl(tg.p.y, L, 64), __shfl(tg.p.z, L, 64));
        tgL.q = Quat{__shfl(tg.q.w, L, 64), __shfl(tg.q.x, L, 64), __shfl(tg.q.y, L, 64), __shfl(tg.q.z, L, 64)};
        float c = 3.4e38f;
        if (has) c = trial_cost<NM>(rb, n, tgL, tt);
        // each searching lane collects its tasks dealt in this pass
#pragma unroll
        for (int k = 0; k < kLsSpread; ++k) {
            const int tk = myrank * A + k;
            const bool mine = k < A && tk >= base && tk < base + 64;
            const float v = __shfl(c, mine ? tk - base : lane, 64);
            if (!done && mine && v < c0) lower |= 1u << k;
        }
    }
    if (!done) {
        const int first = lower ? __builtin_ctz(lower) : -1;
        cnt.pol_trials += first >= 0 ? (uint32_t)(first + 1) : (uint32_t)A;
        if (first >= 0) {
            float a = 1.f;
#pragma unroll
            for (int k = 1; k <= kLsSpread; ++k)
                if (k <= first + 1) a *= kp.inv_beta;
#pragma unroll
            for (int j = 0; j < NM; ++j)
                if (j < n) th[j] = clampf(fmaf(a, dth[j], th[j]), rb->lo[j], rb->hi[j]);
            done = true;
        }
    }
}

// ----------------------------------------------------------------------------
// The same spread line search with the searching lanes' records staged in LDS.
//
// Each lane the alpha = 1 trial did not satisfy writes its joint values, step
// and target to slot r (its rank among those lanes) of the wave's own LDS
// records, structure-of-arrays by field so that a pass reads and writes
// consecutive words.  Task t = (i - 1) nneed + r evaluates trial i of slot r
// and stores its cost at [i - 1][r]; each searching lane then reads its A
// costs, takes the first below c0 and rebuilds that trial (its step read back
// from the records).  Only this wave's lanes touch its records, so no
// workgroup barrier is needed.  Values and choices are those of the
// sequential search.
// ----------------------------------------------------------------------------
template <int NM>
__host__ __device__ constexpr int ls_wave_floats() {
    return (2 * NM + 7 + kLsSpread) * 64;
}

template <int NM>
__device__ __forceinline__ void line_search_lds(RobotRef rb, int n, const Target& tg, const KParams& kp, float* th,
                                                const float* dth, float* tt, float c0, bool& done, Counters& cnt,
                                                float* __restrict__ ws) {
    if (!wave_all(done)) {
        if (!done) {
#pragma unroll
            for (int j = 0; j < NM; ++j)
                if (j < n) tt[j] = clampf(fmaf(1.f, dth[j], th[j]), rb->lo[j], rb->hi[j]);
            const float c1 = trial_cost<NM>(rb, n, tg, tt);
            ++cnt.pol_trials;
            if (c1 < c0) {
#pragma unroll
                for (int j = 0; j < NM; ++j)
                    if (j < n) th[j] = tt[j];
                done = true;
            }
        }
    }
    const int A = kp.ls_A;
    const uint64_t need = __ballot(!done);
    if (A == 0 || need == 0ull) return;
    const int lane = (int)(threadIdx.x & 63u);
    const int nneed = __popcll(need);
    const int ntask = nneed * A;
    const int myrank = __popcll(need & ((1ull << lane) - 1ull));
    float* __restrict__ wth = ws;                     // [NM][64] by rank
    float* __restrict__ wdt = ws + NM * 64;           // [NM][64] by rank
    float* __restrict__ wtg = ws + 2 * NM * 64;       // [7][64] by rank
    float* __restrict__ wc = ws + (2 * NM + 7) * 64;  // [A][64] by rank
    if (!done) {
#pragma unroll
        for (int j = 0; j < NM; ++j) {
            if (j < n) {
                wth[j * 64 + myrank] = th[j];
                wdt[j * 64 + myrank] = dth[j];
            }
        }
        wtg[0 * 64 + myrank] = tg.p.x;
        wtg[1 * 64 + myrank] = tg.p.y;
        wtg[2 * 64 + myrank] = tg.p.z;
        wtg[3 * 64 + myrank] = tg.q.w;
        wtg[4 * 64 + myrank] = tg.q.x;
        wtg[5 * 64 + myrank] = tg.q.y;
        wtg[6 * 64 + myrank] = tg.q.z;
    }
    wave_lds_sync();
    // (t + 1/2) / nneed is at least 1 / 128 away from an integer and t < 512:
    // its FP32 product with the hardware reciprocal (within 1 ulp) floors exactly
    const float inv_need = __builtin_amdgcn_rcpf((float)nneed);
    for (int base = 0; base < ntask; base += 64) {
        const int t = base + lane;
        if (t < ntask) {
            const int im1 = (int)(((float)t + 0.5f) * inv_need);  // trial index - 1
            const int r = t - im1 * nneed;
            float a = 1.f;
#pragma unroll
            for (int k = 1; k <= kLsSpread; ++k)
                if (k <= im1 + 1) a *= kp.inv_beta;
#pragma unroll
            for (int j = 0; j < NM; ++j)
                if (j < n) tt[j] = clampf(fmaf(a, wdt[j * 64 + r], wth[j * 64 + r]), rb->lo[j], rb->hi[j]);
            Target tgL;
            tgL.p = mk(wtg[0 * 64 + r], wtg[1 * 64 + r], wtg[2 * 64 + r]);
            tgL.q = Quat{wtg[3 * 64 + r], wtg[4 * 64 + r], wtg[5 * 64 + r], wtg[6 * 64 + r]};
            wc[im1 * 64 + r] = trial_cost<NM>(rb, n, tgL, tt);
        }
    }
    wave_lds_sync();
    if (!done) {
        int first = -1;
#pragma unroll
        for (int k = kLsSpread - 1; k >= 0; --k)
            if (k < A && wc[k * 64 + myrank] < c0) first = k;
        cnt.pol_trials += first >= 0 ? (uint32_t)(first + 1) : (uint32_t)A;
        if (first >= 0) {
            float a = 1.f;
#pragma unroll
            for (int k = 1; k <= kLsSpread; ++k)
                if (k <= first + 1) a *= kp.inv_beta;
#pragma unroll
            for (int j = 0; j < NM; ++j)
                if (j < n) th[j] = clampf(fmaf(a, wdt[j * 64 + myrank], th[j]), rb->lo[j], rb->hi[j]);
            done = true;
        }
    }
    wave_lds_sync();  // the records are free for the next iteration's writes
}

// ----------------------------------------------------------------------------
// Single-coordinate trial (eq. single-coord): only joint `is` moves, from ts
// to tnew, so the trial pose is the current one turned about that joint's
// axis zs (the same end-effector pose a full FK gives): with u = P_ee - P_is,
// z x u = js and Rodrigues' formula, P' = P_ee + sin(d) (z x u) + (1 - cos d)
// z x (z x u), and q_err' = q_err (x) conj(q_z(d)).  rp0 is the residual
// position t - P_ee, q0 the error quaternion at theta; returns the cost.
// ----------------------------------------------------------------------------
__device__ __forceinline__ float single_trial_cost(Quat q0, V3 zs, V3 js, V3 rp0, float ts, float tnew) {
    const V3 zjs = cross(zs, js);
    float sh, ch;
    sincos_cw(0.5f * (tnew - ts), &sh, &ch);
    const float sd = 2.f * sh * ch, omc = 2.f * sh * sh;
    const V3 rp = axpy(-omc, zjs, axpy(-sd, js, rp0));
    const Quat qn = qmul_conj_axis(q0, zs, ch, sh);
    const float vn = sqrtf(qn.x * qn.x + qn.y * qn.y + qn.z * qn.z);
    const float ph = 2.f * atan2f(vn, fabsf(qn.w));
    return 0.5f * (dot(rp, rp) + ph * ph);
}

// The single-coordinate trials alpha = 1, 1/beta, ..., 1/beta^A spread over
// the wave like the LDS line search: each lane that reaches them writes its
// joint's axis and lever, the residual, its joint value, limits and step to
// the wave's LDS rows (slot = rank among those lanes; 17 + A + 1 <= 26 rows
// of 64, within the line-search rows of any bucket), tasks (lane, alpha) run
// ceil(lanes x (A + 1) / 64) passes, and each lane takes its first trial
// below c0 as the sequential loop does (same values, same choice).
__device__ __forceinline__ void single_coord_lds(const KParams& kp, Quat q0, V3 zs, V3 js, V3 rp0, float ts,
                                                 float los, float his, float step, float c0, float& t_out,
                                                 bool& done, Counters& cnt, float* __restrict__ ws) {
    const int A1 = kp.ls_A + 1;
    const uint64_t need = __ballot(!done);
    if (need == 0ull) return;
    const int lane = (int)(threadIdx.x & 63u);
    const int nneed = __popcll(need);
    const int ntask = nneed * A1;
    const int myrank = __popcll(need & ((1ull << lane) - 1ull));
    float* __restrict__ wr = ws;              // [17][64] by rank
    float* __restrict__ wc = ws + 17 * 64;    // [A + 1][64] by rank
    if (!done) {
        const float rec[17] = {zs.x, zs.y, zs.z, js.x, js.y, js.z, rp0.x, rp0.y, rp0.z,
                               q0.w, q0.x, q0.y, q0.z, ts, los, his, step};
#pragma unroll
        for (int f = 0; f < 17; ++f) wr[f * 64 + myrank] = rec[f];
    }
    wave_lds_sync();
    // (t + 1/2) / nneed is at least 1 / 128 away from an integer and t < 576:
    // its FP32 product with the hardware reciprocal (within 1 ulp) floors exactly
    const float inv_need = __builtin_amdgcn_rcpf((float)nneed);
    for (int base = 0; base < ntask; base += 64) {
        const int t = base + lane;
        if (t < ntask) {
            const int i = (int)(((float)t + 0.5f) * inv_need);  // trial index 0..A
            const int r = t - i * nneed;
            float a = 1.f;
#pragma unroll
            for (int k = 1; k <= kLsSpread; ++k)
                if (k <= i) a *= kp.inv_beta;
            const V3 z = mk(wr[0 * 64 + r], wr[1 * 64 + r], wr[2 * 64 + r]);
            const V3 jv = mk(wr[3 * 64 + r], wr[4 * 64 + r], wr[5 * 64 + r]);
            const V3 r0 = mk(wr[6 * 64 + r], wr[7 * 64 + r], wr[8 * 64 + r]);
            const Quat q{wr[9 * 64 + r], wr[10 * 64 + r], wr[11 * 64 + r], wr[12 * 64 + r]};
            const float tsr = wr[13 * 64 + r];
            const float tnew = clampf(fmaf(a, wr[16 * 64 + r], tsr), wr[14 * 64 + r], wr[15 * 64 + r]);
            wc[i * 64 + r] = single_trial_cost(q, z, jv, r0, tsr, tnew);
        }
    }
    wave_lds_sync();
    if (!done) {
        int first = -1;
#pragma unroll
        for (int k = kLsSpread; k >= 0; --k)
            if (k < A1 && wc[k * 64 + myrank] < c0) first = k;
        cnt.pol_trials += first >= 0 ? (uint32_t)(first + 1) : (uint32_t)A1;
        if (first >= 0) {
            float a = 1.f;
#pragma unroll
            for (int k = 1; k <= kLsSpread; ++k)
                if (k <= first) a *= kp.inv_beta;
            t_out = clampf(fmaf(a, step, ts), los, his);
            done = true;
        }
    }
    wave_lds_sync();  // the rows are free for the next writes
}

// Line-search forms of pj_ik_iter: sequential, spread over the wave through
// shuffles, spread through the wave's LDS records.
constexpr int kLsSeq = 0;
constexpr int kLsShfl = 1;
constexpr int kLsLds = 2;

// ----------------------------------------------------------------------------
// One PJ-IK iteration (Alg. PJ-IK, Sec. IV-B), number `it`, on one seed per
// lane.  LS selects the line-search form above (same results): the spread
// forms run fewer passes; the shuffle form needs more live registers, the
// LDS form needs ls_wave_floats<NM>() floats of LDS per wave at `lsw`.
// LM step: (J^T W^2 J + lam D) dtheta = J^T W^2 e is solved in its 6 x 6
// push-through form dtheta = D^-1 J^T W (W J D^-1 J^T W + lam I)^-1 W e.
// ----------------------------------------------------------------------------
template <int NM, int LS = kLsShfl>
__device__ __forceinline__ void pj_ik_iter(RobotRef rb, int n, const Target& tg, const KParams& kp,
                                           uint32_t m, uint32_t tkey, float* th, bool live, bool& frozen,
                                           Counters& cnt, float* __restrict__ traj, int64_t S, int64_t s, int it,
                                           float& last_ep, float& last_phi, float* __restrict__ lsw = nullptr) {
    V3 Jp[NM], Z[NM];
    float dth[NM], tt[NM];
    const float R = kp.trust_R;
    {
        bool done = true;  // lane needs no further fallback this iteration
        float c0 = 0.f;
        float e6[6], w6[6];
        Quat q0{1.f, 0.f, 0.f, 0.f};  // error quaternion at theta (single-coordinate trials)
        if (!frozen) {
            Frame ee;
            fk_chain<NM, true>(rb, n, th, Jp, Z, ee);
            const Err e = residual(ee, tg);
            last_ep = sqrtf(e.ep2);
            last_phi = e.phi;
            if (e.ep2 < kp.eps_pol2 && e.phi < kp.ups_pol) frozen = true;
            if (live) write_traj<NM>(traj, n, S, s, it, th, last_ep, last_phi);
            if (!frozen) {
                ++cnt.pol_iters;
                done = false;
                c0 = cost_of(e);
                q0 = e.q;
                const V3 om = omega_of(e);
                e6[0] = e.rp.x;
                e6[1] = e.rp.y;
                e6[2] = e.rp.z;
                e6[3] = om.x;
                e6[4] = om.y;
                e6[5] = om.z;
                // Jacobian columns (eq. jacobian); row norms for W
                float rn[6] = {0.f, 0.f, 0.f, 0.f, 0.f, 0.f};
#pragma unroll
                for (int j = 0; j < NM; ++j) {
                    if (j < n) {
                        Jp[j] = cross(Z[j], ee.p - Jp[j]);
                        float c[6];
                        jcol(Jp, Z, j, c);
#pragma unroll
                        for (int r = 0; r < 6; ++r) rn[r] = fmaf(c[r], c[r], rn[r]);
                    }
                }
#pragma unroll
                for (int r = 0; r < 6; ++r)
                    w6[r] = kp.weight_mode == 0 ? div_corr(1.f, fmaxf(sqrtf(rn[r]), 1e-6f)) : 1.f;
                // A = W (sum_j J_j J_j^T / D_j) W + lam I,  D_j = |J_j|^2 (double)
                double A[21];
#pragma unroll
                for (int i = 0; i < 21; ++i) A[i] = 0.0;
#pragma unroll
                for (int j = 0; j < NM; ++j) {
                    if (j < n) {
                        float c[6];
                        jcol(Jp, Z, j, c);
                        double cd[6];
                        double dj = 0.0;
#pragma unroll
                        for (int r = 0; r < 6; ++r) {
                            cd[r] = (double)c[r];
                            dj = fma(cd[r], cd[r], dj);
                        }
                        const double idj = rcp_nr(dj);
#pragma unroll
                        for (int a = 0; a < 6; ++a) {
                            const double ca = cd[a] * idj;
#pragma unroll
                            for (int b = 0; b <= a; ++b) A[tri(a, b)] = fma(ca, cd[b], A[tri(a, b)]);
                        }
                    }
                }
#pragma unroll
                for (int a = 0; a < 6; ++a)
#pragma unroll
                    for (int b = 0; b <= a; ++b)
                        A[tri(a, b)] = A[tri(a, b)] * ((double)w6[a] * (double)w6[b]) + (a == b ? (double)kp.lam : 0.0);
                double inv[6];
                chol6(A, inv);
                double rhs[6], yd[6];
#pragma unroll
                for (int r = 0; r < 6; ++r) rhs[r] = (double)w6[r] * (double)e6[r];
                chol6_solve(A, inv, rhs, yd);
                float y[6];
#pragma unroll
                for (int r = 0; r < 6; ++r) y[r] = (float)(yd[r] * (double)w6[r]);
#pragma unroll
                for (int j = 0; j < NM; ++j) {
                    if (j < n) {
                        float c[6];
                        jcol(Jp, Z, j, c);
                        float dj = 0.f, g = 0.f;
#pragma unroll
                        for (int r = 0; r < 6; ++r) {
                            dj = fmaf(c[r], c[r], dj);
                            g = fmaf(c[r], y[r], g);
                        }
                        dth[j] = clampf(div_corr(g, dj), -R, R);  // trust region, elementwise
                    }
                }
            }
        } else if (live) {
            write_traj<NM>(traj, n, S, s, it, th, last_ep, last_phi);
        }
        // --- backtracking line search (eq. line-search), first decreasing alpha
        if (LS == kLsLds && kp.ls_A <= kLsSpread) {
            line_search_lds<NM>(rb, n, tg, kp, th, dth, tt, c0, done, cnt, lsw);
        } else if (LS == kLsShfl && kp.ls_A <= kLsSpread) {
            line_search_spread<NM>(rb, n, tg, kp, th, dth, tt, c0, done, cnt);
        } else {
            float alpha = 1.f;
            for (int i = 0; i <= kp.ls_A; ++i) {
                if (wave_all(done)) break;
                if (!done) {
#pragma unroll
                    for (int j = 0; j < NM; ++j)
                        if (j < n) tt[j] = clampf(fmaf(alpha, dth[j], th[j]), rb->lo[j], rb->hi[j]);
                    const float c1 = trial_cost<NM>(rb, n, tg, tt);
                    ++cnt.pol_trials;
                    if (c1 < c0) {
#pragma unroll
                        for (int j = 0; j < NM; ++j)
                            if (j < n) th[j] = tt[j];
                        done = true;
                    }
                }
                alpha *= kp.inv_beta;
            }
        }
        // --- dogleg fallback (eq. dogleg)
        if (!wave_all(done)) {
            if (!done) {
                ++cnt.pol_dogleg;
                // g = J^T e, Cauchy length |g|^2 / |J g|^2
                float Jg[6] = {0.f, 0.f, 0.f, 0.f, 0.f, 0.f};
                float gg = 0.f;
#pragma unroll
                for (int j = 0; j < NM; ++j) {
                    if (j < n) {
                        float c[6];
                        jcol(Jp, Z, j, c);
                        float g = 0.f;
#pragma unroll
                        for (int r = 0; r < 6; ++r) g = fmaf(c[r], e6[r], g);
                        dth[j] = g;
                        gg = fmaf(g, g, gg);
#pragma unroll
                        for (int r = 0; r < 6; ++r) Jg[r] = fmaf(c[r], g, Jg[r]);
                    }
                }
                float jgjg = 0.f;
#pragma unroll
                for (int r = 0; r < 6; ++r) jgjg = fmaf(Jg[r], Jg[r], jgjg);
                const float ac = jgjg > 0.f ? gg / jgjg : 0.f;
                // Gauss-Newton: J^T (J J^T + lambda_gn I)^-1 e (system in double)
                double A[21];
#pragma unroll
                for (int i = 0; i < 21; ++i) A[i] = 0.0;
#pragma unroll
                for (int j = 0; j < NM; ++j) {
                    if (j < n) {
                        float c[6];
                        jcol(Jp, Z, j, c);
#pragma unroll
                        for (int a = 0; a < 6; ++a)
#pragma unroll
                            for (int b = 0; b <= a; ++b)
                                A[tri(a, b)] = fma((double)c[a], (double)c[b], A[tri(a, b)]);
                    }
                }
#pragma unroll
                for (int a = 0; a < 6; ++a) A[tri(a, a)] += (double)kp.lambda_gn;
                double inv[6];
                chol6(A, inv);
                double ed[6], yd[6];
#pragma unroll
                for (int r = 0; r < 6; ++r) ed[r] = (double)e6[r];
                chol6_solve(A, inv, ed, yd);
                float y[6];
#pragma unroll
                for (int r = 0; r < 6; ++r) y[r] = (float)yd[r];
                float ngn2 = 0.f, ngd2 = 0.f;
#pragma unroll
                for (int j = 0; j < NM; ++j) {
                    if (j < n) {
                        float c[6];
                        jcol(Jp, Z, j, c);
                        float g = 0.f;
#pragma unroll
                        for (int r = 0; r < 6; ++r) g = fmaf(c[r], y[r], g);
                        tt[j] = g;              // GN step
                        dth[j] = ac * dth[j];   // GD step
                        ngn2 = fmaf(g, g, ngn2);
                        ngd2 = fmaf(dth[j], dth[j], ngd2);
                    }
                }
                const float ngn = sqrtf(ngn2), ngd = sqrtf(ngd2);
                // blend: GN if |GN| <= R; GD scaled to R if |GD| >= R; else the
                // point GN + tau (GD - GN) with norm R and the smallest tau, written
                // as GD + s (GN - GD), s = 1 - tau: the root in s keeps full
                // relative precision when |GN| >> R (near singular J).
                float s_gn = 0.f, scale_gd = 1.f;
                bool use_gn = false;
                if (ngn <= R) {
                    use_gn = true;
                } else if (ngd >= R) {
                    scale_gd = R / ngd;
                } else {
                    float aa = 0.f, bb = 0.f;
#pragma unroll
                    for (int j = 0; j < NM; ++j) {
                        if (j < n) {
                            const float dj = tt[j] - dth[j];
                            aa = fmaf(dj, dj, aa);
                            bb = fmaf(dth[j], dj, bb);
                        }
                    }
                    // aa s^2 + 2 bb s + (|GD|^2 - R^2) = 0, positive root
                    const float cc = ngd2 - R * R;  // < 0
                    const float disc = sqrtf(fmaxf(bb * bb - aa * cc, 0.f));
                    s_gn = bb >= 0.f ? (-cc) / (bb + disc) : (disc - bb) / fmaxf(aa, 1e-30f);
                    s_gn = clampf(s_gn, 0.f, 1.f);
                }
#pragma unroll
                for (int j = 0; j < NM; ++j) {
                    if (j < n) {
                        const float st = use_gn ? tt[j] : fmaf(s_gn, tt[j] - dth[j], scale_gd * dth[j]);
                        tt[j] = clampf(th[j] + st, rb->lo[j], rb->hi[j]);
                    }
                }
                const float c1 = trial_cost<NM>(rb, n, tg, tt);
                ++cnt.pol_trials;
                if (c1 < c0) {
#pragma unroll
                    for (int j = 0; j < NM; ++j)
                        if (j < n) th[j] = tt[j];
                    done = true;
                }
            }
        }
        // --- single-coordinate fallback (eq. single-coord)
        if (!wave_all(done)) {
            int is = 0;
            float step = 0.f;
            if (!done) {
                ++cnt.pol_single;
                float best = -1.f, gbest = 0.f, hbest = 1.f;
#pragma unroll
                for (int j = 0; j < NM; ++j) {
                    if (j < n) {
                        float c[6];
                        jcol(Jp, Z, j, c);
                        float g = 0.f, h = 0.f;
#pragma unroll
                        for (int r = 0; r < 6; ++r) {
                            const float w2 = w6[r] * w6[r];
                            g = fmaf(c[r] * w2, e6[r], g);
                            h = fmaf(c[r] * w2, c[r], h);
                        }
                        if (fabsf(g) > best) {
                            best = fabsf(g);
                            gbest = g;
                            hbest = h;
                            is = j;
                        }
                    }
                }
                step = hbest > 0.f ? clampf(gbest / hbest, -R, R) : 0.f;
            }
            // trials by rigid rotation about joint `is` (single_trial_cost)
            V3 zs = Z[0], js = Jp[0];
            float ts = th[0], los = rb->lo[0], his = rb->hi[0];
#pragma unroll
            for (int j = 0; j < NM; ++j) {
                if (j < n && j == is) {
                    zs = Z[j];
                    js = Jp[j];
                    ts = th[j];
                    los = rb->lo[j];
                    his = rb->hi[j];
                }
            }
            const V3 rp0 = mk(e6[0], e6[1], e6[2]);
            if (LS == kLsLds && kp.ls_A <= kLsSpread) {
                float tnew = ts;
                const bool was = done;
                single_coord_lds(kp, q0, zs, js, rp0, ts, los, his, step, c0, tnew, done, cnt, lsw);
                if (done && !was) {
#pragma unroll
                    for (int j = 0; j < NM; ++j)
                        if (j < n && j == is) th[j] = tnew;
                }
            } else {
                float alpha2 = 1.f;
                for (int i = 0; i <= kp.ls_A; ++i) {
                    if (wave_all(done)) break;
                    if (!done) {
                        const float tnew = clampf(fmaf(alpha2, step, ts), los, his);
                        const float c1 = single_trial_cost(q0, zs, js, rp0, ts, tnew);
                        ++cnt.pol_trials;
                        if (c1 < c0) {
#pragma unroll
                            for (int j = 0; j < NM; ++j)
                                if (j < n && j == is) th[j] = tnew;
                            done = true;
                        }
                    }
                    alpha2 *= kp.inv_beta;
                }
            }
        }
        // --- random perturbation when every step failed
        if (LS == kLsLds) {
            perturb_spread<NM>(rb, n, th, !done, kp.seed, m, tkey, STAGE_POLISH, (uint32_t)it, kp.mu, kp.sigma, lsw);
        } else if (!done) {
            perturb<NM>(rb, n, th, kp.seed, m, tkey, STAGE_POLISH, (uint32_t)it, kp.mu, kp.sigma);
        }
        if (!done) ++cnt.pol_perturb;
    }
}

// Iterations [k0, k1) of PJ-IK on one seed per lane; out_err is the residual
// at the configuration the last iteration produced (when want_err).
template <int NM, int LS = kLsShfl>
__device__ __forceinline__ void pj_ik(RobotRef rb, int n, const Target& tg, const KParams& kp,
                                      uint32_t m, uint32_t tkey, float* th, bool live, bool& frozen,
                                      Counters& cnt, float* __restrict__ traj, int64_t S, int64_t s, int k0,
                                      int k1, Err& out_err, bool want_err = true, float* __restrict__ lsw = nullptr) {
    float last_ep = 0.f, last_phi = 0.f;
    for (int it = k0; it < k1; ++it) {
        if (wave_all(frozen) && !traj) break;
        pj_ik_iter<NM, LS>(rb, n, tg, kp, m, tkey, th, live, frozen, cnt, traj, S, s, it, last_ep, last_phi, lsw);
    }
    if (!want_err) return;  // the caller continues this seed in a later call
    Frame ee;
    V3 Pd[1], Zd[1];
    fk_chain<NM, false>(rb, n, th, Pd, Zd, ee);
    out_err = residual(ee, tg);
    if (live) write_traj<NM>(traj, n, S, s, k1, th, sqrtf(out_err.ep2), out_err.phi);
}

// ----------------------------------------------------------------------------
// lane -> (seed slot, target, seed index within target)
// ----------------------------------------------------------------------------
__device__ __forceinline__ int32_t last_le(const int64_t* __restrict__ a, int32_t count, int64_t v) {
    // largest i in [0, count) with a[i] <= v (a non-decreasing, a[0] <= v)
    int32_t lo = 0, hi = count;
    while (hi - lo > 1) {
        const int32_t mid = (lo + hi) >> 1;
        if (a[mid] <= v)
            lo = mid;
        else
            hi = mid;
    }
    return lo;
}

struct Slot {
    int64_t s;      // seed slot
    int32_t t;      // target id
    uint32_t m;     // seed index within the target
    uint32_t tkey;  // Philox target key
};

__device__ __forceinline__ Slot map_lane(const SeedMap& mp, int64_t v) {
    Slot r;
    r.s = mp.base + v;
    const int32_t b = mp.tb + last_le(mp.voffs + mp.tb, mp.te - mp.tb, r.s);
    r.t = mp.tperm ? mp.tperm[b] : b;
    r.m = (uint32_t)(r.s - mp.voffs[b]);
    r.tkey = mp.tkeys ? mp.tkeys[r.t] : (uint32_t)r.t;
    return r;
}

}  // namespace hjcd
