// FP64 CPU oracle for the batched HJCD-IK solve.  TEST INFRASTRUCTURE ONLY:
// loaded by the test suite, the smoke check and the benchmark's CPU-baseline
// leg, never by the product path.  Plain, slow and step by step: every
// candidate is scored with a full forward-kinematics pass, every linear system
// is the n x n system the paper prints, every collision pair is tested.
// Citations refer to sections / equations / algorithms of arXiv 2510.07514.
#include "hjcd_oracle.h"

#include <algorithm>
#include <atomic>
#include <cmath>
#include <cstring>
#include <limits>
#include <mutex>
#include <thread>
#include <vector>

namespace {

const double kPi = 3.14159265358979323846;
const double kInf = std::numeric_limits<double>::infinity();

// ---------------------------------------------------------------------------
// Operation counts (instrumentation; they never change a result).  Every
// helper below adds the floating-point operations its own body executes to
// the counter of the unit of work being executed: add (add, subtract), mul,
// div, sqrt, and transcendental calls (sin, cos, atan2, acos, log, pow).
// Comparisons, min / max, sign flips and copies are not counted.
// ---------------------------------------------------------------------------
struct Ops {
    uint64_t add, mul, div, sqrt, trans, units;
};
thread_local Ops tl_ops[OR_OPS_NCAT];
thread_local int tl_cat = OR_OPS_EVAL;
std::mutex g_ops_mu;
Ops g_ops[OR_OPS_NCAT];

inline void ops(uint64_t add, uint64_t mul, uint64_t div = 0, uint64_t sq = 0, uint64_t tr = 0) {
    Ops& o = tl_ops[tl_cat];
    o.add += add;
    o.mul += mul;
    o.div += div;
    o.sqrt += sq;
    o.trans += tr;
}

// The operations executed while a Unit is alive go to category c, which
// counts one unit more.
struct Unit {
    int prev;
    explicit Unit(int c) : prev(tl_cat) {
        tl_cat = c;
        tl_ops[c].units++;
    }
    ~Unit() { tl_cat = prev; }
};

// Moves this thread's counts into the process totals.
void flush_ops() {
    std::lock_guard<std::mutex> lk(g_ops_mu);
    for (int c = 0; c < OR_OPS_NCAT; ++c) {
        Ops& t = tl_ops[c];
        g_ops[c].add += t.add;
        g_ops[c].mul += t.mul;
        g_ops[c].div += t.div;
        g_ops[c].sqrt += t.sqrt;
        g_ops[c].trans += t.trans;
        g_ops[c].units += t.units;
        t = Ops{0, 0, 0, 0, 0, 0};
    }
}

// ---------------------------------------------------------------------------
// Rigid transforms (4x4 homogeneous, last row 0 0 0 1), 3-vectors
// ---------------------------------------------------------------------------
struct H4 {
    double m[4][4];
};

H4 eye4() {
    H4 t;
    for (int i = 0; i < 4; ++i)
        for (int j = 0; j < 4; ++j) t.m[i][j] = (i == j) ? 1.0 : 0.0;
    return t;
}

// a b for rigid a, b: rotation rows times rotation columns, translation
// R_a p_b + p_a (the bottom row stays 0 0 0 1).
H4 mul(const H4& a, const H4& b) {
    H4 c = eye4();
    for (int i = 0; i < 3; ++i) {
        for (int j = 0; j < 3; ++j) c.m[i][j] = a.m[i][0] * b.m[0][j] + a.m[i][1] * b.m[1][j] + a.m[i][2] * b.m[2][j];
        c.m[i][3] = a.m[i][3] + a.m[i][0] * b.m[0][3] + a.m[i][1] * b.m[1][3] + a.m[i][2] * b.m[2][3];
    }
    ops(27, 36);
    return c;
}

struct V3 {
    double x, y, z;
};
V3 v3(double x, double y, double z) { return V3{x, y, z}; }
V3 operator+(V3 a, V3 b) {
    ops(3, 0);
    return v3(a.x + b.x, a.y + b.y, a.z + b.z);
}
V3 operator-(V3 a, V3 b) {
    ops(3, 0);
    return v3(a.x - b.x, a.y - b.y, a.z - b.z);
}
V3 operator*(double s, V3 a) {
    ops(0, 3);
    return v3(s * a.x, s * a.y, s * a.z);
}
V3 neg(V3 a) { return v3(-a.x, -a.y, -a.z); }
double dot(V3 a, V3 b) {
    ops(2, 3);
    return a.x * b.x + a.y * b.y + a.z * b.z;
}
V3 cross(V3 a, V3 b) {
    ops(3, 6);
    return v3(a.y * b.z - a.z * b.y, a.z * b.x - a.x * b.z, a.x * b.y - a.y * b.x);
}
double norm(V3 a) {
    ops(0, 0, 0, 1);
    return std::sqrt(dot(a, a));
}

// Quaternion (w, x, y, z), Hamilton convention.
struct Q4 {
    double w;
    V3 v;
};
Q4 qmul(Q4 a, Q4 b) {
    // (a0, a)(b0, b) = (a0 b0 - a.b, a0 b + b0 a + a x b)
    ops(1, 1);
    return Q4{a.w * b.w - dot(a.v, b.v), a.w * b.v + b.w * a.v + cross(a.v, b.v)};
}
Q4 qconj(Q4 a) { return Q4{a.w, neg(a.v)}; }

// Shepperd (1978): pick the largest of trace, R00, R11, R22 for the division.
Q4 quat_from_R(const double R[3][3]) {
    double tr = R[0][0] + R[1][1] + R[2][2];
    Q4 q;
    if (tr >= R[0][0] && tr >= R[1][1] && tr >= R[2][2]) {
        double s = 2.0 * std::sqrt(1.0 + tr);
        q.w = 0.25 * s;
        q.v = v3((R[2][1] - R[1][2]) / s, (R[0][2] - R[2][0]) / s, (R[1][0] - R[0][1]) / s);
        ops(2 + 1 + 3, 2, 3, 1);
    } else if (R[0][0] >= R[1][1] && R[0][0] >= R[2][2]) {
        double s = 2.0 * std::sqrt(1.0 + R[0][0] - R[1][1] - R[2][2]);
        q.w = (R[2][1] - R[1][2]) / s;
        q.v = v3(0.25 * s, (R[0][1] + R[1][0]) / s, (R[0][2] + R[2][0]) / s);
        ops(2 + 3 + 3, 2, 3, 1);
    } else if (R[1][1] >= R[2][2]) {
        double s = 2.0 * std::sqrt(1.0 - R[0][0] + R[1][1] - R[2][2]);
        q.w = (R[0][2] - R[2][0]) / s;
        q.v = v3((R[0][1] + R[1][0]) / s, 0.25 * s, (R[1][2] + R[2][1]) / s);
        ops(2 + 3 + 3, 2, 3, 1);
    } else {
        double s = 2.0 * std::sqrt(1.0 - R[0][0] - R[1][1] + R[2][2]);
        q.w = (R[1][0] - R[0][1]) / s;
        q.v = v3((R[0][2] + R[2][0]) / s, (R[1][2] + R[2][1]) / s, 0.25 * s);
        ops(2 + 3 + 3, 2, 3, 1);
    }
    if (q.w < 0.0) q = Q4{-q.w, neg(q.v)};
    return q;
}

// ---------------------------------------------------------------------------
// Robot, FK (eq. fk) and geometric Jacobian (eq. jacobian)
// ---------------------------------------------------------------------------
struct Robot {
    int n = 0, conv = 0;
    double a[OR_MAX_DOF], d[OR_MAX_DOF], alpha[OR_MAX_DOF], off[OR_MAX_DOF];
    double ca[OR_MAX_DOF], sa[OR_MAX_DOF];  // cos / sin of alpha (constants of the chain)
    double lo[OR_MAX_DOF], hi[OR_MAX_DOF];
    H4 tool;
    std::vector<int> sph_link;
    std::vector<double> sph;  // x y z r
    int gap = 0;
};

bool load_robot(const or_robot* in, Robot& r) {
    if (!in || in->dof < 1 || in->dof > OR_MAX_DOF) return false;
    if (in->convention != 0 && in->convention != 1) return false;
    r.n = in->dof;
    r.conv = in->convention;
    for (int i = 0; i < r.n; ++i) {
        r.a[i] = in->a[i];
        r.d[i] = in->d[i];
        r.alpha[i] = in->alpha[i];
        r.ca[i] = std::cos(r.alpha[i]);
        r.sa[i] = std::sin(r.alpha[i]);
        r.off[i] = in->offset[i];
        r.lo[i] = in->q_min[i];
        r.hi[i] = in->q_max[i];
        if (!(r.lo[i] <= r.hi[i])) return false;
    }
    r.tool = eye4();
    if (in->tool)
        for (int i = 0; i < 4; ++i)
            for (int j = 0; j < 4; ++j) r.tool.m[i][j] = in->tool[4 * i + j];
    r.sph_link.assign(in->sphere_link, in->sphere_link + in->n_spheres);
    r.sph.assign(in->sphere_xyzr, in->sphere_xyzr + 4 * in->n_spheres);
    for (int l : r.sph_link)
        if (l < 0 || l > r.n) return false;
    r.gap = in->min_link_gap;
    return true;
}

struct FK {
    H4 link[OR_MAX_DOF + 1];  // link l frame, link 0 = base = identity
    V3 P[OR_MAX_DOF];         // joint origins
    V3 z[OR_MAX_DOF];         // joint unit axes
    V3 p_ee;
    double R_ee[3][3];
};

V3 col(const H4& t, int c) { return v3(t.m[0][c], t.m[1][c], t.m[2][c]); }

// Modified DH (Craig): {i-1}T_i = Rx(alpha_i) Tx(a_i) Rz(theta_i + o_i) Tz(d_i);
// joint i turns about z of frame i.  Standard DH:
// {i-1}T_i = Rz(theta_i + o_i) Tz(d_i) Tx(a_i) Rx(alpha_i); joint i turns about
// z of frame i-1.  Each link transform is the product of those four
// elementary motions written out (c = cos, s = sin, t = theta + offset):
//   modified: R = [[ct, -st, 0], [ca st, ca ct, -sa], [sa st, sa ct, ca]],
//             p = (a, -sa d, ca d)
//   standard: R = [[ct, -st ca, st sa], [st, ct ca, -ct sa], [0, sa, ca]],
//             p = (a ct, a st, d)
// End effector = T_0n * tool.
H4 dh_link(const Robot& r, int i, double theta) {
    const double t = theta + r.off[i];
    const double ct = std::cos(t), st = std::sin(t);
    const double ca = r.ca[i], sa = r.sa[i];
    ops(1, 6, 0, 0, 2);
    H4 L = eye4();
    if (r.conv == 0) {
        L.m[0][0] = ct;
        L.m[0][1] = -st;
        L.m[0][2] = 0.0;
        L.m[1][0] = ca * st;
        L.m[1][1] = ca * ct;
        L.m[1][2] = -sa;
        L.m[2][0] = sa * st;
        L.m[2][1] = sa * ct;
        L.m[2][2] = ca;
        L.m[0][3] = r.a[i];
        L.m[1][3] = -sa * r.d[i];
        L.m[2][3] = ca * r.d[i];
    } else {
        L.m[0][0] = ct;
        L.m[0][1] = -st * ca;
        L.m[0][2] = st * sa;
        L.m[1][0] = st;
        L.m[1][1] = ct * ca;
        L.m[1][2] = -ct * sa;
        L.m[2][0] = 0.0;
        L.m[2][1] = sa;
        L.m[2][2] = ca;
        L.m[0][3] = r.a[i] * ct;
        L.m[1][3] = r.a[i] * st;
        L.m[2][3] = r.d[i];
    }
    return L;
}

void fk(const Robot& r, const double* th, FK& o) {
    H4 T = eye4();
    o.link[0] = T;
    for (int i = 0; i < r.n; ++i) {
        if (r.conv == 0) {
            T = mul(T, dh_link(r, i, th[i]));
            o.P[i] = col(T, 3);
            o.z[i] = col(T, 2);
        } else {
            o.P[i] = col(T, 3);
            o.z[i] = col(T, 2);
            T = mul(T, dh_link(r, i, th[i]));
        }
        o.link[i + 1] = T;
    }
    H4 E = mul(T, r.tool);
    o.p_ee = col(E, 3);
    for (int i = 0; i < 3; ++i)
        for (int j = 0; j < 3; ++j) o.R_ee[i][j] = E.m[i][j];
}

// Column i of eq. (jacobian): [z_i x (P_ee - P_i); z_i].  J is row-major 6 x n.
void jacobian(const Robot& r, const FK& f, double* J) {
    for (int i = 0; i < r.n; ++i) {
        V3 lin = cross(f.z[i], f.p_ee - f.P[i]);
        J[0 * r.n + i] = lin.x;
        J[1 * r.n + i] = lin.y;
        J[2 * r.n + i] = lin.z;
        J[3 * r.n + i] = f.z[i].x;
        J[4 * r.n + i] = f.z[i].y;
        J[5 * r.n + i] = f.z[i].z;
    }
}

// ---------------------------------------------------------------------------
// Residual: eq. (task_residual), eq. (quat_diff), eq. (angle_axis)
// ---------------------------------------------------------------------------
struct Target {
    V3 p;
    Q4 q;  // unit
};

Target load_target(const double* t7) {
    Target t;
    t.p = v3(t7[0], t7[1], t7[2]);
    double n = std::sqrt(t7[3] * t7[3] + t7[4] * t7[4] + t7[5] * t7[5] + t7[6] * t7[6]);
    t.q = Q4{t7[3] / n, v3(t7[4] / n, t7[5] / n, t7[6] / n)};
    return t;
}

struct Res {
    V3 rp;       // P_t - P_ee
    V3 omega;    // orientation residual
    double phi;  // rotation angle of q_err in [0, pi]
    V3 ahat;     // unit rotation axis (0 when phi = 0)
    V3 v;        // vector part of the canonical q_err (|v| = sin(phi/2))
    double ep, cost;
};

// Switches the category that operations are counted in (no unit counted).
struct Scope {
    int prev;
    explicit Scope(int c) : prev(tl_cat) { tl_cat = c; }
    ~Scope() { tl_cat = prev; }
};

// q_err = q_t (x) q_e^-1 is taken with w >= 0 so that the printed formula
// 2 atan2(|v|, |w|) v/|v| points along the short rotation (reading of eq.
// quat_diff); phi and a_hat of eq. (angle_axis) then follow from the same
// canonical quaternion, phi in [0, pi].
Res residual(const Target& tg, const V3& p_ee, const double R[3][3]) {
    Res r;
    r.rp = tg.p - p_ee;
    Q4 qe = quat_from_R(R);
    Q4 qerr = qmul(tg.q, qconj(qe));
    if (qerr.w < 0.0) qerr = Q4{-qerr.w, neg(qerr.v)};
    double s = norm(qerr.v);
    r.phi = 2.0 * std::atan2(s, qerr.w);
    ops(0, 1, 0, 0, 1);
    r.v = qerr.v;
    if (s > 1e-20) {
        r.omega = (r.phi / s) * qerr.v;
        r.ahat = (1.0 / s) * qerr.v;
        ops(0, 0, 2);
    } else {
        r.omega = (2.0 / qerr.w) * qerr.v;
        r.ahat = v3(0, 0, 0);
        ops(0, 0, 1);
    }
    r.ep = norm(r.rp);
    r.cost = 0.5 * (dot(r.rp, r.rp) + dot(r.omega, r.omega));
    ops(1, 1);
    return r;
}

Res eval(const Robot& rb, const Target& tg, const double* th) {
    FK f;
    fk(rb, th, f);
    return residual(tg, f.p_ee, f.R_ee);
}

double clip(double x, double lo, double hi) { return std::min(std::max(x, lo), hi); }

// ---------------------------------------------------------------------------
// Philox4x32-10 (Salmon, Moraes, Dror, Shaw, SC'11) and normal draws
// ---------------------------------------------------------------------------
void philox(const uint32_t ctr_in[4], const uint32_t key_in[2], uint32_t out[4]) {
    uint32_t c0 = ctr_in[0], c1 = ctr_in[1], c2 = ctr_in[2], c3 = ctr_in[3];
    uint32_t k0 = key_in[0], k1 = key_in[1];
    for (int round = 0; round < 10; ++round) {
        if (round > 0) {
            k0 += 0x9E3779B9u;
            k1 += 0xBB67AE85u;
        }
        uint64_t p0 = (uint64_t)0xD2511F53u * (uint64_t)c0;
        uint64_t p1 = (uint64_t)0xCD9E8D57u * (uint64_t)c2;
        uint32_t hi0 = (uint32_t)(p0 >> 32), lo0 = (uint32_t)p0;
        uint32_t hi1 = (uint32_t)(p1 >> 32), lo1 = (uint32_t)p1;
        c0 = hi1 ^ c1 ^ k0;
        c1 = lo1;
        c2 = hi0 ^ c3 ^ k1;
        c3 = lo0;
    }
    out[0] = c0;
    out[1] = c1;
    out[2] = c2;
    out[3] = c3;
}

enum { ST_INIT = 0, ST_CD = 1, ST_RESAMPLE = 2, ST_POLISH = 3, ST_WARM = 4 };

// The top 24 bits of a word give a uniform in (0, 1) that is exact in both
// single and double precision.
double uni24(uint32_t x) {
    ops(1, 1);
    return ((double)(x >> 8) + 0.5) * (1.0 / 16777216.0);
}

void draw_block(uint64_t seed, uint32_t m, uint32_t tkey, uint32_t stage, uint32_t iter,
                uint32_t block, uint32_t out[4]) {
    uint32_t ctr[4] = {m, tkey, (stage << 24) | (iter & 0xFFFFFFu), block};
    uint32_t key[2] = {(uint32_t)(seed & 0xFFFFFFFFu), (uint32_t)(seed >> 32)};
    philox(ctr, key, out);
}

// Joint j uses word pair (2p, 2p+1), p = (j % 4) / 2, of block j / 4;
// Box-Muller: cos branch for even j, sin branch for odd j.
void normals(uint64_t seed, uint32_t m, uint32_t tkey, uint32_t stage, uint32_t iter, int n,
             double* z) {
    for (int j = 0; j < n; ++j) {
        uint32_t x[4];
        draw_block(seed, m, tkey, stage, iter, (uint32_t)(j / 4), x);
        int p = (j % 4) / 2;
        double u1 = uni24(x[2 * p]), u2 = uni24(x[2 * p + 1]);
        double rad = std::sqrt(-2.0 * std::log(u1));
        z[j] = (j % 2 == 0) ? rad * std::cos(2.0 * kPi * u2) : rad * std::sin(2.0 * kPi * u2);
        ops(0, 3, 0, 1, 2);
    }
}

void uniform_seed(const Robot& rb, uint64_t seed, uint32_t m, uint32_t tkey, double* th) {
    for (int j = 0; j < rb.n; ++j) {
        uint32_t x[4];
        draw_block(seed, m, tkey, ST_INIT, 0, (uint32_t)(j / 4), x);
        th[j] = rb.lo[j] + (rb.hi[j] - rb.lo[j]) * uni24(x[j % 4]);
        ops(2, 1);
    }
}

// theta <- clip(theta + mu + sigma z): the N(mu, Sigma) move of Alg. PO-CCD /
// Alg. PJ-IK / Alg. HJCD-IK with Sigma = sigma^2 I, projected onto the limits.
void perturb(const Robot& rb, const or_params& p, uint32_t m, uint32_t tkey, uint32_t stage,
             uint32_t iter, double* th) {
    double z[OR_MAX_DOF];
    normals(p.rng_seed, m, tkey, stage, iter, rb.n, z);
    for (int j = 0; j < rb.n; ++j) th[j] = clip(th[j] + p.mu + p.sigma * z[j], rb.lo[j], rb.hi[j]);
    ops(2 * rb.n, rb.n);
}

// ---------------------------------------------------------------------------
// Decision margins: the distance (in m or rad) of a discrete decision from
// its switching point.  They do not change the computation; the parity tests
// use them to stop comparing a seed after a near-tie.
// ---------------------------------------------------------------------------
struct Margin {
    double v = kInf;
    void add(double m) { v = std::min(v, m); }
};

// margin of (A && B) given the two conditions and their own margins
double and_margin(bool a, double ma, bool b, double mb) {
    if (a && b) return std::min(ma, mb);
    if (a && !b) return mb;
    if (!a && b) return ma;
    return std::max(ma, mb);
}
// margin of (A || B)
double or_margin(bool a, double ma, bool b, double mb) {
    if (!a && !b) return std::min(ma, mb);
    if (a && !b) return ma;
    if (!a && b) return mb;
    return std::max(ma, mb);
}

void write_row(double* traj, int row, int n, const double* th, const Res& r) {
    if (!traj) return;
    double* o = traj + (size_t)row * (n + 2);
    for (int j = 0; j < n; ++j) o[j] = th[j];
    o[n] = r.ep;
    o[n + 1] = r.phi;
}

// Per-joint candidates of one PO-CCD iteration k at theta (frames f, residual
// r): clipped position steps dp, orientation steps dor, and their scores
// sp = |r_p|^2 and so = |omega|^2 after moving that joint alone.
// v + (+-a, +-a, +-a) with signs from a xorshift sequence keyed by `key`
// (shadow runs only).
V3 jittered(V3 v, double a, uint64_t key) {
    uint64_t x = key * 0x9E3779B97F4A7C15ull + 0x632BE59BD9B4E019ull;
    double sg[3];
    for (int i = 0; i < 3; ++i) {
        x ^= x << 13;
        x ^= x >> 7;
        x ^= x << 17;
        sg[i] = (x >> 11) & 1 ? a : -a;
    }
    return v3(v.x + sg[0], v.y + sg[1], v.z + sg[2]);
}

void cd_candidates(const Robot& rb, const Target& tg, const or_params& p, const double* th, int k,
                   const FK& f, const Res& r, double* dp, double* dor, double* sp, double* so,
                   Margin& mg, double harm) {
    const int n = rb.n;
    // Annealed orientation factor delta(k) of eq. (ori_update).
    double delta = std::max(p.delta_min, p.delta0 * std::pow(p.delta_decay, (double)k));
    ops(0, 1, 0, 0, 1);
    for (int j = 0; j < n; ++j) {
        // Position candidate: eq. (vec_proj) projects u = P_ee - P_j and
        // v = P_t - P_j onto the plane normal to the joint axis; the angle
        // between the projections is eq. (theta_proj).  The sign that turns
        // u_proj onto v_proj comes from z . (u_proj x v_proj).
        V3 z = f.z[j];
        V3 u = f.p_ee - f.P[j];
        V3 v = tg.p - f.P[j];
        V3 up = u - dot(u, z) * z;
        V3 vp = v - dot(v, z) * z;
        if (p.shadow) {
            // shadow run: the projections carry single-precision-sized
            // absolute errors (positions of order 1 m)
            Scope instr(OR_OPS_INSTR);
            up = jittered(up, 1.2e-7, p.shadow * 7919ull + (uint64_t)(k * 64 + j) * 2);
            vp = jittered(vp, 1.2e-7, p.shadow * 7919ull + (uint64_t)(k * 64 + j) * 2 + 1);
        }
        double du = norm(up), dv = norm(vp);
        double d = 0.0;
        if (du >= p.proj_eps && dv >= p.proj_eps) {
            V3 uh = (1.0 / du) * up, vh = (1.0 / dv) * vp;
            double c = clip(dot(uh, vh), -1.0, 1.0);
            double mag = std::acos(c);
            const double sn = dot(z, cross(uh, vh));
            double sgn = sn >= 0.0 ? 1.0 : -1.0;
            d = sgn * mag;
            ops(0, 1, 2, 0, 1);
            // the turning direction is a decision when the step is not ~0
            if (mag > harm) mg.add(std::fabs(sn));
        }
        mg.add(std::fabs(du - p.proj_eps));
        mg.add(std::fabs(dv - p.proj_eps));
        dp[j] = clip(th[j] + d, rb.lo[j], rb.hi[j]) - th[j];
        ops(2, 0);

        // Orientation candidate, eq. (ori_update): delta(k) sgn(a_hat . r_j) phi,
        // sgn(0) = 0.
        double az = dot(r.ahat, z);
        double sg = az > 0.0 ? 1.0 : (az < 0.0 ? -1.0 : 0.0);
        dor[j] = clip(th[j] + delta * sg * r.phi, rb.lo[j], rb.hi[j]) - th[j];
        ops(2, 2);
        if (2.0 * delta * r.phi > harm) {
            Scope instr(OR_OPS_INSTR);
            mg.add(std::fabs(dot(r.v, z)));
        }

        // Scores: full FK at the moved configuration.
        double tt[OR_MAX_DOF];
        std::memcpy(tt, th, sizeof(double) * n);
        tt[j] = th[j] + dp[j];
        Res rp_ = eval(rb, tg, tt);
        sp[j] = dot(rp_.rp, rp_.rp);
        tt[j] = th[j] + dor[j];
        Res ro_ = eval(rb, tg, tt);
        so[j] = dot(ro_.omega, ro_.omega);
        ops(2, 0);
    }
}

// ---------------------------------------------------------------------------
// PO-CCD on one seed (Alg. PO-CCD, Sec. III, Sec. IV-A)
// ---------------------------------------------------------------------------
void po_ccd(const Robot& rb, const Target& tg, const or_params& p, uint32_t m, uint32_t tkey,
            double* th, double* traj, double* margin, or_stage_stats& st, double harm) {
    const int n = rb.n;
    const int K = p.cd_sweeps;
    st = or_stage_stats{0, -1, 0, 0, 0, 0, 0};
    for (int k = 0; k < K; ++k) {
        FK f;
        Res r;
        {
            Unit u(OR_OPS_EVAL);
            fk(rb, th, f);
            r = residual(tg, f.p_ee, f.R_ee);
        }
        write_row(traj, k, n, th, r);
        Margin mg;

        // Coarse exit (end-of-iteration test of Alg. PO-CCD, evaluated on the
        // configuration the previous iteration produced).
        bool ca = r.ep < p.eps_cd, cb = r.phi < p.nu_cd;
        mg.add(and_margin(ca, std::fabs(r.ep - p.eps_cd), cb, std::fabs(r.phi - p.nu_cd)));
        if (ca && cb) {
            st.frozen_at = k;
            if (margin) margin[k] = mg.v;
            for (int kk = k + 1; kk <= K; ++kk) write_row(traj, kk, n, th, r);
            for (int kk = k + 1; kk < K; ++kk)
                if (margin) margin[kk] = kInf;
            return;
        }

        Unit u(OR_OPS_CD_ITER);
        double dp[OR_MAX_DOF], dor[OR_MAX_DOF], sp[OR_MAX_DOF], so[OR_MAX_DOF];
        cd_candidates(rb, tg, p, th, k, f, r, dp, dor, sp, so, mg, harm);

        // Greedy picks: the lowest joint whose score (|r_p| for position, |omega|
        // for orientation) lies within tie_eps of the best one.
        double ds[OR_MAX_DOF], os[OR_MAX_DOF];
        double dmin = kInf, omin = kInf;
        int jp0 = 0, jo0 = 0;  // strict argmins (lowest index), for the tie statistic
        for (int j = 0; j < n; ++j) {
            ds[j] = std::sqrt(sp[j]);
            os[j] = std::sqrt(so[j]);
            if (ds[j] < dmin) {
                dmin = ds[j];
                jp0 = j;
            }
            if (os[j] < omin) {
                omin = os[j];
                jo0 = j;
            }
        }
        const double dlim = dmin + p.tie_eps, olim = omin + p.tie_eps;
        ops(2, 0, 0, 2 * n);
        int jp = -1, jo = -1;
        for (int j = 0; j < n; ++j) {
            if (jp < 0 && ds[j] <= dlim) jp = j;
            if (jo < 0 && os[j] <= olim) jo = j;
        }
        if (jp != jp0 || jo != jo0) st.n_tie_pick++;
        for (int j = 0; j < n; ++j) {
            if (std::fabs(dp[jp]) + std::fabs(dp[j]) > harm) mg.add(std::fabs(ds[j] - dlim));
            if (std::fabs(dor[jo]) + std::fabs(dor[j]) > harm) mg.add(std::fabs(os[j] - olim));
        }

        // theta_hat: both moves if they act on different joints, otherwise the
        // larger one (ties -> position), Sec. IV-A.
        double hat[OR_MAX_DOF];
        std::memcpy(hat, th, sizeof(double) * n);
        if (jp != jo) {
            hat[jp] += dp[jp];
            hat[jo] += dor[jo];
            ops(2, 0);
        } else {
            if (std::fabs(dp[jp]) >= std::fabs(dor[jo]))
                hat[jp] += dp[jp];
            else
                hat[jo] += dor[jo];
            ops(1, 0);
            if (std::fabs(dp[jp] - dor[jo]) > harm)
                mg.add(std::fabs(std::fabs(dp[jp]) - std::fabs(dor[jo])));
        }

        // Accept on an improvement > gamma in position or in orientation,
        // otherwise perturb.
        Res rh = eval(rb, tg, hat);
        double e2p = dot(r.rp, r.rp), e2o = dot(r.omega, r.omega);
        double h2p = dot(rh.rp, rh.rp), h2o = dot(rh.omega, rh.omega);
        bool ia = (e2p - h2p) > p.gamma, ib = (e2o - h2o) > p.gamma;
        ops(2, 0);
        double ma = std::fabs(e2p - h2p - p.gamma) / std::max(std::sqrt(e2p) + std::sqrt(h2p), 1e-30);
        double mb = std::fabs(e2o - h2o - p.gamma) / std::max(std::sqrt(e2o) + std::sqrt(h2o), 1e-30);
        mg.add(or_margin(ia, ma, ib, mb));
        if (ia || ib) {
            std::memcpy(th, hat, sizeof(double) * n);
        } else {
            Unit up(OR_OPS_CD_PERTURB);
            perturb(rb, p, m, tkey, ST_CD, (uint32_t)k, th);
            st.n_perturb++;
        }
        st.iters_run++;
        if (margin) margin[k] = mg.v;
    }
    Res r;
    {
        Unit u(OR_OPS_EVAL);
        r = eval(rb, tg, th);
    }
    write_row(traj, K, n, th, r);
    if (r.ep < p.eps_cd && r.phi < p.nu_cd) st.frozen_at = K;
}

// ---------------------------------------------------------------------------
// Dense helpers for PJ-IK
// ---------------------------------------------------------------------------
// Solve A x = b for symmetric positive definite A (n x n, row-major) by Cholesky.
bool chol_solve(int n, std::vector<double> A, const double* b, double* x) {
    uint64_t fm = 0, fd = 0;  // multiply-subtract pairs, divisions
    for (int j = 0; j < n; ++j) {
        double s = A[j * n + j];
        for (int k = 0; k < j; ++k) s -= A[j * n + k] * A[j * n + k];
        fm += j;
        if (!(s > 0.0)) {
            ops(fm, fm, fd, j + 1);
            return false;
        }
        double l = std::sqrt(s);
        A[j * n + j] = l;
        for (int i = j + 1; i < n; ++i) {
            double t = A[i * n + j];
            for (int k = 0; k < j; ++k) t -= A[i * n + k] * A[j * n + k];
            A[i * n + j] = t / l;
            fm += j;
            fd += 1;
        }
    }
    std::vector<double> y(n);
    for (int i = 0; i < n; ++i) {
        double t = b[i];
        for (int k = 0; k < i; ++k) t -= A[i * n + k] * y[k];
        y[i] = t / A[i * n + i];
        fm += i;
        fd += 1;
    }
    for (int i = n - 1; i >= 0; --i) {
        double t = y[i];
        for (int k = i + 1; k < n; ++k) t -= A[k * n + i] * x[k];
        x[i] = t / A[i * n + i];
        fm += n - 1 - i;
        fd += 1;
    }
    ops(fm, fm, fd, n);
    return true;
}

double vnorm(int n, const double* x) {
    double s = x[0] * x[0];
    for (int i = 1; i < n; ++i) s += x[i] * x[i];
    ops(n - 1, n, 0, 1);
    return std::sqrt(s);
}

// Backtracking line search of eq. (line-search): alpha in [1, 1/beta, ...,
// 1/beta^A]; the first alpha whose clipped iterate lowers the cost wins.
// Returns true and updates theta on success.
bool line_search(const Robot& rb, const Target& tg, const or_params& p, double* th,
                 const double* step, double c0, Margin& mg, or_stage_stats& st, double harm,
                 double* alpha_taken) {
    const int n = rb.n;
    double alpha = 1.0;
    for (int i = 0; i <= p.ls_A; ++i) {
        Unit u(OR_OPS_PJ_TRIAL);
        double tt[OR_MAX_DOF];
        double smax = 0.0;
        for (int j = 0; j < n; ++j) {
            tt[j] = clip(th[j] + alpha * step[j], rb.lo[j], rb.hi[j]);
            smax = std::max(smax, std::fabs(alpha * step[j]));
        }
        ops(n, n);
        Res r = eval(rb, tg, tt);
        st.n_trials++;
        if (smax > harm) mg.add(std::fabs(std::sqrt(2.0 * r.cost) - std::sqrt(2.0 * c0)));
        if (r.cost < c0) {
            std::memcpy(th, tt, sizeof(double) * n);
            if (alpha_taken) *alpha_taken = alpha;
            return true;
        }
        alpha /= p.ls_beta;
        ops(0, 0, 1);
    }
    return false;
}

// ---------------------------------------------------------------------------
// PJ-IK pieces (Alg. PJ-IK, Sec. IV-B)
// ---------------------------------------------------------------------------
// Linearisation at theta: J (6 x n, row-major), e = [r_p; omega], row
// weights w (W = diag(w)), D = diag(J^T J).
struct Lin {
    int n;
    std::vector<double> J;
    double e[6];
    double w[6];
    double Dg[OR_MAX_DOF];
};

Lin linearise(const Robot& rb, const or_params& p, const FK& f, const Res& r) {
    Lin L;
    const int n = rb.n;
    L.n = n;
    L.J.assign(6 * n, 0.0);
    jacobian(rb, f, L.J.data());
    const double e[6] = {r.rp.x, r.rp.y, r.rp.z, r.omega.x, r.omega.y, r.omega.z};
    for (int i = 0; i < 6; ++i) L.e[i] = e[i];
    // W normalises the rows of J (reading of Sec. IV-B).
    for (int i = 0; i < 6; ++i) {
        if (p.weight_mode != 0) {
            L.w[i] = 1.0;
            continue;
        }
        double s = L.J[i * n] * L.J[i * n];
        for (int j = 1; j < n; ++j) s += L.J[i * n + j] * L.J[i * n + j];
        L.w[i] = 1.0 / std::max(std::sqrt(s), 1e-6);
        ops(n - 1, n, 1, 1);
    }
    for (int j = 0; j < n; ++j) {
        double s = L.J[j] * L.J[j];
        for (int i = 1; i < 6; ++i) s += L.J[i * n + j] * L.J[i * n + j];
        L.Dg[j] = s;
    }
    ops(5 * n, 6 * n);
    return L;
}

// eq. (normal-eqs) read with W^T W on both sides and the sign that steps
// toward the target: (J^T W^2 J + lambda D) dtheta = J^T W^2 e, solved as the
// n x n system by Cholesky (the matrix is symmetric: its lower triangle is
// formed and mirrored).  Unclipped.
void lm_step(const Lin& L, const or_params& p, double* dth) {
    const int n = L.n;
    std::vector<double> A(n * n, 0.0);
    double b[OR_MAX_DOF], w2[6], we[6];
    for (int i = 0; i < 6; ++i) {
        w2[i] = L.w[i] * L.w[i];
        we[i] = w2[i] * L.e[i];
    }
    ops(0, 12);
    for (int a = 0; a < n; ++a) {
        for (int c = 0; c <= a; ++c) {
            double s = L.J[a] * w2[0] * L.J[c];
            for (int i = 1; i < 6; ++i) s += L.J[i * n + a] * w2[i] * L.J[i * n + c];
            if (a == c) s += p.lam * L.Dg[a];
            A[a * n + c] = s;
            A[c * n + a] = s;
        }
        double s = L.J[a] * we[0];
        for (int i = 1; i < 6; ++i) s += L.J[i * n + a] * we[i];
        b[a] = s;
    }
    const uint64_t pairs = (uint64_t)n * (n + 1) / 2;
    ops(5 * pairs + n + 5 * n, 12 * pairs + n + 6 * n);
    chol_solve(n, A, b, dth);
}

// eq. (dogleg): gradient step dGD = alpha_c J^T e with the Cauchy length
// alpha_c = |g|^2 / |J g|^2, Gauss-Newton step dGN = J^T (J J^T + lambda_gn I)^-1 e,
// blended as dGN + tau (dGD - dGN) with the smallest tau in [0, 1] whose step
// has 2-norm <= R.
void dogleg_step(const Lin& L, const or_params& p, double* step, double* gd, double* gn) {
    const int n = L.n;
    const double R = p.trust_R;
    double g[OR_MAX_DOF];
    for (int j = 0; j < n; ++j) {
        double s = L.J[j] * L.e[0];
        for (int i = 1; i < 6; ++i) s += L.J[i * n + j] * L.e[i];
        g[j] = s;
    }
    double Jg[6];
    for (int i = 0; i < 6; ++i) {
        double s = L.J[i * n] * g[0];
        for (int j = 1; j < n; ++j) s += L.J[i * n + j] * g[j];
        Jg[i] = s;
    }
    double jgjg = Jg[0] * Jg[0];  // |J g|^2
    for (int i = 1; i < 6; ++i) jgjg += Jg[i] * Jg[i];
    double gg = g[0] * g[0];
    for (int j = 1; j < n; ++j) gg += g[j] * g[j];
    double ac = jgjg > 0.0 ? gg / jgjg : 0.0;
    for (int j = 0; j < n; ++j) gd[j] = ac * g[j];
    ops(5 * n + 6 * (n - 1) + 5 + (n - 1), 6 * n + 6 * n + 6 + n + n, 1);
    std::vector<double> JJt(36, 0.0);
    for (int a = 0; a < 6; ++a)
        for (int c = 0; c <= a; ++c) {
            double s = L.J[a * n] * L.J[c * n];
            for (int j = 1; j < n; ++j) s += L.J[a * n + j] * L.J[c * n + j];
            if (a == c) s += p.lambda_gn;
            JJt[a * 6 + c] = s;
            JJt[c * 6 + a] = s;
        }
    ops(21 * (n - 1) + 6, 21 * n);
    double y[6];
    chol_solve(6, JJt, L.e, y);
    for (int j = 0; j < n; ++j) {
        double s = L.J[j] * y[0];
        for (int i = 1; i < 6; ++i) s += L.J[i * n + j] * y[i];
        gn[j] = s;
    }
    ops(5 * n, 6 * n);
    double ngn = vnorm(n, gn), ngd = vnorm(n, gd);
    if (ngn <= R) {
        for (int j = 0; j < n; ++j) step[j] = gn[j];
    } else if (ngd >= R) {
        for (int j = 0; j < n; ++j) step[j] = R * gd[j] / ngd;
        ops(0, n, n);
    } else {
        // |gn + tau d|^2 = R^2 is a convex quadratic, > 0 at tau = 0 and < 0 at
        // tau = 1: its smaller root, in the cancellation-free form.
        double aa = 0.0, bb = 0.0;
        for (int j = 0; j < n; ++j) {
            double dj = gd[j] - gn[j];
            aa += dj * dj;
            bb += gn[j] * dj;
        }
        double cc = ngn * ngn - R * R;
        double den = -bb + std::sqrt(std::max(bb * bb - aa * cc, 0.0));
        double tau = den > 0.0 ? clip(cc / den, 0.0, 1.0) : 0.0;
        for (int j = 0; j < n; ++j) step[j] = gn[j] + tau * (gd[j] - gn[j]);
        ops(3 * n + 3 + 2 * n, 2 * n + 4 + n, 1, 1);
    }
}

// eq. (single-coord): the coordinate i* with the largest |g^W_i|, g^W =
// J^T W^2 e = -d/dtheta 0.5 |W r|^2 (ties -> lower i), moved by the
// coordinate-Newton length g^W_i* / (J^T W^2 J)_i*i*, clipped to [-R, R].
int single_step(const Lin& L, const or_params& p, double* step, Margin& mg) {
    const int n = L.n;
    double gw[OR_MAX_DOF], w2[6], we[6];
    for (int i = 0; i < 6; ++i) {
        w2[i] = L.w[i] * L.w[i];
        we[i] = w2[i] * L.e[i];
    }
    int is = 0;
    for (int j = 0; j < n; ++j) {
        double s = L.J[j] * we[0];
        for (int i = 1; i < 6; ++i) s += L.J[i * n + j] * we[i];
        gw[j] = s;
        if (std::fabs(gw[j]) > std::fabs(gw[is])) is = j;
    }
    for (int j = 0; j < n; ++j)
        if (j != is) mg.add(std::fabs(std::fabs(gw[is]) - std::fabs(gw[j])));
    double h = L.J[is] * w2[0] * L.J[is];
    for (int i = 1; i < 6; ++i) h += L.J[i * n + is] * w2[i] * L.J[i * n + is];
    for (int j = 0; j < n; ++j) step[j] = 0.0;
    step[is] = h > 0.0 ? clip(gw[is] / h, -p.trust_R, p.trust_R) : 0.0;
    ops(5 * n + 5, 12 + 6 * n + 12, 1);
    return is;
}

// ---------------------------------------------------------------------------
// Conditioning of a PJ-IK step (test instrumentation, not part of the
// method): how far the step taken moves (infinity norm, rad) when J and e
// carry single-precision-sized errors.  Near singular configurations the
// damped systems amplify such errors up to 1/lambda.
// ---------------------------------------------------------------------------
enum StepKind { STEP_LM = 0, STEP_DOGLEG = 1, STEP_SINGLE = 2, STEP_PERTURB = 3 };

Lin perturbed(const Lin& L, const or_params& p, uint64_t key) {
    Lin P = L;
    uint64_t x = key * 0x9E3779B97F4A7C15ull + 0x2545F4914F6CDD1Dull;
    auto sgn = [&x]() {
        x ^= x << 13;
        x ^= x >> 7;
        x ^= x << 17;
        return (x >> 11) & 1 ? 1.0 : -1.0;
    };
    const int n = L.n;
    for (int i = 0; i < 6 * n; ++i) P.J[i] = L.J[i] * (1.0 + 2.4e-7 * sgn()) + 1e-7 * sgn();
    for (int i = 0; i < 6; ++i) P.e[i] = L.e[i] + 3e-7 * sgn();
    for (int i = 0; i < 6; ++i) {
        double s = 0.0;
        for (int j = 0; j < n; ++j) s += P.J[i * n + j] * P.J[i * n + j];
        P.w[i] = (p.weight_mode == 0) ? 1.0 / std::max(std::sqrt(s), 1e-6) : 1.0;
    }
    for (int j = 0; j < n; ++j) {
        double s = 0.0;
        for (int i = 0; i < 6; ++i) s += P.J[i * n + j] * P.J[i * n + j];
        P.Dg[j] = s;
    }
    return P;
}

void step_of_kind(const Lin& L, const or_params& p, int kind, double alpha, int is, double* out) {
    const int n = L.n;
    if (kind == STEP_LM) {
        lm_step(L, p, out);
        for (int j = 0; j < n; ++j) out[j] = alpha * clip(out[j], -p.trust_R, p.trust_R);
    } else if (kind == STEP_DOGLEG) {
        double gd[OR_MAX_DOF], gn[OR_MAX_DOF];
        dogleg_step(L, p, out, gd, gn);
    } else {
        double gw = 0.0, h = 0.0;
        for (int i = 0; i < 6; ++i) {
            gw += L.J[i * n + is] * L.w[i] * L.w[i] * L.e[i];
            h += L.J[i * n + is] * L.w[i] * L.w[i] * L.J[i * n + is];
        }
        for (int j = 0; j < n; ++j) out[j] = 0.0;
        out[is] = alpha * (h > 0.0 ? clip(gw / h, -p.trust_R, p.trust_R) : 0.0);
    }
}

double step_sensitivity(const Lin& L, const or_params& p, int kind, double alpha, int is, int it) {
    if (kind == STEP_PERTURB) return 0.0;
    const int n = L.n;
    double base[OR_MAX_DOF], alt[OR_MAX_DOF];
    step_of_kind(L, p, kind, alpha, is, base);
    double worst = 0.0;
    for (int rep = 0; rep < 4; ++rep) {
        Lin P = perturbed(L, p, (uint64_t)(it * 8 + rep + 1));
        step_of_kind(P, p, kind, alpha, is, alt);
        for (int j = 0; j < n; ++j) worst = std::max(worst, std::fabs(alt[j] - base[j]));
    }
    return worst;
}

// ---------------------------------------------------------------------------
// PJ-IK on one seed (Alg. PJ-IK, Sec. IV-B)
// ---------------------------------------------------------------------------
void pj_ik(const Robot& rb, const Target& tg, const or_params& p, uint32_t m, uint32_t tkey,
           double* th, double* traj, double* margin, double* sens, or_stage_stats& st, double harm) {
    const int n = rb.n;
    const int K = p.polish_iters;
    const double R = p.trust_R;
    st = or_stage_stats{0, -1, 0, 0, 0, 0, 0};
    for (int it = 0; it < K; ++it) {
        FK f;
        Res r;
        {
            Unit u(OR_OPS_EVAL);
            fk(rb, th, f);
            r = residual(tg, f.p_ee, f.R_ee);
        }
        write_row(traj, it, n, th, r);
        Margin mg;
        // Exit test of Alg. PJ-IK, evaluated on the configuration the previous
        // iteration produced.
        bool ca = r.ep < p.eps_pol, cb = r.phi < p.ups_pol;
        mg.add(and_margin(ca, std::fabs(r.ep - p.eps_pol), cb, std::fabs(r.phi - p.ups_pol)));
        if (ca && cb) {
            st.frozen_at = it;
            if (margin) margin[it] = mg.v;
            for (int kk = it + 1; kk <= K; ++kk) write_row(traj, kk, n, th, r);
            for (int kk = it + 1; kk < K; ++kk)
                if (margin) margin[kk] = kInf;
            for (int kk = it; kk < K; ++kk)
                if (sens) sens[kk] = 0.0;
            return;
        }
        const double c0 = r.cost;
        Lin L;
        double dth[OR_MAX_DOF];
        {
            Unit u(OR_OPS_PJ_ITER);
            L = linearise(rb, p, f, r);
            if (p.shadow) L = perturbed(L, p, p.shadow * 1000003ull + (uint64_t)it);
            // LM step, trust-region clamp, backtracking line search.
            lm_step(L, p, dth);
            for (int j = 0; j < n; ++j) dth[j] = clip(dth[j], -R, R);
        }
        double alpha = 1.0;
        int kind = STEP_LM, is = 0;
        bool ok = line_search(rb, tg, p, th, dth, c0, mg, st, harm, &alpha);
        if (!ok) {
            // Dogleg fallback, one trial.
            kind = STEP_DOGLEG;
            alpha = 1.0;
            st.n_dogleg++;
            double step[OR_MAX_DOF], gd[OR_MAX_DOF], gn[OR_MAX_DOF];
            {
                Unit u(OR_OPS_PJ_DOGLEG);
                dogleg_step(L, p, step, gd, gn);
            }
            Unit u(OR_OPS_PJ_TRIAL);
            double tt[OR_MAX_DOF], smax = 0.0;
            for (int j = 0; j < n; ++j) {
                tt[j] = clip(th[j] + step[j], rb.lo[j], rb.hi[j]);
                smax = std::max(smax, std::fabs(step[j]));
            }
            ops(n, 0);
            Res rr = eval(rb, tg, tt);
            st.n_trials++;
            if (smax > harm) mg.add(std::fabs(std::sqrt(2.0 * rr.cost) - std::sqrt(2.0 * c0)));
            if (rr.cost < c0) {
                std::memcpy(th, tt, sizeof(double) * n);
                ok = true;
            }
        }
        if (!ok) {
            // Single-coordinate fallback with the same line search.
            st.n_single++;
            double step[OR_MAX_DOF];
            kind = STEP_SINGLE;
            {
                Unit u(OR_OPS_PJ_SINGLE);
                is = single_step(L, p, step, mg);
            }
            ok = line_search(rb, tg, p, th, step, c0, mg, st, harm, &alpha);
        }
        if (!ok) {
            Unit u(OR_OPS_PJ_PERTURB);
            kind = STEP_PERTURB;
            perturb(rb, p, m, tkey, ST_POLISH, (uint32_t)it, th);
            st.n_perturb++;
        }
        if (sens) {
            Scope instr(OR_OPS_INSTR);
            sens[it] = step_sensitivity(L, p, kind, alpha, is, it);
        }
        st.iters_run++;
        if (margin) margin[it] = mg.v;
    }
    Res r;
    {
        Unit u(OR_OPS_EVAL);
        r = eval(rb, tg, th);
    }
    write_row(traj, K, n, th, r);
    if (r.ep < p.eps_pol && r.phi < p.ups_pol) st.frozen_at = K;
}

// ---------------------------------------------------------------------------
// Collision (Sec. IV-C), flat: every robot sphere against every obstacle and
// every allowed self pair.
// ---------------------------------------------------------------------------
struct Scene {
    std::vector<double> sph, box;
};

void collide(const Robot& rb, const Scene& sc, const double* th, int& flag, double& mind) {
    FK f;
    fk(rb, th, f);
    const int ns = (int)rb.sph_link.size();
    std::vector<V3> c(ns);
    std::vector<double> rad(ns);
    for (int s = 0; s < ns; ++s) {
        const H4& T = f.link[rb.sph_link[s]];
        const double* q = &rb.sph[4 * s];
        c[s] = v3(T.m[0][0] * q[0] + T.m[0][1] * q[1] + T.m[0][2] * q[2] + T.m[0][3],
                  T.m[1][0] * q[0] + T.m[1][1] * q[1] + T.m[1][2] * q[2] + T.m[1][3],
                  T.m[2][0] * q[0] + T.m[2][1] * q[1] + T.m[2][2] * q[2] + T.m[2][3]);
        rad[s] = q[3];
    }
    ops(9 * ns, 9 * ns);
    flag = 0;
    mind = kInf;
    const int no = (int)sc.sph.size() / 4, nb = (int)sc.box.size() / 6;
    for (int s = 0; s < ns; ++s) {
        for (int o = 0; o < no; ++o) {
            const double* ob = &sc.sph[4 * o];
            V3 dlt = c[s] - v3(ob[0], ob[1], ob[2]);
            double rr = rad[s] + ob[3];
            if (dot(dlt, dlt) < rr * rr) flag = 1;
            ops(1, 1);
            Scope instr(OR_OPS_INSTR);
            mind = std::min(mind, norm(dlt) - rr);
        }
        for (int o = 0; o < nb; ++o) {
            const double* bx = &sc.box[6 * o];
            double cs[3] = {c[s].x, c[s].y, c[s].z};
            double q2 = 0.0;
            for (int k = 0; k < 3; ++k) {
                double ex = std::max(0.0, std::fabs(cs[k] - bx[k]) - bx[3 + k]);
                q2 += ex * ex;
            }
            if (q2 < rad[s] * rad[s]) flag = 1;
            ops(9, 4);
            mind = std::min(mind, std::sqrt(q2) - rad[s]);
        }
    }
    if (rb.gap > 0) {
        for (int a = 0; a < ns; ++a)
            for (int b = a + 1; b < ns; ++b) {
                if (std::abs(rb.sph_link[a] - rb.sph_link[b]) < rb.gap) continue;
                V3 dlt = c[a] - c[b];
                double rr = rad[a] + rad[b];
                if (dot(dlt, dlt) < rr * rr) flag = 1;
                ops(1, 1);
                Scope instr(OR_OPS_INSTR);
                mind = std::min(mind, norm(dlt) - rr);
            }
    }
}

// Stable order by (flag, cost, index): the final argmin of Alg. HJCD-IK
// extended to the best k, colliding seeds after every collision-free one.
void select_order(int m, const int32_t* flag, const double* cost, int k, int32_t* order) {
    std::vector<int> idx(m);
    for (int i = 0; i < m; ++i) idx[i] = i;
    std::stable_sort(idx.begin(), idx.end(), [&](int a, int b) {
        int fa = flag[a] != 0, fb = flag[b] != 0;
        if (fa != fb) return fa < fb;
        if (cost[a] != cost[b]) return cost[a] < cost[b];
        return a < b;
    });
    for (int i = 0; i < k; ++i) order[i] = i < m ? idx[i] : -1;
}

}  // namespace

// ---------------------------------------------------------------------------
// C API
// ---------------------------------------------------------------------------
extern "C" {

int or_fk(const or_robot* rbi, const double* theta, double* p_ee, double* R_ee, double* quat,
          double* joint_P, double* joint_z, double* link_T, double* J) {
    Robot rb;
    if (!load_robot(rbi, rb)) return -1;
    FK f;
    fk(rb, theta, f);
    if (p_ee) {
        p_ee[0] = f.p_ee.x;
        p_ee[1] = f.p_ee.y;
        p_ee[2] = f.p_ee.z;
    }
    if (R_ee)
        for (int i = 0; i < 3; ++i)
            for (int j = 0; j < 3; ++j) R_ee[3 * i + j] = f.R_ee[i][j];
    if (quat) {
        Q4 q = quat_from_R(f.R_ee);
        quat[0] = q.w;
        quat[1] = q.v.x;
        quat[2] = q.v.y;
        quat[3] = q.v.z;
    }
    for (int i = 0; i < rb.n; ++i) {
        if (joint_P) {
            joint_P[3 * i] = f.P[i].x;
            joint_P[3 * i + 1] = f.P[i].y;
            joint_P[3 * i + 2] = f.P[i].z;
        }
        if (joint_z) {
            joint_z[3 * i] = f.z[i].x;
            joint_z[3 * i + 1] = f.z[i].y;
            joint_z[3 * i + 2] = f.z[i].z;
        }
    }
    if (link_T)
        for (int l = 0; l <= rb.n; ++l)
            for (int i = 0; i < 3; ++i)
                for (int j = 0; j < 4; ++j) link_T[12 * l + 4 * i + j] = f.link[l].m[i][j];
    if (J) jacobian(rb, f, J);
    return 0;
}

void or_quat_from_R(const double* R, double* q) {
    double M[3][3];
    for (int i = 0; i < 3; ++i)
        for (int j = 0; j < 3; ++j) M[i][j] = R[3 * i + j];
    Q4 x = quat_from_R(M);
    q[0] = x.w;
    q[1] = x.v.x;
    q[2] = x.v.y;
    q[3] = x.v.z;
}

void or_residual(const double* p_t, const double* q_t, const double* p_ee, const double* R_ee,
                 double* out) {
    double t7[7] = {p_t[0], p_t[1], p_t[2], q_t[0], q_t[1], q_t[2], q_t[3]};
    Target tg = load_target(t7);
    double M[3][3];
    for (int i = 0; i < 3; ++i)
        for (int j = 0; j < 3; ++j) M[i][j] = R_ee[3 * i + j];
    Res r = residual(tg, v3(p_ee[0], p_ee[1], p_ee[2]), M);
    double v[11] = {r.rp.x, r.rp.y, r.rp.z, r.omega.x, r.omega.y, r.omega.z, r.phi,
                    r.ahat.x, r.ahat.y, r.ahat.z, r.cost};
    std::memcpy(out, v, sizeof(v));
}

void or_philox4x32_10(const uint32_t* ctr, const uint32_t* key, uint32_t* out) { philox(ctr, key, out); }

void or_normals(uint64_t rng_seed, uint32_t seed_idx, uint32_t target_key, uint32_t stage,
                uint32_t iter, int dof, double* z) {
    normals(rng_seed, seed_idx, target_key, stage, iter, dof, z);
}

void or_uniform_seed(const or_robot* rbi, uint64_t rng_seed, uint32_t seed_idx,
                     uint32_t target_key, double* theta) {
    Robot rb;
    if (!load_robot(rbi, rb)) return;
    uniform_seed(rb, rng_seed, seed_idx, target_key, theta);
}

static const double kHarm = 1e-6;

int or_cd(const or_robot* rbi, const double* target, const or_params* pr, uint32_t seed_idx,
          uint32_t target_key, double* theta, double* traj, double* margin, or_stage_stats* st) {
    Robot rb;
    if (!load_robot(rbi, rb) || !pr) return -1;
    Target tg = load_target(target);
    or_stage_stats s;
    po_ccd(rb, tg, *pr, seed_idx, target_key, theta, traj, margin, s, kHarm);
    flush_ops();
    if (st) *st = s;
    return 0;
}

int or_polish(const or_robot* rbi, const double* target, const or_params* pr, uint32_t seed_idx,
              uint32_t target_key, double* theta, double* traj, double* margin, double* sens,
              or_stage_stats* st) {
    Robot rb;
    if (!load_robot(rbi, rb) || !pr) return -1;
    Target tg = load_target(target);
    or_stage_stats s;
    pj_ik(rb, tg, *pr, seed_idx, target_key, theta, traj, margin, sens, s, kHarm);
    flush_ops();
    if (st) *st = s;
    return 0;
}

int or_cd_candidates(const or_robot* rbi, const double* target, const or_params* pr,
                     const double* theta, int32_t k, double* dp, double* dor, double* sp,
                     double* so) {
    Robot rb;
    if (!load_robot(rbi, rb) || !pr) return -1;
    Target tg = load_target(target);
    FK f;
    fk(rb, theta, f);
    Res r = residual(tg, f.p_ee, f.R_ee);
    Margin mg;
    cd_candidates(rb, tg, *pr, theta, k, f, r, dp, dor, sp, so, mg, kHarm);
    return 0;
}

int or_pjik_steps(const or_robot* rbi, const double* target, const or_params* pr,
                  const double* theta, double* lm, double* gd, double* gn, double* dogleg,
                  double* single, int32_t* single_idx) {
    Robot rb;
    if (!load_robot(rbi, rb) || !pr) return -1;
    Target tg = load_target(target);
    FK f;
    fk(rb, theta, f);
    Res r = residual(tg, f.p_ee, f.R_ee);
    Lin L = linearise(rb, *pr, f, r);
    lm_step(L, *pr, lm);
    dogleg_step(L, *pr, dogleg, gd, gn);
    Margin mg;
    *single_idx = single_step(L, *pr, single, mg);
    return 0;
}

int or_collide(const or_robot* rbi, const or_scene* sci, const double* theta, int32_t* flag,
               double* min_signed_dist) {
    Robot rb;
    if (!load_robot(rbi, rb)) return -1;
    Scene sc;
    if (sci) {
        sc.sph.assign(sci->spheres, sci->spheres + 4 * sci->n_spheres);
        sc.box.assign(sci->boxes, sci->boxes + 6 * sci->n_boxes);
    }
    int f;
    double md;
    {
        Unit u(OR_OPS_COLLIDE);
        collide(rb, sc, theta, f, md);
    }
    flush_ops();
    if (flag) *flag = f;
    if (min_signed_dist) *min_signed_dist = md;
    return 0;
}

int or_select(int32_t m, const int32_t* flag, const double* cost, int32_t k, int32_t* order) {
    if (m < 0 || k < 0) return -1;
    select_order(m, flag, cost, k, order);
    return 0;
}

// Top-K ranking and noisy replication for one target (Alg. HJCD-IK): its M
// seeds th [M*n] with costs cst [M] are ranked by (cost, index); copy i of
// rank kk (i < floor(B/K), kk < K) is written to row i*K + kk of out
// [floor(B/K)*K*n] as clip(theta + mu + sigma z), z drawn for seed index
// i*K + kk at stage RESAMPLE.  A target with fewer than K seeds (M < K, M >= 1)
// repeats its ranked seeds cyclically: rank kk takes the seed of rank kk mod M.
void resample_target(const Robot& rb, const or_params& p, int M, const double* th, const double* cst,
                     uint32_t tkey, double* out) {
    const int n = rb.n;
    const int K = p.resample_K;
    const int copies = p.resample_B / K;
    std::vector<int> idx(M);
    for (int i = 0; i < M; ++i) idx[i] = i;
    std::stable_sort(idx.begin(), idx.end(), [&](int a, int b) {
        if (cst[a] != cst[b]) return cst[a] < cst[b];
        return a < b;
    });
    for (int i = 0; i < copies; ++i)
        for (int kk = 0; kk < K; ++kk) {
            Unit u(OR_OPS_RESAMPLE);
            double* x = out + (size_t)(i * K + kk) * n;
            std::memcpy(x, th + (size_t)idx[kk % M] * n, sizeof(double) * n);
            perturb(rb, p, (uint32_t)(i * K + kk), tkey, ST_RESAMPLE, 0, x);
        }
}

// Warm start for a target on a path (Sec. V, the hardware demonstration:
// each pose is solved from the solution set of the previous one): seed m of
// target t starts at previous solution m mod k, unchanged for m < k and
// moved by clip(. + mu + sigma z) otherwise, z drawn for seed index m at
// stage WARM, iteration 0.
int or_warm_seeds(const or_robot* rbi, int32_t T, int32_t k, const double* q_prev, int32_t M,
                  const uint32_t* target_keys, const or_params* pr, double* q_out) {
    Robot rb;
    if (!load_robot(rbi, rb) || !pr || T < 0 || k < 1 || M < 0) return -1;
    const int n = rb.n;
    for (int t = 0; t < T; ++t) {
        const uint32_t tkey = target_keys ? target_keys[t] : (uint32_t)t;
        for (int m = 0; m < M; ++m) {
            const double* src = q_prev + (size_t)(t * k + m % k) * n;
            double* x = q_out + ((size_t)t * M + m) * n;
            for (int j = 0; j < n; ++j) x[j] = clip(src[j], rb.lo[j], rb.hi[j]);
            if (m >= k) perturb(rb, *pr, (uint32_t)m, tkey, ST_WARM, 0, x);
        }
    }
    flush_ops();
    return 0;
}

// Selection nearest to a reference configuration (the tracking variant of the
// final selection): seeds that are collision free with err_p <= succ_pos and
// err_o <= succ_ori come first, ordered by squared joint distance to q_ref;
// every other seed follows in the (flag, cost) order; ties go to the lower
// index.
int or_select_near(int32_t m, int32_t dof, const int32_t* flag, const double* cost, const double* err_p,
                   const double* err_o, const double* q, const double* q_ref, double succ_pos, double succ_ori,
                   int32_t k, int32_t* order) {
    if (m < 0 || k < 0 || dof < 1) return -1;
    std::vector<int> cls(m);
    std::vector<double> key(m);
    for (int i = 0; i < m; ++i) {
        const bool ok = flag[i] == 0 && err_p[i] <= succ_pos && err_o[i] <= succ_ori;
        cls[i] = ok ? 0 : (flag[i] == 0 ? 1 : 2);
        if (ok) {
            double d2 = 0.0;
            for (int j = 0; j < dof; ++j) {
                const double dj = q[(size_t)i * dof + j] - q_ref[j];
                d2 += dj * dj;
            }
            key[i] = d2;
        } else {
            key[i] = cost[i];
        }
    }
    std::vector<int> idx(m);
    for (int i = 0; i < m; ++i) idx[i] = i;
    std::stable_sort(idx.begin(), idx.end(), [&](int a, int b) {
        if (cls[a] != cls[b]) return cls[a] < cls[b];
        if (key[a] != key[b]) return key[a] < key[b];
        return a < b;
    });
    for (int i = 0; i < k; ++i) order[i] = i < m ? idx[i] : -1;
    return 0;
}

int or_resample(const or_robot* rbi, int32_t T, const int64_t* offsets, const double* q_in,
                const double* cost_in, const uint32_t* target_keys, const or_params* pr, double* q_out) {
    Robot rb;
    if (!load_robot(rbi, rb) || !pr || T < 0 || pr->resample_K < 1 || pr->resample_B < pr->resample_K) return -1;
    for (int t = 0; t < T; ++t)
        if (offsets[t + 1] <= offsets[t]) return -1;
    const int n = rb.n;
    const int64_t Bp = (int64_t)(pr->resample_B / pr->resample_K) * pr->resample_K;
    for (int t = 0; t < T; ++t) {
        const int64_t b0 = offsets[t];
        const int M = (int)(offsets[t + 1] - b0);
        resample_target(rb, *pr, M, q_in + (size_t)b0 * n, cost_in + b0,
                        target_keys ? target_keys[t] : (uint32_t)t, q_out + (size_t)(t * Bp) * n);
    }
    flush_ops();
    return 0;
}

int or_solve(const or_robot* rbi, const or_scene* sci, int32_t T, const double* targets,
             const int64_t* offsets, const double* seeds, const uint32_t* target_keys,
             const or_params* pr, double* q_seed, double* errp_seed, double* erro_seed,
             double* cost_seed, int32_t* flag_seed, double* q_out, double* err_p, double* err_o,
             int32_t* flag_out, int32_t* n_free, int32_t* solved, int32_t nthreads) {
    Robot rb;
    if (!load_robot(rbi, rb) || !pr || T < 0) return -1;
    const bool resample = pr->resample_K > 0;
    if (resample && pr->resample_B < pr->resample_K) return -1;
    for (int t = 0; t < T; ++t) {
        if (offsets[t + 1] < offsets[t]) return -1;
        if (resample && offsets[t + 1] == offsets[t]) return -1;  // nothing to rank
    }
    Scene sc;
    if (sci) {
        sc.sph.assign(sci->spheres, sci->spheres + 4 * sci->n_spheres);
        sc.box.assign(sci->boxes, sci->boxes + 6 * sci->n_boxes);
    }
    const or_params p = *pr;
    const int n = rb.n;
    const int k = p.top_k;
    // seeds polished per target with resampling: floor(B/K) copies of the K best
    const int Bp = resample ? (p.resample_B / p.resample_K) * p.resample_K : 0;

    auto work = [&](int t) {
        Target tg = load_target(targets + 7 * (size_t)t);
        const uint32_t tkey = target_keys ? target_keys[t] : (uint32_t)t;
        const int64_t b0 = offsets[t];
        const int M = (int)(offsets[t + 1] - offsets[t]);
        // Stage 1: seeds + PO-CCD (Alg. HJCD-IK, first line).
        std::vector<double> th((size_t)M * n);
        std::vector<double> cst(M);
        or_stage_stats s;
        for (int m = 0; m < M; ++m) {
            double* x = &th[(size_t)m * n];
            if (seeds) {
                for (int j = 0; j < n; ++j) x[j] = clip(seeds[(size_t)(b0 + m) * n + j], rb.lo[j], rb.hi[j]);
            } else {
                Unit u(OR_OPS_INIT);
                uniform_seed(rb, p.rng_seed, (uint32_t)m, tkey, x);
            }
            po_ccd(rb, tg, p, (uint32_t)m, tkey, x, nullptr, nullptr, s, kHarm);
            Unit u(OR_OPS_EVAL);
            cst[m] = eval(rb, tg, x).cost;
        }
        // Optional top-K and noisy replication (Alg. HJCD-IK).
        int Mb = M;
        int64_t base = b0;
        if (resample) {
            std::vector<double> nth((size_t)Bp * n);
            resample_target(rb, p, M, th.data(), cst.data(), tkey, nth.data());
            th.swap(nth);
            Mb = Bp;
            base = (int64_t)t * Bp;
        }
        // Stage 2: PJ-IK, stage 3: collision filter and selection.
        std::vector<int32_t> fl(Mb);
        std::vector<double> c2(Mb), ep(Mb), eo(Mb);
        for (int m = 0; m < Mb; ++m) {
            double* x = &th[(size_t)m * n];
            pj_ik(rb, tg, p, (uint32_t)m, tkey, x, nullptr, nullptr, nullptr, s, kHarm);
            Res r;
            {
                Unit u(OR_OPS_EVAL);
                r = eval(rb, tg, x);
            }
            c2[m] = r.cost;
            ep[m] = r.ep;
            eo[m] = r.phi;
            double md;
            int f;
            {
                Unit u(OR_OPS_COLLIDE);
                collide(rb, sc, x, f, md);
            }
            fl[m] = f;
            if (q_seed) std::memcpy(q_seed + (size_t)(base + m) * n, x, sizeof(double) * n);
            if (errp_seed) errp_seed[base + m] = r.ep;
            if (erro_seed) erro_seed[base + m] = r.phi;
            if (cost_seed) cost_seed[base + m] = r.cost;
            if (flag_seed) flag_seed[base + m] = f;
        }
        std::vector<int32_t> ord(k);
        {
            Unit u(OR_OPS_SELECT);
            select_order(Mb, fl.data(), c2.data(), k, ord.data());
        }
        int nf = 0;
        for (int m = 0; m < Mb; ++m) nf += fl[m] == 0;
        int ok = 0;
        for (int i = 0; i < k; ++i) {
            size_t o = (size_t)t * k + i;
            int m = ord[i];
            if (m < 0) {
                if (q_out)
                    for (int j = 0; j < n; ++j) q_out[o * n + j] = 0.0;
                if (err_p) err_p[o] = kInf;
                if (err_o) err_o[o] = kInf;
                if (flag_out) flag_out[o] = 255;
                continue;
            }
            if (q_out) std::memcpy(q_out + o * n, &th[(size_t)m * n], sizeof(double) * n);
            if (err_p) err_p[o] = ep[m];
            if (err_o) err_o[o] = eo[m];
            if (flag_out) flag_out[o] = fl[m];
            if (fl[m] == 0 && ep[m] <= p.succ_pos && eo[m] <= p.succ_ori) ok = 1;
        }
        if (n_free) n_free[t] = nf;
        if (solved) solved[t] = ok;
    };

    int nt = nthreads > 0 ? nthreads : (int)std::max(1u, std::thread::hardware_concurrency());
    nt = std::min(nt, std::max(T, 1));
    std::vector<std::thread> pool;
    std::atomic_int counter{0};
    for (int w = 0; w < nt; ++w)
        pool.emplace_back([&]() {
            for (;;) {
                int t = counter.fetch_add(1);
                if (t >= T) break;
                work(t);
            }
            flush_ops();
        });
    for (auto& th : pool) th.join();
    return 0;
}

void or_ops_reset(void) {
    std::lock_guard<std::mutex> lk(g_ops_mu);
    for (int c = 0; c < OR_OPS_NCAT; ++c) {
        g_ops[c] = Ops{0, 0, 0, 0, 0, 0};
        tl_ops[c] = Ops{0, 0, 0, 0, 0, 0};
    }
}

int or_ops_get(int32_t cat, uint64_t* out) {
    if (cat < 0 || cat >= OR_OPS_NCAT || !out) return -1;
    flush_ops();
    std::lock_guard<std::mutex> lk(g_ops_mu);
    const Ops& o = g_ops[cat];
    out[0] = o.add;
    out[1] = o.mul;
    out[2] = o.div;
    out[3] = o.sqrt;
    out[4] = o.trans;
    out[5] = o.units;
    return 0;
}

}  // extern "C"
