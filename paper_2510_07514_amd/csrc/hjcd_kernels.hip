// Kernels of libhjcd for gfx950 (CDNA4, wave64).  Citations refer to
// arXiv 2510.07514.
#include <hip/hip_runtime.h>
#include <stdint.h>

#include "hjcd_device.hpp"
#include "hjcd_launch.hpp"

namespace hjcd {

// ----------------------------------------------------------------------------
// FK + Jacobian of S configurations (eq. fk, eq. jacobian)
// ----------------------------------------------------------------------------
template <int NM>
__global__ __launch_bounds__(256) void k_fk(const DevRobot* __restrict__ rb, int n, int64_t S,
                                            const float* __restrict__ q, float* __restrict__ pose,
                                            float* __restrict__ jac) {
    const int64_t s = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (s >= S) return;
    float th[NM];
#pragma unroll
    for (int j = 0; j < NM; ++j) th[j] = j < n ? q[(int64_t)j * S + s] : 0.f;
    V3 P[NM], Z[NM];
    Frame ee;
    fk_chain<NM, true>(rb, n, th, P, Z, ee);
    const Quat qe = quat_of(ee);
    pose[s] = ee.p.x;
    pose[S + s] = ee.p.y;
    pose[2 * S + s] = ee.p.z;
    pose[3 * S + s] = qe.w;
    pose[4 * S + s] = qe.x;
    pose[5 * S + s] = qe.y;
    pose[6 * S + s] = qe.z;
    if (jac) {
#pragma unroll
        for (int j = 0; j < NM; ++j) {
            if (j < n) {
                const V3 l = cross(Z[j], ee.p - P[j]);
                const float c[6] = {l.x, l.y, l.z, Z[j].x, Z[j].y, Z[j].z};
#pragma unroll
                for (int r = 0; r < 6; ++r) jac[((int64_t)r * n + j) * S + s] = c[r];
            }
        }
    }
}

// ----------------------------------------------------------------------------
// Collision filter (Sec. IV-C).  One wave per block; every link frame of a
// lane goes to LDS ([link][12][64], lane fastest, conflict free).  For each
// link the coarse enclosing sphere is tested first and the link's fine
// spheres only when some lane's coarse test hits; a wave stops as soon as
// all its lanes collide.
// ----------------------------------------------------------------------------
// Link frames of the collision pass in LDS as (unit quaternion, origin):
// 7 floats per link and lane, [link][7][64] with the lane fastest (conflict
// free).  Rebuilding the rotation from the quaternion costs ~2e-7 relative,
// i.e. < 1e-7 m on a sphere centre, far inside the 1e-5 m contact band.
constexpr int kFrameFloats = 7;

__device__ __forceinline__ void lds_store_frame(float* lds, int l, int lane, const Frame& T) {
    float* b = lds + (l * kFrameFloats) * 64 + lane;
    const Quat q = quat_of<true>(T);
    b[0] = q.w;
    b[64] = q.x;
    b[128] = q.y;
    b[192] = q.z;
    b[256] = T.p.x;
    b[320] = T.p.y;
    b[384] = T.p.z;
}

__device__ __forceinline__ Frame lds_load_frame(const float* lds, int l, int lane) {
    const float* b = lds + (l * kFrameFloats) * 64 + lane;
    const float w = b[0], x = b[64], y = b[128], z = b[192];
    const float x2 = x + x, y2 = y + y, z2 = z + z;
    const float xx = x * x2, yy = y * y2, zz = z * z2;
    const float xy = x * y2, xz = x * z2, yz = y * z2;
    const float wx = w * x2, wy = w * y2, wz = w * z2;
    Frame T;
    T.X = mk(1.f - (yy + zz), xy + wz, xz - wy);
    T.Y = mk(xy - wz, 1.f - (xx + zz), yz + wx);
    T.Z = mk(xz + wy, yz - wx, 1.f - (xx + yy));
    T.p = mk(b[256], b[320], b[384]);
    return T;
}

__device__ __forceinline__ V3 xform(const Frame& T, float x, float y, float z) {
    return axpy(z, T.Z, axpy(y, T.Y, axpy(x, T.X, T.p)));
}

__device__ __forceinline__ float box_d2(V3 c, const float* __restrict__ b) {
    const float ex = fmaxf(0.f, fabsf(c.x - b[0]) - b[4]);
    const float ey = fmaxf(0.f, fabsf(c.y - b[1]) - b[5]);
    const float ez = fmaxf(0.f, fabsf(c.z - b[2]) - b[6]);
    return fmaf(ex, ex, fmaf(ey, ey, ez * ez));
}

__device__ __forceinline__ uint64_t wave_min_u64(uint64_t v);
__device__ __forceinline__ uint64_t cost_key(float c, uint32_t m);

constexpr int kObsGroup = 8;  // obstacles whose loads are issued together (measured: 1, 2, 4, 8)

// One environment sphere (centre co, radius ro) against link spheres f0 ..
// f0 + fc - 1 of the link with frame F, for the lanes whose coarse test `ch`
// hit; counts the coarse test of every lane not yet colliding.  Returns true
// when every lane of the wave collides (the caller stops).
__device__ __forceinline__ bool sphere_obstacle(const DevRobot* __restrict__ rb, const Frame& F, int f0, int fc,
                                                V3 co, float ro, bool ch, bool& hit, uint32_t& n_coarse,
                                                uint32_t& n_fine) {
    n_coarse += hit ? 0u : 1u;
    if (!wave_any(ch)) return false;
    for (int k = 0; k < fc; ++k) {
        const float* sp = rb->sph[f0 + k];
        if (ch && !hit) {
            const V3 c = xform(F, sp[0], sp[1], sp[2]);
            const V3 df = c - co;
            const float r2 = sp[3] + ro;
            ++n_fine;
            if (dot(df, df) < r2 * r2) hit = true;
        }
    }
    return wave_all(hit);
}

// One environment box (centre b[0..2], half extents b[4..6]) against the
// link spheres, for the lanes whose coarse test `ch` hit.
__device__ __forceinline__ void box_obstacle(const DevRobot* __restrict__ rb, const Frame& F, int f0, int fc,
                                             const float* __restrict__ b, bool ch, bool& hit, uint32_t& n_coarse,
                                             uint32_t& n_fine) {
    n_coarse += hit ? 0u : 1u;
    if (!wave_any(ch)) return;
    for (int k = 0; k < fc; ++k) {
        const float* sp = rb->sph[f0 + k];
        if (ch && !hit) {
            const V3 c = xform(F, sp[0], sp[1], sp[2]);
            ++n_fine;
            if (box_d2(c, b) < sp[3] * sp[3]) hit = true;
        }
    }
}

__device__ __forceinline__ int wave_max_i32(int v) {
#pragma unroll
    for (int o = 32; o > 0; o >>= 1) v = max(v, __shfl_xor(v, o, 64));
    return v;
}

// The obstacles of the grid cell holding this lane's coarse centre cc
// (radius Rc <= the grid's margin) against the link's spheres f0 .. f0 + fc
// - 1 (frame F): coarse test per listed obstacle, fine tests for the lanes
// whose coarse test hit.  Every obstacle the flat loops would find touching
// is listed, so the flag is the same.
__device__ __forceinline__ void grid_obstacles(const DevRobot* __restrict__ rb, const ObstacleGrid& g, const Frame& F,
                                               int f0, int fc, V3 cc, float Rc, const float* __restrict__ os,
                                               int n_osph, const float* __restrict__ ob, bool& hit,
                                               uint32_t& n_coarse, uint32_t& n_fine) {
    int32_t c0 = 0, len = 0;
    if (!hit) {
        const int ix = (int)floorf((cc.x - g.lo[0]) * g.inv_h);
        const int iy = (int)floorf((cc.y - g.lo[1]) * g.inv_h);
        const int iz = (int)floorf((cc.z - g.lo[2]) * g.inv_h);
        if (ix >= 0 && ix < g.n[0] && iy >= 0 && iy < g.n[1] && iz >= 0 && iz < g.n[2]) {
            const int64_t cell = ((int64_t)ix * g.n[1] + iy) * g.n[2] + iz;
            c0 = g.start[cell];
            len = g.start[cell + 1] - c0;
        }
    }
    const int steps = wave_max_i32(len);
    for (int i = 0; i < steps; ++i) {
        if (wave_all(hit)) break;
        const bool has = !hit && i < len;
        const int32_t o = has ? g.items[c0 + i] : 0;
        const bool sphere = o < n_osph;
        V3 co = mk(0.f, 0.f, 0.f);
        float ro = 0.f;
        const float* b = ob;
        bool ch = false;
        if (has) {
            if (sphere) {
                co = mk(os[4 * o], os[4 * o + 1], os[4 * o + 2]);
                ro = os[4 * o + 3];
                const V3 d = cc - co;
                const float rr = Rc + ro;
                ch = dot(d, d) < rr * rr;
            } else {
                b = ob + 8 * (o - n_osph);
                ch = box_d2(cc, b) < Rc * Rc;
            }
        }
        n_coarse += has ? 1u : 0u;
        if (!wave_any(ch)) continue;
        for (int k = 0; k < fc; ++k) {
            const float* sp = rb->sph[f0 + k];
            if (ch && !hit) {
                const V3 c = xform(F, sp[0], sp[1], sp[2]);
                ++n_fine;
                if (sphere) {
                    const V3 df = c - co;
                    const float r2 = sp[3] + ro;
                    if (dot(df, df) < r2 * r2) hit = true;
                } else if (box_d2(c, b) < sp[3] * sp[3]) {
                    hit = true;
                }
            }
        }
    }
}

// Collision test of one lane whose joint values are q[i * q_stride + s];
// inactive lanes count as done so the wave can leave early.  Returns the
// collision flag of an active lane.  ENV: the obstacle tests, link by link;
// SELF: every link frame to the wave's LDS rows and the self pairs after the
// walk.  A lane's tests, counts and early exits are those of the one-pass
// form whichever parts a call runs (a lane that collides stops testing; a
// wave leaves once all its lanes collide), so running ENV, then SELF on the
// lanes still free, gives the same flags and counters.
template <bool ENV = true, bool SELF = true>
__device__ __forceinline__ bool collide_lane(const DevRobot* __restrict__ rb, int n, float* lds, int lane,
                                             bool active, const float* __restrict__ q, int64_t q_stride,
                                             int64_t s, const float* __restrict__ os, int n_osph,
                                             const float* __restrict__ ob, int n_obox, const ObstacleGrid& g,
                                             uint32_t& n_coarse, uint32_t& n_fine) {
    bool hit = !active;
    // environment, link by link along the chain walk (the frame is in
    // registers); for the self pairs every frame is kept in LDS
    Frame F = identity_frame();
    for (int l = 0; l <= n; ++l) {
        if (l > 0) {
            const float th = active ? q[(int64_t)(l - 1) * q_stride + s] : 0.f;
            chain_step(rb, l - 1, th, F);
        }
        if (wave_all(hit)) break;  // the self pairs are skipped too
        if (SELF) lds_store_frame(lds, l, lane, F);
        if (!ENV) continue;
        const float Rc = rb->coarse[l][3];
        if (Rc < 0.f) continue;
        const V3 cc = xform(F, rb->coarse[l][0], rb->coarse[l][1], rb->coarse[l][2]);
        const int f0 = rb->link_first[l], fc = rb->link_count[l];
        if (g.start) {
            grid_obstacles(rb, g, F, f0, fc, cc, Rc, os, n_osph, ob, hit, n_coarse, n_fine);
            continue;
        }
        // Obstacles in groups of kObsGroup: the group's (uniform) loads and
        // coarse distances first, so the loads of a group are in flight
        // together, then the tests in obstacle order exactly as one at a time
        // (same flags, counters and early exits).
        bool stop = false;
        int o = 0;
        for (; o + kObsGroup <= n_osph && !stop; o += kObsGroup) {
            V3 co[kObsGroup];
            float ro[kObsGroup], d2[kObsGroup];
#pragma unroll
            for (int i = 0; i < kObsGroup; ++i) {
                const float* q4 = os + 4 * (o + i);
                co[i] = mk(q4[0], q4[1], q4[2]);
                ro[i] = q4[3];
                const V3 d = cc - co[i];
                d2[i] = dot(d, d);
            }
#pragma unroll
            for (int i = 0; i < kObsGroup; ++i) {
                const float rr = Rc + ro[i];
                if (sphere_obstacle(rb, F, f0, fc, co[i], ro[i], !hit && d2[i] < rr * rr, hit, n_coarse, n_fine)) {
                    stop = true;
                    break;
                }
            }
        }
        for (; o < n_osph && !stop; ++o) {
            const V3 co = mk(os[4 * o], os[4 * o + 1], os[4 * o + 2]);
            const float ro = os[4 * o + 3];
            const V3 d = cc - co;
            const float rr = Rc + ro;
            stop = sphere_obstacle(rb, F, f0, fc, co, ro, !hit && dot(d, d) < rr * rr, hit, n_coarse, n_fine);
        }
        o = 0;
        stop = wave_all(hit);
        for (; o + kObsGroup <= n_obox && !stop; o += kObsGroup) {
            float bd2[kObsGroup];
#pragma unroll
            for (int i = 0; i < kObsGroup; ++i) bd2[i] = box_d2(cc, ob + 8 * (o + i));
#pragma unroll
            for (int i = 0; i < kObsGroup; ++i) {
                if (wave_all(hit)) {
                    stop = true;
                    break;
                }
                box_obstacle(rb, F, f0, fc, ob + 8 * (o + i), !hit && bd2[i] < Rc * Rc, hit, n_coarse, n_fine);
            }
        }
        for (; o < n_obox && !wave_all(hit); ++o)
            box_obstacle(rb, F, f0, fc, ob + 8 * o, !hit && box_d2(cc, ob + 8 * o) < Rc * Rc, hit, n_coarse, n_fine);
    }
    // self collision on the allowed link pairs
    if (!SELF) return hit;
    for (int pi = 0; pi < rb->n_pairs && !wave_all(hit); ++pi) {
        const int la = rb->pair_a[pi], lb = rb->pair_b[pi];
        const Frame Fa = lds_load_frame(lds, la, lane);
        const Frame Fb = lds_load_frame(lds, lb, lane);
        const V3 ca = xform(Fa, rb->coarse[la][0], rb->coarse[la][1], rb->coarse[la][2]);
        const V3 cb = xform(Fb, rb->coarse[lb][0], rb->coarse[lb][1], rb->coarse[lb][2]);
        const V3 d = ca - cb;
        const float rr = rb->coarse[la][3] + rb->coarse[lb][3];
        const bool ch = !hit && dot(d, d) < rr * rr;
        n_coarse += hit ? 0u : 1u;
        if (wave_any(ch)) {
            const int fa = rb->link_first[la], na = rb->link_count[la];
            const int fb = rb->link_first[lb], nb = rb->link_count[lb];
            for (int i = 0; i < na; ++i) {
                const float* sa = rb->sph[fa + i];
                const V3 c1 = xform(Fa, sa[0], sa[1], sa[2]);
                for (int k = 0; k < nb; ++k) {
                    const float* sb = rb->sph[fb + k];
                    if (ch && !hit) {
                        const V3 c2 = xform(Fb, sb[0], sb[1], sb[2]);
                        const V3 df = c1 - c2;
                        const float r2 = sa[3] + sb[3];
                        ++n_fine;
                        if (dot(df, df) < r2 * r2) hit = true;
                    }
                }
            }
        }
    }
    return hit;
}

// Obstacle tests, one seed per lane: no LDS, so the occupancy is set by
// registers alone (the link frames of the self pairs, 7 floats per link and
// lane in LDS, would hold it to a few waves per CU on long chains).
__global__ __launch_bounds__(256) void k_collide_env(CollideArgs a) {
    const int lane = (int)(threadIdx.x & 63u);
    const int64_t s = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    const bool live = s < a.S;
    uint32_t n_coarse = 0, n_fine = 0;
    const bool hit = collide_lane<true, false>(a.rb, a.n, nullptr, lane, live, a.q, a.q_stride, s, a.osph,
                                               a.n_osph, a.obox, a.n_obox, a.grid, n_coarse, n_fine);
    if (live) a.flag[s] = hit ? 1 : 0;
    if (a.counters) {
        Counters c;
        c.coll_coarse = live ? n_coarse : 0u;
        c.coll_fine = live ? n_fine : 0u;
        flush_counters(c, a.counters, true);
    }
}

// Self pairs of the seeds the obstacle tests left free.  Wave w scans seeds
// [w P, (w + 1) P) 64 at a time and queues the free ones in LDS; each time
// 64 are queued it tests them, one per lane (frames to LDS, then the pairs),
// and the rest at the end, so the LDS-bound pass runs on full waves of the
// seeds that need it (on cluttered scenes a few percent).
constexpr int kSelfQueue = 128;

__global__ __launch_bounds__(64) void k_collide_self(CollideArgs a, int64_t P) {
    extern __shared__ float lds[];
    const int lane = (int)threadIdx.x;
    int32_t* queue = (int32_t*)(lds + (a.n + 1) * kFrameFloats * 64);  // [kSelfQueue], wave-local
    const int64_t b0 = (int64_t)blockIdx.x * P;
    const int64_t b1 = b0 + P < a.S ? b0 + P : a.S;
    uint32_t n_coarse = 0, n_fine = 0;
    int qn = 0;  // queued seeds (uniform)
    auto run = [&](int count) {
        const bool act = lane < count;
        const int64_t s = b0 + (act ? (int64_t)queue[lane] : 0);  // queued as offsets from b0
        const bool hit = collide_lane<false, true>(a.rb, a.n, lds, lane, act, a.q, a.q_stride, s, a.osph, a.n_osph,
                                                   a.obox, a.n_obox, a.grid, n_coarse, n_fine);
        if (act && hit) a.flag[s] = 1;
    };
    for (int64_t base = b0; base < b1; base += 64) {
        const int64_t s = base + lane;
        const bool free = s < b1 && a.flag[s] == 0;
        const uint64_t m = __ballot(free);
        if (free) queue[qn + __popcll(m & ((1ull << lane) - 1ull))] = (int32_t)(s - b0);
        qn += __popcll(m);  // qn < 64 before, so at most 127 entries
        wave_lds_sync();
        if (qn >= 64) {
            run(64);
            wave_lds_sync();
            const int rest = qn - 64;
            const int32_t t = lane < rest ? queue[64 + lane] : 0;
            wave_lds_sync();
            if (lane < rest) queue[lane] = t;
            qn = rest;
            wave_lds_sync();
        }
    }
    if (qn > 0) run(qn);
    if (a.counters) {
        Counters c;
        c.coll_coarse = n_coarse;
        c.coll_fine = n_fine;
        flush_counters(c, a.counters, true);
    }
}

// Serving: collision test of a chunk's blocks (one wave per block entry).
__global__ __launch_bounds__(64) void k_serve_check(ServeCheckArgs a) {
    extern __shared__ float lds[];
    const int e = blockIdx.x;
    const int lane = threadIdx.x;
    const ServeBlock blk = a.blocks[e];
    const int64_t s = (int64_t)blk.block * 64 + lane;
    const uint8_t st = a.st.sstate[s];
    const bool want = (st & SLOT_LIVE) && !(st & SLOT_RETIRED) && !(st & SLOT_CHECKED) &&
                      (a.all_lanes[e] || (st & SLOT_POL_FROZEN));
    uint32_t n_coarse = 0, n_fine = 0;
    const bool hit = collide_lane(a.rb, a.n, lds, lane, want, a.st.q, a.st.C, s, a.osph, a.n_osph, a.obox,
                                  a.n_obox, a.grid, n_coarse, n_fine);
    if (want) a.st.sstate[s] = (uint8_t)(st | SLOT_CHECKED | (hit ? SLOT_COLLIDES : 0));
}

// Serving: per-target decision, one wave per listed target.
__global__ __launch_bounds__(64) void k_serve_reduce(ServeReduceArgs a) {
    const int i = blockIdx.x;
    const int lane = threadIdx.x;
    const int64_t f = a.first_slot[i];
    const int32_t M = a.n_seeds[i];
    uint64_t best_ok = ~0ull, best_any = ~0ull;
    for (int32_t m = lane; m < M; m += 64) {
        const int64_t s = f + m;
        const uint8_t st = a.st.sstate[s];
        if (!(st & SLOT_CHECKED)) continue;
        const bool coll = (st & SLOT_COLLIDES) != 0;
        const uint64_t key = cost_key(a.st.cost[s], (uint32_t)m);
        if (!coll && a.st.err_p[s] <= a.succ_pos && a.st.err_o[s] <= a.succ_ori && key < best_ok) best_ok = key;
        const uint64_t kf = ((uint64_t)coll << 63) | key;
        if (kf < best_any) best_any = kf;
    }
    best_ok = wave_min_u64(best_ok);
    best_any = wave_min_u64(best_any);
    int32_t status = 0;
    uint64_t pick = ~0ull;
    if (best_ok != ~0ull) {
        status = 1;
        pick = best_ok;
    } else if (a.final_[i]) {
        status = 2;
        pick = best_any;
    }
    float* row = a.res + (int64_t)i * (a.n + 3);
    if (status != 0 && pick != ~0ull) {
        const int64_t s = f + (int64_t)(uint32_t)pick;
        if (lane < a.n) row[lane] = a.st.q[(int64_t)lane * a.st.C + s];
        if (lane == 0) {
            row[a.n] = a.st.err_p[s];
            row[a.n + 1] = a.st.err_o[s];
            row[a.n + 2] = (a.st.sstate[s] & SLOT_COLLIDES) ? 1.f : 0.f;
        }
    } else if (status != 0) {
        if (lane < a.n) row[lane] = 0.f;
        if (lane == 0) {
            row[a.n] = __builtin_inff();
            row[a.n + 1] = __builtin_inff();
            row[a.n + 2] = 255.f;
        }
    }
    if (lane == 0) a.status[i] = status;
    if (status != 0)
        for (int32_t m = lane; m < M; m += 64) a.st.sstate[f + m] |= SLOT_RETIRED;
}

// Serving: slot and target-table initialisation of admitted requests (one
// workgroup each).
__global__ __launch_bounds__(256) void k_serve_admit(const ServeAdmit* __restrict__ adm,
                                                     const float* __restrict__ up_pose, float* __restrict__ tgt_pose,
                                                     uint32_t* __restrict__ tgt_key, ServeState st) {
    const ServeAdmit r = adm[blockIdx.x];
    const int32_t live = r.n_targets * r.M;
    for (int32_t i = threadIdx.x; i < r.padded; i += blockDim.x) {
        const int64_t s = r.base + i;
        if (i < live) {
            st.sstate[s] = SLOT_LIVE;
            st.slot_target[s] = r.tbl0 + i / r.M;
            st.slot_m[s] = (uint32_t)(i % r.M);
        } else {
            st.sstate[s] = 0;
            st.slot_target[s] = 0;
            st.slot_m[s] = 0;
        }
    }
    for (int32_t k = threadIdx.x; k < r.n_targets; k += blockDim.x) {
        const float* src = up_pose + (int64_t)(r.up0 + k) * 7;
#pragma unroll
        for (int d = 0; d < 7; ++d) tgt_pose[(int64_t)d * st.Tc + r.tbl0 + k] = src[d];
        tgt_key[r.tbl0 + k] = r.key0 + (uint32_t)k;
    }
}

// ----------------------------------------------------------------------------
// Per-target ordering by 64-bit keys, one wave per target.  Keys are unique
// (they carry the seed index), so the r-th smallest key is the smallest key
// above the (r-1)-th: k rounds of a lane-strided scan and a wave minimum.
// ----------------------------------------------------------------------------
__device__ __forceinline__ uint64_t wave_min_u64(uint64_t v) {
#pragma unroll
    for (int o = 32; o > 0; o >>= 1) {
        const uint32_t lo = __shfl_xor((uint32_t)v, o, 64);
        const uint32_t hi = __shfl_xor((uint32_t)(v >> 32), o, 64);
        const uint64_t w = ((uint64_t)hi << 32) | lo;
        v = w < v ? w : v;
    }
    return v;
}

__device__ __forceinline__ uint64_t cost_key(float c, uint32_t m) {
    const uint32_t b = __float_as_uint(c) & 0x7FFFFFFFu;  // costs are >= 0
    return ((uint64_t)b << 32) | m;
}

// Key of the nearest-solution order: class (0: collision free within the
// success tolerances, 1: other collision-free seeds, 2: colliding) in bits
// 62-63, then the squared joint distance to the reference (class 0) or the
// cost (>= 0, sign bit dropped) in bits 31-61, then the seed index.
__device__ __forceinline__ uint64_t near_key(uint32_t cls, float v, uint32_t m) {
    const uint32_t b = __float_as_uint(v) & 0x7FFFFFFFu;
    return ((uint64_t)cls << 62) | ((uint64_t)b << 31) | (uint64_t)(m & 0x7FFFFFFFu);
}

// Final selection (Alg. HJCD-IK, last line): order (flag != 0, cost, index);
// with a reference configuration per target (a.q_ref), the tracking order of
// near_key.
__global__ __launch_bounds__(64) void k_select(SelectArgs a) {
    const int b = blockIdx.x;
    const int t = a.tperm ? a.tperm[b] : b;
    const int lane = threadIdx.x;
    const int64_t b0 = a.offsets[b];
    const int64_t M = a.offsets[b + 1] - b0;
    uint32_t nf = 0;
    for (int64_t m = lane; m < M; m += 64) nf += a.flag[b0 + m] == 0 ? 1u : 0u;
    nf = wave_sum(nf);
    uint64_t prev = 0;
    bool ok = false;
    for (int r = 0; r < a.k; ++r) {
        uint64_t best = ~0ull;
        for (int64_t m = lane; m < M; m += 64) {
            const int64_t sm = b0 + m;
            uint64_t key;
            if (a.q_ref) {
                const bool fr = a.flag[sm] == 0;
                const bool good = fr && a.err_p[sm] <= a.succ_pos && a.err_o[sm] <= a.succ_ori;
                float v = a.cost[sm];
                if (good) {
                    v = 0.f;
                    for (int j = 0; j < a.n; ++j) {
                        const float d = a.q[(int64_t)j * a.S + sm] - a.q_ref[(int64_t)t * a.n_stride + j];
                        v = fmaf(d, d, v);
                    }
                }
                key = near_key(good ? 0u : (fr ? 1u : 2u), v, (uint32_t)m);
            } else {
                key = ((uint64_t)(a.flag[sm] != 0) << 63) | cost_key(a.cost[sm], (uint32_t)m);
            }
            if ((r == 0 || key > prev) && key < best) best = key;
        }
        best = wave_min_u64(best);
        const int64_t o = (int64_t)t * a.k + r;
        if (best == ~0ull) {
            if (lane < a.n_stride) a.q_out[o * a.n_stride + lane] = 0.f;
            if (lane == 0) {
                a.ep_out[o] = __builtin_inff();
                a.eo_out[o] = __builtin_inff();
                a.fl_out[o] = 255;
            }
            continue;
        }
        prev = best;
        const int64_t s = b0 + (int64_t)(a.q_ref ? (uint32_t)(best & 0x7FFFFFFFull) : (uint32_t)best);
        if (lane < a.n_stride) a.q_out[o * a.n_stride + lane] = lane < a.n ? a.q[(int64_t)lane * a.S + s] : 0.f;
        const float ep = a.err_p[s], eo = a.err_o[s];
        const uint8_t fl = a.flag[s];
        if (lane == 0) {
            a.ep_out[o] = ep;
            a.eo_out[o] = eo;
            a.fl_out[o] = fl;
        }
        ok = ok || (fl == 0 && ep <= a.succ_pos && eo <= a.succ_ori);
    }
    if (lane == 0) {
        a.n_free[t] = (int32_t)nf;
        a.solved[t] = ok ? 1 : 0;
    }
}

// Mid top-K ranking (Alg. HJCD-IK): K smallest (cost, index) per target.
__global__ __launch_bounds__(64) void k_rank(int32_t T, const int64_t* __restrict__ offsets,
                                             const float* __restrict__ cost, int32_t K,
                                             int32_t* __restrict__ rank) {
    const int t = blockIdx.x;
    const int lane = threadIdx.x;
    const int64_t b0 = offsets[t];
    const int64_t M = offsets[t + 1] - b0;
    uint64_t prev = 0;
    for (int r = 0; r < K; ++r) {
        if (r >= M) {
            if (lane == 0) rank[(int64_t)t * K + r] = M > 0 ? rank[(int64_t)t * K + (r % M)] : -1;
            continue;
        }
        uint64_t best = ~0ull;
        for (int64_t m = lane; m < M; m += 64) {
            const uint64_t key = cost_key(cost[b0 + m], (uint32_t)m);
            if ((r == 0 || key > prev) && key < best) best = key;
        }
        best = wave_min_u64(best);
        prev = best;
        if (lane == 0) rank[(int64_t)t * K + r] = (int32_t)(uint32_t)best;
    }
}

// Noisy copies: slot b*Bp + i*K + kk <- clip(q[rank kk] + mu + sigma z).
template <int NM>
__global__ __launch_bounds__(256) void k_replicate(const DevRobot* __restrict__ rb, int n, int32_t tb,
                                                   int32_t te, const int64_t* __restrict__ offsets,
                                                   const int32_t* __restrict__ tperm, int64_t S_in,
                                                   const float* __restrict__ q_in,
                                                   const int32_t* __restrict__ rank, int32_t K, int32_t Bp,
                                                   const uint32_t* __restrict__ tkeys, uint64_t seed,
                                                   float mu, float sigma, float* __restrict__ q_out,
                                                   int64_t Sout) {
    const int64_t v = (int64_t)tb * Bp + (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (v >= (int64_t)te * Bp) return;
    const int32_t b = (int32_t)(v / Bp);
    const int32_t j = (int32_t)(v % Bp);
    const int32_t kk = j % K;
    const int64_t src = offsets[b] + rank[(int64_t)b * K + kk];
    const int32_t t = tperm ? tperm[b] : b;
    float th[NM];
#pragma unroll
    for (int i = 0; i < NM; ++i) th[i] = i < n ? q_in[(int64_t)i * S_in + src] : 0.f;
    perturb<NM>(rb, n, th, seed, (uint32_t)j, tkeys ? tkeys[t] : (uint32_t)t, STAGE_RESAMPLE, 0, mu, sigma);
#pragma unroll
    for (int i = 0; i < NM; ++i)
        if (i < n) q_out[(int64_t)i * Sout + v] = th[i];
}

// Warm start on a path: seed m of target t starts at previous solution
// m mod k (row t*k + m%k of q_prev [T*k][n_stride]), clipped to the limits,
// and for m >= k moved by clip(. + mu + sigma z), z drawn for seed index m at
// stage WARM.  q_out [n][T*M].
template <int NM>
__global__ __launch_bounds__(256) void k_warm(const DevRobot* __restrict__ rb, int n, int32_t T, int32_t k,
                                              int32_t n_stride, const float* __restrict__ q_prev, int32_t M,
                                              const uint32_t* __restrict__ tkeys, uint64_t seed, float mu,
                                              float sigma, float* __restrict__ q_out) {
    const int64_t v = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    const int64_t S = (int64_t)T * M;
    if (v >= S) return;
    const int32_t t = (int32_t)(v / M);
    const int32_t m = (int32_t)(v % M);
    const int64_t src = ((int64_t)t * k + m % k) * n_stride;
    float th[NM];
#pragma unroll
    for (int i = 0; i < NM; ++i) th[i] = i < n ? clampf(q_prev[src + i], rb->lo[i], rb->hi[i]) : 0.f;
    if (m >= k)
        perturb<NM>(rb, n, th, seed, (uint32_t)m, tkeys ? tkeys[t] : (uint32_t)t, STAGE_WARM, 0, mu, sigma);
#pragma unroll
    for (int i = 0; i < NM; ++i)
        if (i < n) q_out[(int64_t)i * S + v] = th[i];
}

// Caller layout -> robot-grouped layout.
__global__ __launch_bounds__(256) void k_gather(int n, int32_t T, const int64_t* __restrict__ offsets,
                                                const int64_t* __restrict__ voffs,
                                                const int32_t* __restrict__ tperm, int64_t S,
                                                int64_t in_stride, const float* __restrict__ q_in,
                                                float* __restrict__ q_out) {
    const int64_t v = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (v >= S) return;
    const int32_t b = last_le(voffs, T, v);
    const int32_t t = tperm ? tperm[b] : b;
    const int64_t src = offsets[t] + (v - voffs[b]);
    for (int i = 0; i < n; ++i) q_out[(int64_t)i * S + v] = q_in[(int64_t)i * in_stride + src];
}

__global__ void k_philox(uint32_t c0, uint32_t c1, uint32_t c2, uint32_t c3, uint32_t k0, uint32_t k1,
                         int64_t count, uint32_t* __restrict__ out) {
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= count) return;
    const U4 r = philox(U4{c0 + (uint32_t)i, c1, c2, c3}, k0, k1);
    out[4 * i] = r.a;
    out[4 * i + 1] = r.b;
    out[4 * i + 2] = r.c;
    out[4 * i + 3] = r.d;
}

// ----------------------------------------------------------------------------
// launchers
// ----------------------------------------------------------------------------
static inline unsigned blocks_for(int64_t count, int per) { return (unsigned)((count + per - 1) / per); }

#define HJCD_DISPATCH_NM(n, CALL) \
    do {                          \
        if ((n) <= 8) {           \
            CALL(8);              \
        } else if ((n) <= 16) {   \
            CALL(16);             \
        } else if ((n) <= 24) {   \
            CALL(24);             \
        } else {                  \
            CALL(32);             \
        }                         \
    } while (0)

// The per-seed solve kernels come in finer buckets: exact 6- and 7-joint
// instances, then bounds 8, 12, 16, 20, 24, 32 (a bucket's arrays take
// registers for all its joints, so the padding costs occupancy).
#define HJCD_DISPATCH_SOLVE(n, CALL) \
    do {                             \
        if ((n) == 6) {              \
            CALL(6);                 \
        } else if ((n) == 7) {       \
            CALL(7);                 \
        } else if ((n) <= 8) {       \
            CALL(8);                 \
        } else if ((n) <= 12) {      \
            CALL(12);                \
        } else if ((n) <= 16) {      \
            CALL(16);                \
        } else if ((n) <= 20) {      \
            CALL(20);                \
        } else if ((n) <= 24) {      \
            CALL(24);                \
        } else {                     \
            CALL(32);                \
        }                            \
    } while (0)

template <int NM>
hipError_t launch_solve_nm(const SolveArgs& a, hipStream_t st);

hipError_t launch_solve(const SolveArgs& a, hipStream_t st) {
    if (a.map.Sv <= 0) return hipSuccess;
#define L_SOLVE(NMV) return launch_solve_nm<NMV>(a, st)
    HJCD_DISPATCH_SOLVE(a.n, L_SOLVE);
#undef L_SOLVE
}

hipError_t launch_fk(const DevRobot* rb, int n, int64_t S, const float* q, float* pose, float* jac,
                     hipStream_t st) {
    if (S <= 0) return hipSuccess;
    const unsigned nb = blocks_for(S, 256);
#define L_FK(NMV) hipLaunchKernelGGL(k_fk<NMV>, dim3(nb), dim3(256), 0, st, rb, n, S, q, pose, jac)
    HJCD_DISPATCH_NM(n, L_FK);
#undef L_FK
    return hipGetLastError();
}

hipError_t launch_collide(const CollideArgs& a, hipStream_t st) {
    if (a.S <= 0) return hipSuccess;
    hipLaunchKernelGGL(k_collide_env, dim3(blocks_for(a.S, 256)), dim3(256), 0, st, a);
    if (a.n_pairs <= 0) return hipGetLastError();
    // scanning waves: four rounds of what the LDS lets a 256-CU part hold at
    // once (160 KB per CU), each scanning a 64-seed multiple
    const size_t lds = (size_t)(a.n + 1) * kFrameFloats * 64 * sizeof(float) + kSelfQueue * sizeof(int32_t);
    const int64_t per_cu = (int64_t)((160u << 10) / lds) < 1 ? 1 : (int64_t)((160u << 10) / lds);
    const int64_t cap = 256 * per_cu * 4;
    const int64_t waves = (a.S + 63) / 64 < cap ? (a.S + 63) / 64 : cap;
    const int64_t P = ((a.S + waves - 1) / waves + 63) / 64 * 64;
    const unsigned nb = (unsigned)((a.S + P - 1) / P);
    hipLaunchKernelGGL(k_collide_self, dim3(nb), dim3(64), lds, st, a, P);
    return hipGetLastError();
}

template <int NM>
hipError_t launch_serve_chunk_nm(const ServeChunkArgs& a, hipStream_t st);

hipError_t launch_serve_chunk(const ServeChunkArgs& a, hipStream_t st) {
    if (a.nb <= 0) return hipSuccess;
#define L_CHUNK(NMV) return launch_serve_chunk_nm<NMV>(a, st)
    HJCD_DISPATCH_SOLVE(a.n, L_CHUNK);
#undef L_CHUNK
}

hipError_t launch_serve_check(const ServeCheckArgs& a, hipStream_t st) {
    if (a.nb <= 0) return hipSuccess;
    const size_t lds = (size_t)(a.n + 1) * kFrameFloats * 64 * sizeof(float);
    hipLaunchKernelGGL(k_serve_check, dim3(a.nb), dim3(64), lds, st, a);
    return hipGetLastError();
}

hipError_t launch_serve_reduce(const ServeReduceArgs& a, hipStream_t st) {
    if (a.nt <= 0) return hipSuccess;
    hipLaunchKernelGGL(k_serve_reduce, dim3(a.nt), dim3(64), 0, st, a);
    return hipGetLastError();
}

hipError_t launch_serve_admit(const ServeAdmit* adm, int32_t n_adm, const float* up_pose, float* tgt_pose,
                              uint32_t* tgt_key, ServeState sst, hipStream_t st) {
    if (n_adm <= 0) return hipSuccess;
    hipLaunchKernelGGL(k_serve_admit, dim3(n_adm), dim3(256), 0, st, adm, up_pose, tgt_pose, tgt_key, sst);
    return hipGetLastError();
}

hipError_t launch_select(const SelectArgs& a, hipStream_t st) {
    if (a.T <= 0) return hipSuccess;
    hipLaunchKernelGGL(k_select, dim3(a.T), dim3(64), 0, st, a);
    return hipGetLastError();
}

hipError_t launch_rank(int32_t T, const int64_t* offsets, const float* cost, int32_t K, int32_t* rank,
                       hipStream_t st) {
    if (T <= 0) return hipSuccess;
    hipLaunchKernelGGL(k_rank, dim3(T), dim3(64), 0, st, T, offsets, cost, K, rank);
    return hipGetLastError();
}

hipError_t launch_replicate(const DevRobot* rb, int n, int32_t tb, int32_t te, int32_t T,
                            const int64_t* offsets, const int32_t* tperm, int64_t S_in,
                            const float* q_in, const int32_t* rank, int32_t K, int32_t Bp,
                            const uint32_t* tkeys, uint64_t seed, float mu, float sigma, float* q_out,
                            hipStream_t st) {
    const int64_t cnt = (int64_t)(te - tb) * Bp;
    if (cnt <= 0) return hipSuccess;
    const int64_t Sout = (int64_t)T * Bp;
    const unsigned nb = blocks_for(cnt, 256);
#define L_REP(NMV)                                                                                  \
    hipLaunchKernelGGL(k_replicate<NMV>, dim3(nb), dim3(256), 0, st, rb, n, tb, te, offsets, tperm, \
                       S_in, q_in, rank, K, Bp, tkeys, seed, mu, sigma, q_out, Sout)
    HJCD_DISPATCH_NM(n, L_REP);
#undef L_REP
    return hipGetLastError();
}

hipError_t launch_warm(const DevRobot* rb, int n, int32_t T, int32_t k, int32_t n_stride, const float* q_prev,
                       int32_t M, const uint32_t* tkeys, uint64_t seed, float mu, float sigma, float* q_out,
                       hipStream_t st) {
    const int64_t S = (int64_t)T * M;
    if (S <= 0) return hipSuccess;
    const unsigned nb = blocks_for(S, 256);
#define L_WARM(NMV)                                                                                       \
    hipLaunchKernelGGL(k_warm<NMV>, dim3(nb), dim3(256), 0, st, rb, n, T, k, n_stride, q_prev, M, tkeys, \
                       seed, mu, sigma, q_out)
    HJCD_DISPATCH_NM(n, L_WARM);
#undef L_WARM
    return hipGetLastError();
}

hipError_t launch_gather(int n, int32_t T, const int64_t* offsets, const int64_t* voffs,
                         const int32_t* tperm, int64_t S, int64_t in_stride, const float* q_in,
                         float* q_out, hipStream_t st) {
    if (S <= 0) return hipSuccess;
    hipLaunchKernelGGL(k_gather, dim3(blocks_for(S, 256)), dim3(256), 0, st, n, T, offsets, voffs, tperm, S,
                       in_stride, q_in, q_out);
    return hipGetLastError();
}

hipError_t launch_philox(uint32_t c0, uint32_t c1, uint32_t c2, uint32_t c3, uint32_t k0, uint32_t k1,
                         int64_t count, uint32_t* out, hipStream_t st) {
    if (count <= 0) return hipSuccess;
    hipLaunchKernelGGL(k_philox, dim3(blocks_for(count, 256)), dim3(256), 0, st, c0, c1, c2, c3, k0, k1,
                       count, out);
    return hipGetLastError();
}

}  // namespace hjcd
