// Device-resident robot table of libhjcd.  Built once on the host by
// hjcd_load_robot and read by the kernels with wave-uniform indices only, so
// every field reaches the lanes through scalar loads.
#pragma once

#include <stdint.h>

#include "../../include/hjcd.h"

namespace hjcd {

constexpr int kMaxLinks = HJCD_MAX_DOF + 1;
constexpr int kMaxPairs = kMaxLinks * (kMaxLinks - 1) / 2;

struct alignas(16) DevRobot {
    int32_t n;          // joints
    int32_t conv;       // 0 modified DH, 1 standard DH
    int32_t tool_rot;   // tool rotation differs from identity
    int32_t n_sph;      // link spheres
    int32_t n_pairs;    // self-collision link pairs
    int32_t pad[3];
    // per joint
    float off[HJCD_MAX_DOF], lo[HJCD_MAX_DOF], hi[HJCD_MAX_DOF];
    float ca[HJCD_MAX_DOF], sa[HJCD_MAX_DOF], a[HJCD_MAX_DOF], d[HJCD_MAX_DOF];
    float px[HJCD_MAX_DOF], py[HJCD_MAX_DOF], pz[HJCD_MAX_DOF];  // modified DH: (a, -d sa, d ca)
    float tool[12];                                            // row-major 3 x 4
    // per link (0..n): spheres sorted by link
    int32_t link_first[kMaxLinks], link_count[kMaxLinks];
    float coarse[kMaxLinks][4];  // enclosing sphere in the link frame (x, y, z, R), R < 0: none
    // self-collision link pairs (la < lb, lb - la >= gap, both with spheres)
    uint8_t pair_a[kMaxPairs], pair_b[kMaxPairs];
    float sph[HJCD_MAX_SPHERES][4];  // x, y, z, r in the link frame
};

}  // namespace hjcd
