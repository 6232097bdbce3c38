// Internal declarations shared by the host toolkit and the device runtime of
// libswe.so.  Not part of the public ABI (include/swe.h).
#pragma once

#include <cstdint>
#include <string>
#include <vector>

#include "../../include/swe.h"

// A sub-domain as the host toolkit builds it (swe_subdomain_view gives the
// arrays): local numbering, ghost layers, neighbour table, peers and lists.
struct swe_subdomain {
    int32_t n_owned = 0, n_total = 0, n_peers = 0, n_send = 0;
    std::vector<int32_t> l2g, layer, owner, nbr, peers, recv_off, send_off, send_idx;
};

namespace swe {

// Packed per-cell word (4th int of the neighbour quad):
//   bits 0..5   local edge index, in the neighbour, of the shared edge (2 bits per edge)
//   bits 6..8   edge m is oriented with this cell as the L side (smaller global id)
//   bit  9      owned cell (counts in the CFL reduction)
//   bits 16..31 scenario index (batched ensembles; 0 otherwise)
constexpr int kOwnedBit = 9;
constexpr int kScenShift = 16;
constexpr int kMaxScenarios = 1 << 15;

// Geometry of one mesh prepared on the host in double precision.
struct HostGeometry {
    std::vector<double> cell;    // [4*n]  inv_area, inradius, manning^2, 0
    std::vector<double> he_geo;  // [12*n] per half-edge: nx, ny, L, d_mid
    std::vector<double> he_dist; // [12*n] per half-edge: 1/d_up, 1/d_fwd, 1/d_central, d_fwd
    std::vector<int32_t> nbr4;   // [4*n]  nbr0, nbr1, nbr2, packed word
    double inflow_length = 0.0;  // sum of SWE_BC_INFLOW edge lengths over owned cells
};

// Validates the mesh and fills g.  Returns SWE_OK or SWE_ERR_MESH with msg.
int prepare_geometry(const swe_mesh &m, int scenario, HostGeometry &g, std::string &msg);

}  // namespace swe
