// Host half of the proximity queries of geometry processing (the area queries of
// Algorithms 1 and 2): validation, a uniform cell grid and the counting sort of the points
// into it, shared by the entry points that run the device query.
#pragma once

#include <cstdint>
#include <string>
#include <vector>

#include "../../include/gigaqbx.h"
#include "kernels.hpp"

namespace gq {

struct NearQuery {
  AssocGrid g{};
  std::vector<int64_t> start;             // cell c holds sorted points [start[c], start[c+1])
  std::vector<double> px, py, pz;         // points in cell order
  std::vector<double> qx, qy, qz;         // queries, structure of arrays
};

// Validates the arguments of gq_points_near and fills Q with a grid of at most max_cells
// cells.  done is set when no device work is needed (no queries; or no points, in which
// case every flag of hit is set to 0).
gq_status near_prepare(int64_t n_q, const double* q_xyz, const double* radius, int64_t n_p,
                       const double* p_xyz, uint8_t* hit, int64_t max_cells, NearQuery& Q,
                       bool& done);

// Records the thread-local message returned by gq_last_error and returns st.
gq_status set_error(gq_status st, const std::string& msg);

}  // namespace gq
