// Internal helpers shared by the host-side translation units.
#pragma once
#include <string>
#include <vector>

#include "../../include/fetiF.h"
#include "host_sparse.hpp"

namespace fetif {

bool pattern_from_sub(const fetiF_subdomain& s, Pattern& A, std::string& err);
void options_defaults(const fetiF_options* in, fetiF_options& o);
// flags[node] = 1 for every node holding a DOF that carries a Lagrange
// multiplier (b_dof); false if a b_dof is out of range
bool multiplier_nodes(const fetiF_subdomain& s, std::vector<char>& flags);

}  // namespace fetif
