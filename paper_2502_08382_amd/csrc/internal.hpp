// Internal helpers shared by the host-side translation units.
#pragma once
#include <string>

#include "../../include/fetiF.h"
#include "host_sparse.hpp"

namespace fetif {

bool pattern_from_sub(const fetiF_subdomain& s, Pattern& A, std::string& err);
void options_defaults(const fetiF_options* in, fetiF_options& o);

}  // namespace fetif
