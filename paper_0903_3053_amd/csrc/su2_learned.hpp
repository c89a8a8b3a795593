// su2_learned.hpp -- what the lattice context needs from the learned-proposal module.
#pragma once

#include <stdint.h>

// Parameters of the network 1 -> 64 -> 64 -> 33.
constexpr int kLearnedParams = 64 + 64 + 64 * 64 + 64 + 33 * 64 + 33;  // 6433

// The current knot table of the network (device [G][33], knots at alpha_g =
// g * alpha_max / (G - 1)); false if none was tabulated.
bool su2_learned_table(const float **knots, uint32_t *G, float *alpha_max);
const char *su2_learned_error();
