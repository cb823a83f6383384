// Hierarchy construction on the host (see build.cpp).
#pragma once

#include "host.hpp"

namespace ldgs {

void eval_field(const ldgs_field& f, int d, int64_t n, const double* x, const int* phase, double* out);
void build_fine_level(const ldgs_problem& P, const Geometry& g, const Basis& B, Level& L);
void coarsen_level(const ldgs_problem& P, const Geometry& g, const Basis& B, const Level& F, Level& C);
void set_scaling(Level& L, const Geometry& g);
int colour_count(int scheme, int d);
bool colouring_is_proper(const Level& L, int d, int scheme, int gamma, int64_t* bad_e);
void set_colouring(Level& L, int d, int scheme);

}  // namespace ldgs
