// Internal interface of the quad-precision FC-Gram builder.
#pragma once
#include <vector>

namespace fcs {
// Q (d x d) Gram basis values at the matching points and A (C x d)
// continuation values, row-major; false on unsupported (d, C).
bool fc_continuation(int d, int C, double* Q, double* A);
// Dense n x n FC operator (kind 0: first derivative, 1: second derivative,
// both in index units; 2: filter; 3: smearing filter), row t / column s,
// cached; nullptr on
// unsupported arguments.
const std::vector<double>* fc_operator(int n, int d, int C, int kind);
}  // namespace fcs

namespace fcs {
// 16 x 16 orthonormal discrete polynomial basis (row = point, column = degree).
void modal_basis16(double* out);
}  // namespace fcs
