// Host-side coupling tensors and path enumeration.
#pragma once
#include <vector>

namespace mpip {

struct Path {
  int l1, l2, l3;
};

double wigner3j(int j1, int j2, int j3, int m1, int m2, int m3);
bool natural_path(int l1, int l2, int l3);
// Frobenius-normalised real Gaunt tensor, row-major (m1, m2, m3); false if
// the triple is not a natural-parity path with degrees <= 2.
bool coupling_tensor(int l1, int l2, int l3, double* out);
// Paths of layer t (1-based): l1 over the input degrees ({0} at t = 1, else
// 0..l_max), then l2, then l3, ascending -- the column order of W3.
std::vector<Path> layer_paths(int t, int l_max);

}  // namespace mpip
