// Host check of the hierarchy construction under the address and undefined-
// behaviour sanitizers: for a set of grid shapes, build the hierarchy and
// check what the operator must satisfy.  Prints "ok" and returns 0 when every
// check holds.
#include <cmath>
#include <cstdio>
#include <vector>

#include "../../paper_1904_03808_amd/csrc/hierarchy.h"
#include "../../paper_1904_03808_amd/csrc/packed_stencil.h"

namespace {

int oidx(int oz, int oy, int ox) { return (oz + 1) * 9 + (oy + 1) * 3 + (ox + 1); }

bool check_level(const qs::HostLevel& L, int level) {
  const int nz = L.nz;
  const double* S = L.stencil.data();
  double scale = 0.0;
  for (double v : L.stencil) scale = std::fmax(scale, std::fabs(v));
  // wall rows are zero
  for (int e = 0; e < qs::kStencil; ++e)
    if (S[e] != 0.0 || S[static_cast<size_t>(nz) * qs::kStencil + e] != 0.0) {
      std::printf("level %d: nonzero wall row\n", level);
      return false;
    }
  // symmetry of K: the block from (k) to (k+oz, o) is the transpose of the
  // block from (k+oz) back to (k, -o), for interior planes on both ends
  for (int k = 1; k < nz; ++k)
    for (int oz = -1; oz <= 1; ++oz) {
      const int k2 = k + oz;
      if (k2 < 1 || k2 > nz - 1) continue;
      for (int oy = -1; oy <= 1; ++oy)
        for (int ox = -1; ox <= 1; ++ox)
          for (int c = 0; c < 3; ++c)
            for (int d = 0; d < 3; ++d) {
              const double a = S[static_cast<size_t>(k) * qs::kStencil + oidx(oz, oy, ox) * 9 + c * 3 + d];
              const double b = S[static_cast<size_t>(k2) * qs::kStencil + oidx(-oz, -oy, -ox) * 9 + d * 3 + c];
              if (std::fabs(a - b) > 1e-12 * scale) {
                std::printf("level %d: asymmetric at k=%d o=(%d,%d,%d) c=%d d=%d\n", level, k, oz, oy,
                            ox, c, d);
                return false;
              }
            }
    }
  // dinv is the inverse of the centre block
  for (int k = 1; k < nz; ++k) {
    const double* A = S + static_cast<size_t>(k) * qs::kStencil + oidx(0, 0, 0) * 9;
    const double* X = L.dinv.data() + static_cast<size_t>(k) * 9;
    for (int r = 0; r < 3; ++r)
      for (int c = 0; c < 3; ++c) {
        double s = 0.0;
        for (int m = 0; m < 3; ++m) s += A[r * 3 + m] * X[m * 3 + c];
        if (std::fabs(s - (r == c ? 1.0 : 0.0)) > 1e-12) {
          std::printf("level %d: centre inverse off at k=%d\n", level, k);
          return false;
        }
      }
  }
  return true;
}

// The packed form (packed_stencil.h) of every plane: the entries it keeps
// are the stencil's, in order, 150 per plane, with the inverse and the centre
// diagonal after them; the entries it leaves out (couplings between
// different components where the offset along one of them is zero, which
// vanish in exact arithmetic) are below 1e-14 of
// the largest entry; and a planted non-zero in a left-out place is refused.
bool check_packing(const qs::HostLevel& L, int level) {
  std::vector<double> P;
  if (!qs::pack_level(L, &P)) {
    std::printf("level %d: pack_level refused the hierarchy\n", level);
    return false;
  }
  double scale = 0.0;
  for (double v : L.stencil) scale = std::fmax(scale, std::fabs(v));
  for (int k = 1; k < L.nz; ++k) {
    const double* S = L.stencil.data() + static_cast<size_t>(k) * qs::kStencil;
    const double* Q = P.data() + static_cast<size_t>(k) * qs::kPackedStencil;
    int n = 0;
    for (int oz = 0; oz < 3; ++oz)
      for (int oy = 0; oy < 3; ++oy)
        for (int ox = 0; ox < 3; ++ox)
          for (int c = 0; c < 3; ++c)
            for (int d = 0; d < 3; ++d) {
              const double v = S[(oz * 9 + oy * 3 + ox) * 9 + c * 3 + d];
              const bool centre = oz == 1 && oy == 1 && ox == 1;
              bool good = true;
              if (centre && c == d)
                good = Q[qs::kPackedCentre + c] == v;
              else if (!centre && qs::packed_used(oz, oy, ox, c, d))
                good = Q[n++] == v;
              else
                good = std::fabs(v) <= 1e-14 * scale;
              if (!good) {
                std::printf("level %d: packed entry wrong at k=%d o=(%d,%d,%d) c=%d d=%d\n", level, k,
                            oz, oy, ox, c, d);
                return false;
              }
            }
    if (n != qs::kPackedEntries) {
      std::printf("level %d: %d packed entries\n", level, n);
      return false;
    }
    for (int e = 0; e < 9; ++e)
      if (Q[qs::kPackedInv + e] != L.dinv[static_cast<size_t>(k) * 9 + e]) {
        std::printf("level %d: packed inverse wrong at k=%d\n", level, k);
        return false;
      }
  }
  // an x-y coupling at the face offset (0, 0, +1) may not be packed away
  qs::HostLevel bad = L;
  const int k = L.nz / 2;
  bad.stencil[static_cast<size_t>(k) * qs::kStencil + (2 * 9 + 1 * 3 + 1) * 9 + 0 * 3 + 1] = 1e-6 * scale;
  if (qs::pack_level(bad, &P)) {
    std::printf("level %d: a planted coupling was packed away\n", level);
    return false;
  }
  return true;
}

}  // namespace

int main() {
  const double lam = 0.35 / (1.35 * 0.3), mu = 1.0 / 2.7;
  struct Shape {
    int nx, ny, nz, mc;
  };
  const Shape shapes[] = {{16, 16, 16, 8},  {32, 32, 32, 4},  {24, 20, 20, 8}, {40, 24, 32, 4},
                          {64, 64, 32, 4},  {80, 80, 40, 8},  {12, 10, 2, 8},  {48, 48, 12, 4},
                          {128, 10, 8, 4},  {16, 16, 64, 16}, {96, 96, 96, 8}};
  for (const Shape& s : shapes) {
    qs::HostHierarchy H;
    const int rc = qs::build_hierarchy(s.nx, s.ny, s.nz, 1.0 / s.nz, lam, mu, s.mc, &H);
    if (rc != 0) {
      std::printf("shape %d x %d x %d: build returned %d\n", s.nx, s.ny, s.nz, rc);
      return 1;
    }
    for (size_t l = 0; l < H.levels.size(); ++l)
      if (!check_level(H.levels[l], static_cast<int>(l)) ||
          !check_packing(H.levels[l], static_cast<int>(l)))
        return 1;
    const int n = H.n_coarse;
    for (int r = 0; r < n; ++r)
      for (int c = 0; c < r; ++c)
        if (std::fabs(H.coarse_inv[static_cast<size_t>(r) * n + c] -
                      H.coarse_inv[static_cast<size_t>(c) * n + r]) >
            1e-9 * std::fabs(H.coarse_inv[static_cast<size_t>(r) * n + r])) {
          std::printf("shape %d x %d x %d: coarse inverse not symmetric\n", s.nx, s.ny, s.nz);
          return 1;
        }
  }
  // shapes that cannot be coarsened are refused, not built
  qs::HostHierarchy H;
  if (qs::build_hierarchy(33, 32, 32, 1.0 / 32, lam, mu, 8, &H) == 0) return 1;
  if (qs::build_hierarchy(80, 80, 40, 1.0 / 40, lam, mu, 4, &H) == 0) return 1;
  std::printf("ok\n");
  return 0;
}
