// Host construction of the multigrid hierarchy: fine stencil, Galerkin
// coarse stencils (Sec. 3.6, A_k = R_{k-1} A_{k-1} T_k with R = T^T) and the
// dense inverse of the coarsest operator.
#include "hierarchy.h"

#include "packed_stencil.h"

#include <algorithm>
#include <cmath>
#include <cstring>

namespace qs {

static inline int oidx(int oz, int oy, int ox) { return (oz + 1) * 9 + (oy + 1) * 3 + (ox + 1); }

int plan_levels(int nx, int ny, int nz, int min_coarse_nz, std::vector<int>* dims) {
  dims->clear();
  if (nx < 2 || ny < 2 || nz < 2 || min_coarse_nz < 2) return -2;
  for (;;) {
    dims->push_back(nx);
    dims->push_back(ny);
    dims->push_back(nz);
    if (nz <= min_coarse_nz) break;
    if ((nx | ny | nz) & 1) return -2;
    if (nx < 4 || ny < 4 || nz < 4) return -2;
    nx /= 2;
    ny /= 2;
    nz /= 2;
  }
  long long unknowns = 3LL * nx * ny * (nz - 1);
  if (unknowns > 6144) return -2;
  return 0;
}

void fine_stencil(int nz, double h, double lam, double mu, std::vector<double>* S) {
  S->assign(static_cast<size_t>(nz + 1) * kStencil, 0.0);
  const double ih2 = 1.0 / (h * h);
  const int unit[3][3] = {{0, 0, 1}, {0, 1, 0}, {1, 0, 0}};  // (oz,oy,ox) of x, y, z
  for (int k = 1; k < nz; ++k) {
    double* P = S->data() + static_cast<size_t>(k) * kStencil;
    for (int c = 0; c < 3; ++c) {
      double diag = 0.0;
      for (int a = 0; a < 3; ++a) {
        const double kap = (a == c) ? lam + 2.0 * mu : mu;
        const int* u = unit[a];
        P[oidx(u[0], u[1], u[2]) * 9 + c * 3 + c] -= kap * ih2;
        P[oidx(-u[0], -u[1], -u[2]) * 9 + c * 3 + c] -= kap * ih2;
        diag += 2.0 * kap * ih2;
      }
      P[oidx(0, 0, 0) * 9 + c * 3 + c] += diag;
      for (int d = 0; d < 3; ++d) {
        if (d == c) continue;
        for (int s = -1; s <= 1; s += 2)
          for (int t = -1; t <= 1; t += 2) {
            const int oz = s * unit[c][0] + t * unit[d][0];
            const int oy = s * unit[c][1] + t * unit[d][1];
            const int ox = s * unit[c][2] + t * unit[d][2];
            P[oidx(oz, oy, ox) * 9 + c * 3 + d] -= (lam + mu) * 0.25 * s * t * ih2;
          }
      }
    }
  }
}

// 1-D trilinear weight of a fine node at distance d (in fine cells) from the
// fine image 2I of a coarse node I.
static inline double w1(int d) { return d == 0 ? 1.0 : ((d == 1 || d == -1) ? 0.5 : 0.0); }

void galerkin_stencil(const std::vector<double>& Sf, int nzf, std::vector<double>* Sc) {
  const int nzc = nzf / 2;
  Sc->assign(static_cast<size_t>(nzc + 1) * kStencil, 0.0);
  for (int K = 1; K < nzc; ++K) {
    double* C = Sc->data() + static_cast<size_t>(K) * kStencil;
    // fine node f = 2I + df carries weight wf from coarse node I = (0,0,K)
    for (int dfz = -1; dfz <= 1; ++dfz)
      for (int dfy = -1; dfy <= 1; ++dfy)
        for (int dfx = -1; dfx <= 1; ++dfx) {
          const double wf = w1(dfz) * w1(dfy) * w1(dfx);
          const int kf = 2 * K + dfz;  // interior for 1 <= K <= nzc-1
          const double* F = Sf.data() + static_cast<size_t>(kf) * kStencil;
          for (int qz = -1; qz <= 1; ++qz) {
            const int kg = kf + qz;
            if (kg < 1 || kg > nzf - 1) continue;  // wall couplings are not in A_II
            for (int qy = -1; qy <= 1; ++qy)
              for (int qx = -1; qx <= 1; ++qx) {
                const double* B = F + oidx(qz, qy, qx) * 9;
                bool zero = true;
                for (int e = 0; e < 9; ++e) zero = zero && (B[e] == 0.0);
                if (zero) continue;
                const int gz = dfz + qz, gy = dfy + qy, gx = dfx + qx;  // g - 2I
                for (int Oz = -1; Oz <= 1; ++Oz) {
                  const int KJ = K + Oz;
                  if (KJ < 1 || KJ > nzc - 1) continue;  // coarse walls carry no unknown
                  const double wz = w1(gz - 2 * Oz);
                  if (wz == 0.0) continue;
                  for (int Oy = -1; Oy <= 1; ++Oy) {
                    const double wy = w1(gy - 2 * Oy);
                    if (wy == 0.0) continue;
                    for (int Ox = -1; Ox <= 1; ++Ox) {
                      const double wx = w1(gx - 2 * Ox);
                      if (wx == 0.0) continue;
                      const double w = wf * wz * wy * wx;
                      double* D = C + oidx(Oz, Oy, Ox) * 9;
                      for (int e = 0; e < 9; ++e) D[e] += w * B[e];
                    }
                  }
                }
              }
          }
        }
  }
}

static bool invert3(const double* A, double* X) {
  const double a = A[0], b = A[1], c = A[2], d = A[3], e = A[4], f = A[5], g = A[6], h = A[7],
               i = A[8];
  const double co0 = e * i - f * h, co1 = -(d * i - f * g), co2 = d * h - e * g;
  const double det = a * co0 + b * co1 + c * co2;
  if (!(std::fabs(det) > 0.0)) return false;
  const double id = 1.0 / det;
  X[0] = co0 * id;
  X[1] = -(b * i - c * h) * id;
  X[2] = (b * f - c * e) * id;
  X[3] = co1 * id;
  X[4] = (a * i - c * g) * id;
  X[5] = -(a * f - c * d) * id;
  X[6] = co2 * id;
  X[7] = -(a * h - b * g) * id;
  X[8] = (a * e - b * d) * id;
  return true;
}

// Inverse of a symmetric positive definite matrix via Cholesky: M = L L^T,
// W = L^{-1}, M^{-1} = W^T W.  Returns false if M is not positive definite.
static bool spd_inverse(std::vector<double>& M, int n, std::vector<double>* out) {
  std::vector<double> L(static_cast<size_t>(n) * n, 0.0);
  for (int j = 0; j < n; ++j) {
    const double* Lj = &L[static_cast<size_t>(j) * n];
    double s = M[static_cast<size_t>(j) * n + j];
    for (int k = 0; k < j; ++k) s -= Lj[k] * Lj[k];
    if (!(s > 0.0)) return false;
    const double ljj = std::sqrt(s);
    L[static_cast<size_t>(j) * n + j] = ljj;
    for (int i = j + 1; i < n; ++i) {
      const double* Li = &L[static_cast<size_t>(i) * n];
      double t = M[static_cast<size_t>(i) * n + j];
      for (int k = 0; k < j; ++k) t -= Li[k] * Lj[k];
      L[static_cast<size_t>(i) * n + j] = t / ljj;
    }
  }
  // W = L^{-1}, lower triangular, stored transposed (Wt[j][i] = W[i][j]) so
  // that both loops below run over contiguous memory.
  std::vector<double> Wt(static_cast<size_t>(n) * n, 0.0);
  for (int j = 0; j < n; ++j) {
    double* col = &Wt[static_cast<size_t>(j) * n];  // column j of W
    col[j] = 1.0 / L[static_cast<size_t>(j) * n + j];
    for (int i = j + 1; i < n; ++i) {
      const double* Li = &L[static_cast<size_t>(i) * n];
      double t = 0.0;
      for (int k = j; k < i; ++k) t += Li[k] * col[k];
      col[i] = -t / Li[i];
    }
  }
  out->assign(static_cast<size_t>(n) * n, 0.0);
  for (int i = 0; i < n; ++i) {
    const double* ci = &Wt[static_cast<size_t>(i) * n];
    for (int j = 0; j <= i; ++j) {
      const double* cj = &Wt[static_cast<size_t>(j) * n];
      double t = 0.0;
      for (int k = i; k < n; ++k) t += ci[k] * cj[k];
      (*out)[static_cast<size_t>(i) * n + j] = t;
      (*out)[static_cast<size_t>(j) * n + i] = t;
    }
  }
  return true;
}

int build_hierarchy(int nx, int ny, int nz, double h, double lam, double mu,
                    int min_coarse_nz, HostHierarchy* H) {
  std::vector<int> dims;
  if (plan_levels(nx, ny, nz, min_coarse_nz, &dims) != 0) return -2;
  const int nlev = static_cast<int>(dims.size() / 3);
  H->levels.assign(nlev, HostLevel());
  for (int l = 0; l < nlev; ++l) {
    HostLevel& L = H->levels[l];
    L.nx = dims[3 * l];
    L.ny = dims[3 * l + 1];
    L.nz = dims[3 * l + 2];
    if (l == 0)
      fine_stencil(L.nz, h, lam, mu, &L.stencil);
    else
      galerkin_stencil(H->levels[l - 1].stencil, H->levels[l - 1].nz, &L.stencil);
    L.dinv.assign(static_cast<size_t>(L.nz + 1) * 9, 0.0);
    for (int k = 1; k < L.nz; ++k)
      if (!invert3(L.stencil.data() + static_cast<size_t>(k) * kStencil + oidx(0, 0, 0) * 9,
                   L.dinv.data() + static_cast<size_t>(k) * 9))
        return -2;
  }
  // dense coarsest operator on its interior unknowns, wrapped offsets summed
  const HostLevel& G = H->levels.back();
  const int gx = G.nx, gy = G.ny, gz = G.nz;
  const int n = 3 * gx * gy * (gz - 1);
  H->n_coarse = n;
  std::vector<double> M(static_cast<size_t>(n) * n, 0.0);
  auto row_of = [&](int c, int k, int j, int i) {
    return ((c * (gz - 1) + (k - 1)) * gy + j) * gx + i;
  };
  for (int k = 1; k < gz; ++k) {
    const double* P = G.stencil.data() + static_cast<size_t>(k) * kStencil;
    for (int j = 0; j < gy; ++j)
      for (int i = 0; i < gx; ++i)
        for (int oz = -1; oz <= 1; ++oz) {
          const int kk = k + oz;
          if (kk < 1 || kk > gz - 1) continue;
          for (int oy = -1; oy <= 1; ++oy)
            for (int ox = -1; ox <= 1; ++ox) {
              const double* B = P + oidx(oz, oy, ox) * 9;
              const int jj = ((j + oy) % gy + gy) % gy, ii = ((i + ox) % gx + gx) % gx;
              for (int c = 0; c < 3; ++c)
                for (int d = 0; d < 3; ++d)
                  M[static_cast<size_t>(row_of(c, k, j, i)) * n + row_of(d, kk, jj, ii)] +=
                      B[c * 3 + d];
            }
        }
  }
  if (!spd_inverse(M, n, &H->coarse_inv)) return -2;
  return 0;
}

// Packs the plane stencils of one level (packed_stencil.h).  Returns false if
// an entry that the packing leaves out (a cross-component coupling at a zero
// offset along one of its components, zero in exact arithmetic) exceeds 1e-12
// of the largest entry of the level.
bool pack_level(const HostLevel& hl, std::vector<double>* out) {
  const int planes = hl.nz + 1;
  out->assign(static_cast<size_t>(planes) * kPackedStencil, 0.0);
  double big = 0.0, left_out = 0.0;
  for (int k = 0; k < planes; ++k) {
    const double* S = hl.stencil.data() + static_cast<size_t>(k) * kStencil;
    double* P = out->data() + static_cast<size_t>(k) * kPackedStencil;
    int n = 0;
    for (int oz = 0; oz < 3; ++oz)
      for (int oy = 0; oy < 3; ++oy)
        for (int ox = 0; ox < 3; ++ox)
          for (int c = 0; c < 3; ++c)
            for (int d = 0; d < 3; ++d) {
              const double v = S[(oz * 9 + oy * 3 + ox) * 9 + c * 3 + d];
              big = std::max(big, std::fabs(v));
              const bool centre = oz == 1 && oy == 1 && ox == 1;
              if (centre && c == d)
                P[kPackedCentre + c] = v;
              else if (!centre && packed_used(oz, oy, ox, c, d))
                P[n++] = v;
              else
                left_out = std::max(left_out, std::fabs(v));
            }
    for (int e = 0; e < 9; ++e) P[kPackedInv + e] = hl.dinv[static_cast<size_t>(k) * 9 + e];
  }
  return left_out <= 1e-12 * big;
}

}  // namespace qs
