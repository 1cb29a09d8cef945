// Host-side construction of the multigrid hierarchy (no HIP here).
//
// A level operator is a per-z-plane 27-point block stencil:
//   S[k][o][c][d], o = (oz+1)*9 + (oy+1)*3 + (ox+1),
// the 3x3 block coupling component c of node (i,j,k) to component d of node
// (i+ox, j+oy, k+oz).  Homogeneous stiffness and uniform spacing make every
// level invariant under x/y translation, so one stencil per plane is exact.
#pragma once
#include <cstddef>
#include <vector>

namespace qs {

constexpr int kStencil = 27 * 9;  // doubles per plane

struct HostLevel {
  int nx = 0, ny = 0, nz = 0;
  std::vector<double> stencil;  // (nz+1) * kStencil, rows k=0 and k=nz zero
  std::vector<double> dinv;     // (nz+1) * 9, inverse of the centre block
};

struct HostHierarchy {
  std::vector<HostLevel> levels;
  int n_coarse = 0;                // unknowns of the coarsest level
  std::vector<double> coarse_inv;  // n_coarse^2, row-major, symmetric
};

// Level count and dimensions without building anything.  Returns 0 on
// success, -2 (shape error) otherwise.
int plan_levels(int nx, int ny, int nz, int min_coarse_nz, std::vector<int>* dims);

// Fine operator stencil (Eq. col_snd_deriv and the mixed difference of
// Sec. 3.4 applied to -div(C : grad v)); the k=1 and k=nz-1 rows keep their
// couplings to the wall nodes.
void fine_stencil(int nz, double h, double lam, double mu, std::vector<double>* S);

// Galerkin coarse stencil A_c = T^T A_f T on the interior unknowns, by
// composing stencils on the infinite x/y lattice.
void galerkin_stencil(const std::vector<double>& Sf, int nzf, std::vector<double>* Sc);

// The plane stencils of one level in the packed form of packed_stencil.h
// ((nz + 1) * kPackedStencil entries).  Returns false if an entry the packing
// leaves out exceeds 1e-12 of the largest entry of the level.
bool pack_level(const HostLevel& hl, std::vector<double>* out);

// Full hierarchy; returns 0, or -2 for a shape error.
int build_hierarchy(int nx, int ny, int nz, double h, double lam, double mu,
                    int min_coarse_nz, HostHierarchy* H);

}  // namespace qs
