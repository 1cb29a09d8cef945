// Pointwise STZ update, projection right-hand side and stress correction
// (paper Secs. 3.1, 3.3, 3.4), and their reverse-mode derivatives.
//
// Cell tensors are [6][nz][ny][nx] in Voigt order (xx, yy, zz, yz, xz, xy);
// cell (i,j,k) has corners i..i+1, j..j+1 (wrapped), k..k+1.  Node vectors
// are [3][nz+1][ny][nx].  One thread per cell or per interior node; these
// kernels stream their inputs once and are HBM-bound.
#include "device.h"

namespace qs {

namespace {

constexpr int VA[6] = {0, 1, 2, 1, 0, 0};
constexpr int VB[6] = {0, 1, 2, 2, 2, 1};

struct CellIdx {
  int i, j, k, ip, jp;
};

__device__ __forceinline__ bool cell_of(int t, int nx, int ny, int nz, CellIdx* c) {
  if (t >= nx * ny * nz) return false;
  c->i = t % nx;
  c->j = (t / nx) % ny;
  c->k = t / (nx * ny);
  c->ip = c->i + 1 == nx ? 0 : c->i + 1;
  c->jp = c->j + 1 == ny ? 0 : c->j + 1;
  return true;
}

// Velocity gradient L[a][b] = d v_a / d x_b at a cell centre: the average of
// the four edge differences parallel to x_b (Eq. stag_stenc).
// Velocity gradient of a cell from its eight corner nodes, get(a, dz, dy, dx)
// returning component a at corner (dz, dy, dx).
template <typename G>
__device__ __forceinline__ void cell_gradient_from(G get, double ih4, double L[3][3]) {
#pragma unroll
  for (int a = 0; a < 3; ++a) {
    double f[2][2][2];
#pragma unroll
    for (int dz = 0; dz < 2; ++dz)
#pragma unroll
      for (int dy = 0; dy < 2; ++dy)
#pragma unroll
        for (int dx = 0; dx < 2; ++dx) f[dz][dy][dx] = get(a, dz, dy, dx);
    double gx = 0.0, gy = 0.0, gz = 0.0;
#pragma unroll
    for (int p = 0; p < 2; ++p)
#pragma unroll
      for (int q = 0; q < 2; ++q) {
        gx += f[p][q][1] - f[p][q][0];
        gy += f[p][1][q] - f[p][0][q];
        gz += f[1][p][q] - f[0][p][q];
      }
    L[a][0] = gx * ih4;
    L[a][1] = gy * ih4;
    L[a][2] = gz * ih4;
  }
}

__device__ __forceinline__ void cell_gradient(const double* __restrict__ v, int nx, int ny, int nz,
                                              const CellIdx& c, double ih4, double L[3][3]) {
  const int P = nx * ny, C = (nz + 1) * P;
  const int xs[2] = {c.i, c.ip}, ys[2] = {c.j, c.jp};
  cell_gradient_from(
      [&](int a, int dz, int dy, int dx) { return v[a * C + (c.k + dz) * P + ys[dy] * nx + xs[dx]]; },
      ih4, L);
}

__device__ __forceinline__ void load_voigt(const double* __restrict__ s, int N, int o, double S[3][3]) {
#pragma unroll
  for (int n = 0; n < 6; ++n) {
    const double val = s[n * N + o];
    S[VA[n]][VB[n]] = val;
    S[VB[n]][VA[n]] = val;
  }
}

// Scalar plastic rate of Eq. stz_dpl and its partial derivatives in sbar
// and chi; zero (with zero derivatives) at or below yield.
struct Plastic {
  double D, dD_ds, dD_dchi;
};

__device__ __forceinline__ Plastic plastic_rate(double sbar, double chi, const StzArgs& a) {
  Plastic p{0.0, 0.0, 0.0};
  if (sbar > a.s_y) {
    const double A = exp(-1.0 / chi) * exp(-a.delta_over_T) / a.tau0;
    const double bs = a.beta * sbar;
    const double ch = cosh(bs), sh = sinh(bs);
    const double f = 1.0 - a.s_y / sbar;
    p.D = A * ch * f;
    p.dD_ds = A * (a.beta * sh * f + ch * a.s_y / (sbar * sbar));
    p.dD_dchi = p.D / (chi * chi);
  }
  return p;
}

// Velocity at the cell centre: the mean of the cell's eight corner nodes.
// Mean of the eight corner velocities of a cell (get as for cell_gradient_from).
template <typename G>
__device__ __forceinline__ void cell_velocity_from(G get, double u[3]) {
#pragma unroll
  for (int a = 0; a < 3; ++a) {
    double acc = 0.0;
#pragma unroll
    for (int dz = 0; dz < 2; ++dz)
#pragma unroll
      for (int dy = 0; dy < 2; ++dy)
#pragma unroll
        for (int dx = 0; dx < 2; ++dx) acc += get(a, dz, dy, dx);
    u[a] = acc / 8.0;
  }
}

// Eq. ENO from the five values f(-2..2) along one axis and the velocity u
// along it: the upwind three-point formula where the point is more curved
// than its upwind neighbour, the centred difference otherwise (times 2h).
__device__ __forceinline__ double eno_2h(double fm2, double fm1, double f0, double fp1, double fp2,
                                         double u) {
#pragma clang fp contract(off)
  const double cm = fabs(f0 - 2.0 * fm1 + fm2);
  const double c0 = fabs(fp1 - 2.0 * f0 + fm1);
  const double cp = fabs(fp2 - 2.0 * fp1 + f0);
  if (u < 0.0 && c0 > cp) return -fp2 + 4.0 * fp1 - 3.0 * f0;
  if (u > 0.0 && c0 > cm) return 3.0 * f0 - 4.0 * fm1 + fm2;
  return fp1 - fm1;
}

// D^pl alone (Eq. stz_dpl), for the sub-step loop.
__device__ __forceinline__ double plastic_D(double sbar, double chi, const StzArgs& a) {
  if (!(sbar > a.s_y)) return 0.0;
  const double A = exp(-1.0 / chi) * exp(-a.delta_over_T) / a.tau0;
  return A * cosh(a.beta * sbar) * (1.0 - a.s_y / sbar);
}

constexpr int kMaxSubsteps = 65536;
constexpr int kImplicitBisections = 64;

__device__ __forceinline__ void deviator(const double S[3][3], double S0[3][3], double* sbar) {
  const double pr = (S[0][0] + S[1][1] + S[2][2]) * (1.0 / 3.0);
  double q = 0.0;
#pragma unroll
  for (int a = 0; a < 3; ++a)
#pragma unroll
    for (int b = 0; b < 3; ++b) {
      S0[a][b] = S[a][b] - (a == b ? pr : 0.0);
      q += S0[a][b] * S0[a][b];
    }
  *sbar = sqrt(0.5 * q);
}

// D^pl of a cell of step n, and of the ghost cell beyond a z wall: sigma and
// chi linearly extrapolated from the wall cell o0 and its inner neighbour o1.
// D^pl is 0 where chi is not positive (possible only for an extrapolation).
__device__ __forceinline__ double dpl_of(const double S[3][3], double x, const StzArgs& a) {
  double S0[3][3], sb;
  deviator(S, S0, &sb);
  return x > 0.0 ? plastic_rate(sb, x, a).D : 0.0;
}

__device__ __forceinline__ double dpl_cell(const double* __restrict__ sigma,
                                           const double* __restrict__ chi, int N, int o,
                                           const StzArgs& a) {
  double S[3][3];
  load_voigt(sigma, N, o, S);
  return dpl_of(S, chi[o], a);
}

__device__ __forceinline__ double dpl_ghost(const double* __restrict__ sigma,
                                            const double* __restrict__ chi, int N, int o0, int o1,
                                            const StzArgs& a, double* xg) {
  double S[3][3];
#pragma unroll
  for (int n = 0; n < 6; ++n) {
    const double val = 2.0 * sigma[n * N + o0] - sigma[n * N + o1];
    S[VA[n]][VB[n]] = val;
    S[VB[n]][VA[n]] = val;
  }
  *xg = 2.0 * chi[o0] - chi[o1];
  return dpl_of(S, *xg, a);
}

// div(D^pl grad chi) at cell c (Eq. chi_evo): flux form over the six faces,
// face coefficient (D_c + D_n)/2, in the order y+1, y-1, x+1, x-1, z-1, z+1.
__device__ __forceinline__ double chi_flux_divergence(const double* __restrict__ sigma,
                                                      const double* __restrict__ chi,
                                                      const double* __restrict__ Dcell, int nx,
                                                      int ny, int nz, const CellIdx& c, int o,
                                                      double Dc, double xc, const StzArgs& a) {
  const int N = nx * ny * nz, P = nx * ny;
  const int im = c.i == 0 ? nx - 1 : c.i - 1, jm = c.j == 0 ? ny - 1 : c.j - 1;
  const int base = c.k * P;
  const int nb[4] = {base + c.jp * nx + c.i, base + jm * nx + c.i, base + c.j * nx + c.ip,
                     base + c.j * nx + im};
  double s = 0.0;
#pragma unroll
  for (int q = 0; q < 4; ++q) {
    const double Dn = Dcell[nb[q]];
    s += 0.5 * (Dc + Dn) * (chi[nb[q]] - xc);
  }
  double xn, Dn;
  if (c.k > 0) {
    Dn = Dcell[o - P];
    xn = chi[o - P];
  } else if (a.chi_wall) {  // no flux through the wall face
    Dn = Dc;
    xn = xc;
  } else {
    Dn = dpl_ghost(sigma, chi, N, o, o + P, a, &xn);
  }
  s += 0.5 * (Dc + Dn) * (xn - xc);
  if (c.k < nz - 1) {
    Dn = Dcell[o + P];
    xn = chi[o + P];
  } else if (a.chi_wall) {
    Dn = Dc;
    xn = xc;
  } else {
    Dn = dpl_ghost(sigma, chi, N, o, o - P, a, &xn);
  }
  s += 0.5 * (Dc + Dn) * (xn - xc);
  return s / (a.h * a.h);
}

// DIFF: with the diffusion term of Eq. chi_evo (l > 0); each cell evaluates
// D^pl of its six neighbours itself, from sigma and chi of step n.
// D^pl of every cell (0 where chi is not positive), for the diffusion term.
__global__ __launch_bounds__(256) void k_dpl_cells(const double* __restrict__ sigma,
                                                   const double* __restrict__ chi,
                                                   double* __restrict__ D, int N, StzArgs a) {
  const int t = blockIdx.x * blockDim.x + threadIdx.x;
  if (t >= N) return;
  D[t] = dpl_cell(sigma, chi, N, t, a);
}

// The cell update of the STZ step from the velocity gradient L, the stress S
// and chi of cell t (and, with ADV, adv(n) = the advection term
// (u . grad) sigma of Voigt component n, evaluated when that component is
// written): writes sigma*[.][t] and chi'[t].
template <bool DIFF, bool ADV, typename Adv>
__device__ __forceinline__ void stz_update(const double* __restrict__ sigma,
                                           const double* __restrict__ chi,
                                           double* __restrict__ sstar, double* __restrict__ chi1,
                                           const double* __restrict__ Dcell, int nx, int ny, int nz,
                                           const CellIdx& c, int t, const double L[3][3],
                                           const double S[3][3], double x, const Adv& adv,
                                           const StzArgs& a) {
  const int N = nx * ny * nz;
  double S0[3][3], sbar;
  deviator(S, S0, &sbar);
  const Plastic pl = plastic_rate(sbar, x, a);
  const double trL = L[0][0] + L[1][1] + L[2][2];
  double xn;
  if (a.n_sub == 1) {
    const double rho = pl.D > 0.0 ? pl.D / sbar : 0.0;
    // C : (rho S0) = lambda tr(rho S0) I + 2 mu rho S0, and tr(S0) = 0
#pragma unroll
    for (int n = 0; n < 6; ++n) {
      const int p = VA[n], q = VB[n];
      double LS = 0.0, SLt = 0.0;
#pragma unroll
      for (int m = 0; m < 3; ++m) {
        LS += L[p][m] * S[m][q];
        SLt += S[p][m] * L[q][m];
      }
      const double rate = LS + SLt - trL * S[p][q] - 2.0 * a.mu * rho * S0[p][q];
      double val = S[p][q] + a.dt * rate;
      if (ADV) val = val - a.dt * adv(n);
      sstar[n * N + t] = val;
    }
    xn = x + (a.dt / a.c0) * (2.0 * sbar * pl.D / a.s_y) * (a.chi_inf - x);
  } else if (a.n_sub == -2) {
    // backward Euler of the local relaxation, chi held at step n: the root of
    // s - sbar + 2 mu dt D^pl(s) in [s_Y, sbar] by bisection; the deviator
    // shrinks to it, chi' = (chi + c chi_inf) / (1 + c)
    double s1 = sbar;
    if (sbar > a.s_y) {
      double lo = a.s_y, hi = sbar;
      for (int it = 0; it < kImplicitBisections; ++it) {
        const double mid = 0.5 * (lo + hi);
        const double g = mid - sbar + 2.0 * a.mu * a.dt * plastic_D(mid, x, a);
        if (g < 0.0)
          lo = mid;
        else
          hi = mid;
      }
      s1 = hi;
    }
    const double scale = sbar > a.s_y ? s1 / (sbar > 0.0 ? sbar : 1.0) : 1.0;
    const double D1 = plastic_D(s1, x, a);
    const double cg = (a.dt / a.c0) * (2.0 * s1 * D1 / a.s_y);
    xn = (x + cg * a.chi_inf) / (1.0 + cg);
#pragma unroll
    for (int n = 0; n < 6; ++n) {
      const int p = VA[n], q = VB[n];
      double LS = 0.0, SLt = 0.0;
#pragma unroll
      for (int m = 0; m < 3; ++m) {
        LS += L[p][m] * S[m][q];
        SLt += S[p][m] * L[q][m];
      }
      double val = (S[p][q] - (1.0 - scale) * S0[p][q]) + a.dt * (LS + SLt - trL * S[p][q]);
      if (ADV) val = val - a.dt * adv(n);
      sstar[n * N + t] = val;
    }
  } else {
    // sub-steps of the plastic terms from the state of step n
    int M = a.n_sub;
    if (M < 0) {
      const double m = ceil(4.0 * a.mu * a.dt * pl.dD_ds);
      M = !(m < static_cast<double>(kMaxSubsteps)) ? kMaxSubsteps : (m < 1.0 ? 1 : static_cast<int>(m));
    }
    const double tau = a.dt / M;
    double Sp[3][3], xp = x;
#pragma unroll
    for (int p = 0; p < 3; ++p)
#pragma unroll
      for (int q = 0; q < 3; ++q) Sp[p][q] = S[p][q];
    for (int it = 0; it < M; ++it) {
      double P0[3][3], sb;
      deviator(Sp, P0, &sb);
      const double D = plastic_D(sb, xp, a);
      const double r = D > 0.0 ? D / sb : 0.0;
#pragma unroll
      for (int p = 0; p < 3; ++p)
#pragma unroll
        for (int q = 0; q < 3; ++q) Sp[p][q] = Sp[p][q] - tau * (2.0 * a.mu * r * P0[p][q]);
      xp = xp + (tau / a.c0) * (2.0 * sb * D / a.s_y) * (a.chi_inf - xp);
    }
#pragma unroll
    for (int n = 0; n < 6; ++n) {
      const int p = VA[n], q = VB[n];
      double LS = 0.0, SLt = 0.0;
#pragma unroll
      for (int m = 0; m < 3; ++m) {
        LS += L[p][m] * S[m][q];
        SLt += S[p][m] * L[q][m];
      }
      double val = Sp[p][q] + a.dt * (LS + SLt - trL * S[p][q]);
      if (ADV) val = val - a.dt * adv(n);
      sstar[n * N + t] = val;
    }
    xn = xp;
  }
  if (DIFF) {
    // the cell's own D^pl as in the flux form (0 where chi is not positive)
    const double Dc = x > 0.0 ? pl.D : 0.0;
    xn = xn + (a.dt / a.c0) * a.l2 * chi_flux_divergence(sigma, chi, Dcell, nx, ny, nz, c, t, Dc, x, a);
  }
  chi1[t] = xn;
}

// One thread per cell (no advection).
template <bool DIFF>
__global__ __launch_bounds__(256) void k_stz_step(const double* __restrict__ v,
                                                  const double* __restrict__ sigma,
                                                  const double* __restrict__ chi,
                                                  double* __restrict__ sstar,
                                                  double* __restrict__ chi1,
                                                  const double* __restrict__ Dcell, int nx, int ny,
                                                  int nz, StzArgs a) {
  CellIdx c;
  const int t = blockIdx.x * blockDim.x + threadIdx.x;
  if (!cell_of(t, nx, ny, nz, &c)) return;
  double L[3][3], S[3][3];
  cell_gradient(v, nx, ny, nz, c, 0.25 / a.h, L);
  load_voigt(sigma, nx * ny * nz, t, S);
  stz_update<DIFF, false>(sigma, chi, sstar, chi1, Dcell, nx, ny, nz, c, t, L, S, chi[t],
                          [](int) { return 0.0; }, a);
}

// sigma of one Voigt component f at plane e of column col; in z, the layers
// past the walls continue the two nearest layers linearly (Sec. 3.5).
__device__ __forceinline__ double z_layer(const double* __restrict__ f, int P, int nz, int col,
                                          int e) {
#pragma clang fp contract(off)
  if (e >= 0 && e <= nz - 1) return f[col + e * P];
  if (e < 0) {
    const double b0 = f[col], b1 = f[col + P];
    const double d0 = b1 - b0;
    return e == -1 ? b0 - d0 : b0 - 2.0 * d0;
  }
  const double t1 = f[col + (nz - 1) * P], t0 = f[col + (nz - 2) * P];
  const double d1 = t1 - t0;
  return e == nz ? t1 + d1 : t1 + 2.0 * d1;
}

// With the advection of the stress (Eq. sig_star_evol): one thread per cell,
// a workgroup per 16 x 16 tile of one cell plane.  Eq. ENO reads two cells on
// each side along x, y and z; x and y come from the tile staged in LDS, and
// the mapping keeps the z reads in cache: a band of 16 rows (all tiles along
// x) goes to one XCD (workgroup w runs on XCD w mod 8), whose workgroups take
// the band plane after plane and tile after tile.  The planes k-2 .. k+2 of a
// band are then in flight together and share that XCD's L2.  Each derivative
// is Eq. ENO along its axis (x and y wrap; in z the layers past the walls
// continue the two nearest layers linearly, Sec. 3.5), with u the mean of the
// cell's eight corner velocities; no fused multiply-adds here, so the branch
// choices of Eq. ENO are taken on the same FP64 values as the oracle's.
constexpr int kTile = 16;

template <bool DIFF>
__global__ __launch_bounds__(kTile * kTile) void k_stz_step_adv(const double* __restrict__ v,
                                                               const double* __restrict__ sigma,
                                                               const double* __restrict__ chi,
                                                               double* __restrict__ sstar,
                                                               double* __restrict__ chi1,
                                                               const double* __restrict__ Dcell,
                                                               int nx, int ny, int nz, int ntx,
                                                               int bands, StzArgs a) {
#pragma clang fp contract(off)
  const int w = blockIdx.x;
  const int xcd = w & 7, slot = w >> 3;
  const int per_band = nz * ntx;
  const int band = (slot / per_band) * 8 + xcd;
  if (band >= bands) return;
  const int r = slot - (slot / per_band) * per_band;
  const int k = r / ntx, tx = r - k * ntx;
  const int lx = static_cast<int>(threadIdx.x) % kTile, ly = static_cast<int>(threadIdx.x) / kTile;
  const int i0 = tx * kTile, j0 = band * kTile;
  // cells past the grid edge (ragged last tile) compute on a clamped cell and
  // write nothing; they take part in the staging and the barriers
  const bool active = i0 + lx < nx && j0 + ly < ny;
  CellIdx c;
  c.i = min(i0 + lx, nx - 1);
  c.j = min(j0 + ly, ny - 1);
  c.k = k;
  c.ip = c.i + 1 == nx ? 0 : c.i + 1;
  c.jp = c.j + 1 == ny ? 0 : c.j + 1;
  const int P = nx * ny, N = P * nz;
  const int col = c.j * nx + c.i;
  const int t = k * P + col;
  // The six advection terms, one component at a time (a loop that is not
  // unrolled keeps one copy of the stencil code and few registers), parked in
  // LDS slots of this thread until the update writes each component.  The
  // component's plane k over the tile and two cells around it (x and y wrap)
  // is staged in LDS, so each value is loaded once instead of by the five
  // cells that use it; the four z neighbours of the cell's own column come
  // from memory.  The next component's values are loaded while one is
  // computed.  Before that, the tile's corner nodes (17 x 17 columns, node
  // planes k and k+1) pass through the same LDS as advs and fcell, so each
  // node is loaded once instead of by the eight cells around it.
  constexpr int kW = kTile + 4;  // staged rows and columns
  constexpr int kT = kTile * kTile;
  __shared__ double pool[2 * 6 * kT];
  double(*advs)[kT] = reinterpret_cast<double(*)[kT]>(pool);
  double(*fcell)[kT] = reinterpret_cast<double(*)[kT]>(pool + 6 * kT);  // the cell's own sigma
  double(*vt)[2][kTile + 1][kTile + 2] = reinterpret_cast<double(*)[2][kTile + 1][kTile + 2]>(pool);
  static_assert(3 * 2 * (kTile + 1) * (kTile + 2) <= 2 * 6 * kT, "corner nodes fit the pool");
  __shared__ double tl[kW][kW + 1];
  const double ih2 = 1.0 / (2.0 * a.h);
  int soff[2];  // plane offsets of this thread's two staged cells (the second may be unused)
#pragma unroll
  for (int q = 0; q < 2; ++q) {
    const int e = min(static_cast<int>(threadIdx.x) + q * kT, kW * kW - 1);
    const int sy = e / kW, sx = e - sy * kW;
    const int gj = ((j0 - 2 + sy) % ny + ny) % ny, gi = ((i0 - 2 + sx) % nx + nx) % nx;
    soff[q] = gj * nx + gi;
  }
  const bool second = static_cast<int>(threadIdx.x) + kT < kW * kW;
  auto fetch = [&](int n, double sv[2], double zv[4]) {
    const double* g = sigma + n * N;
    sv[0] = g[k * P + soff[0]];
    sv[1] = g[k * P + soff[1]];
    const int ks[4] = {k - 2, k - 1, k + 1, k + 2};
#pragma unroll
    for (int q = 0; q < 4; ++q) zv[q] = z_layer(g, P, nz, col, ks[q]);
  };
  double sv[2], zv[4];
  fetch(0, sv, zv);
  {
    constexpr int kNodes = 3 * 2 * (kTile + 1) * (kTile + 1);
    constexpr int kPer = (kNodes + kT - 1) / kT;
    double nv[kPer];
    int comp[kPer], dz[kPer], yy[kPer], xx[kPer];
#pragma unroll
    for (int q = 0; q < kPer; ++q) {
      const int e = min(static_cast<int>(threadIdx.x) + q * kT, kNodes - 1);
      comp[q] = e / (2 * (kTile + 1) * (kTile + 1));
      const int rem = e - comp[q] * 2 * (kTile + 1) * (kTile + 1);
      dz[q] = rem / ((kTile + 1) * (kTile + 1));
      const int rem2 = rem - dz[q] * (kTile + 1) * (kTile + 1);
      yy[q] = rem2 / (kTile + 1);
      xx[q] = rem2 - yy[q] * (kTile + 1);
      const int gi = (i0 + xx[q]) % nx, gj = (j0 + yy[q]) % ny;
      nv[q] = v[comp[q] * (nz + 1) * P + (k + dz[q]) * P + gj * nx + gi];
    }
#pragma unroll
    for (int q = 0; q < kPer; ++q)
      if (static_cast<int>(threadIdx.x) + q * kT < kNodes) vt[comp[q]][dz[q]][yy[q]][xx[q]] = nv[q];
  }
  __syncthreads();
  const int ci = c.i - i0, cj = c.j - j0;  // the cell within the tile (clamped cells included)
  auto corner = [&](int cmp, int ez, int ey, int ex) { return vt[cmp][ez][cj + ey][ci + ex]; };
  double L[3][3], S[3][3], u[3];
  cell_gradient_from(corner, 0.25 / a.h, L);
  cell_velocity_from(corner, u);
#pragma unroll 1
  for (int n = 0; n < 6; ++n) {
    __syncthreads();  // the previous component's reads of tl (at n = 0: of the corner nodes) are done
    tl[threadIdx.x / kW][threadIdx.x % kW] = sv[0];
    if (second) tl[(threadIdx.x + kT) / kW][(threadIdx.x + kT) % kW] = sv[1];
    double z[4];
#pragma unroll
    for (int q = 0; q < 4; ++q) z[q] = zv[q];
    __syncthreads();
    if (n < 5) fetch(n + 1, sv, zv);  // in flight while component n is computed
    const double* row = &tl[ly + 2][lx + 2];
    const double f0 = row[0];
    const double dx = eno_2h(row[-2], row[-1], f0, row[1], row[2], u[0]);
    const double dy = eno_2h(tl[ly][lx + 2], tl[ly + 1][lx + 2], f0, tl[ly + 3][lx + 2],
                             tl[ly + 4][lx + 2], u[1]);
    const double dz = eno_2h(z[0], z[1], f0, z[2], z[3], u[2]);
    advs[n][threadIdx.x] = (u[0] * dx + u[1] * dy + u[2] * dz) * ih2;
    fcell[n][threadIdx.x] = f0;
  }
  if (!active) return;
#pragma unroll
  for (int n = 0; n < 6; ++n) {
    const double val = fcell[n][threadIdx.x];
    S[VA[n]][VB[n]] = val;
    S[VB[n]][VA[n]] = val;
  }
  stz_update<DIFF, true>(sigma, chi, sstar, chi1, Dcell, nx, ny, nz, c, t, L, S, chi[t],
                         [&](int n) { return advs[n][threadIdx.x]; }, a);
}

// Node divergence of a cell field (corner form of Eq. stag_stenc): for
// interior node (i,j,k) the cells (i-1..i, j-1..j, k-1..k).  `get(n, cell)`
// returns component n of the tensor stored per cell.
struct NodeCells {
  int cell[2][2][2];  // [ez][ey][ex] -> flat cell index
};

__device__ __forceinline__ bool node_of(int t, int nx, int ny, int nz, int* i, int* j, int* k,
                                        NodeCells* nc) {
  if (t >= nx * ny * (nz - 1)) return false;
  *i = t % nx;
  *j = (t / nx) % ny;
  *k = 1 + t / (nx * ny);
  const int xs[2] = {*i == 0 ? nx - 1 : *i - 1, *i};
  const int ys[2] = {*j == 0 ? ny - 1 : *j - 1, *j};
#pragma unroll
  for (int ez = 0; ez < 2; ++ez)
#pragma unroll
    for (int ey = 0; ey < 2; ++ey)
#pragma unroll
      for (int ex = 0; ex < 2; ++ex) nc->cell[ez][ey][ex] = ((*k - 1 + ez) * ny + ys[ey]) * nx + xs[ex];
  return true;
}

// d/dx_b at a node of a cell scalar g given its 8 values g[ez][ey][ex].
__device__ __forceinline__ double node_diff(const double g[2][2][2], int b) {
  double s = 0.0;
#pragma unroll
  for (int p = 0; p < 2; ++p)
#pragma unroll
    for (int q = 0; q < 2; ++q) {
      if (b == 0) s += g[p][q][1] - g[p][q][0];
      if (b == 1) s += g[p][1][q] - g[p][0][q];
      if (b == 2) s += g[1][p][q] - g[0][p][q];
    }
  return s;
}

// Explicit method (Sec. 3.2): the new velocity at an interior node,
//   v' = v + dt ((D_h sigma)/rho - (v . grad) v + kappa lap v),
// all from step n: D_h sigma as in k_rhs, the Laplacian by Eq. col_snd_deriv,
// the advection by Eq. ENO with the node's own velocity (ghost node past a
// wall: 2 v_wall - v of the node inside it).  Writes interior nodes of vout.
__global__ __launch_bounds__(256) void k_explicit_velocity(const double* __restrict__ v,
                                                           const double* __restrict__ sigma,
                                                           double* __restrict__ vout, int nx, int ny,
                                                           int nz, double h, double dt, double rho,
                                                           double kappa) {
  int i, j, k;
  NodeCells nc;
  const int t = blockIdx.x * blockDim.x + threadIdx.x;
  if (!node_of(t, nx, ny, nz, &i, &j, &k, &nc)) return;
  const int N = nx * ny * nz, P = nx * ny, C = (nz + 1) * P;
  double div[3] = {0.0, 0.0, 0.0};
#pragma unroll
  for (int n = 0; n < 6; ++n) {
    double g[2][2][2];
#pragma unroll
    for (int ez = 0; ez < 2; ++ez)
#pragma unroll
      for (int ey = 0; ey < 2; ++ey)
#pragma unroll
        for (int ex = 0; ex < 2; ++ex) g[ez][ey][ex] = sigma[n * N + nc.cell[ez][ey][ex]];
    const int p = VA[n], q = VB[n];
    div[p] += node_diff(g, q);
    if (p != q) div[q] += node_diff(g, p);
  }
  const int o = k * P + j * nx + i;
  const int row = o - i;
  const double u[3] = {v[o], v[C + o], v[2 * C + o]};
  const double h2 = 2.0 * h;
#pragma unroll
  for (int a = 0; a < 3; ++a) {
    const double* f = v + a * C;
    double g[5];
#pragma unroll
    for (int s = -2; s <= 2; ++s) g[s + 2] = f[row + (i + s + 2 * nx) % nx];
    const double dx = eno_2h(g[0], g[1], g[2], g[3], g[4], u[0]);
    const double lx = g[1] + g[3] - 2.0 * g[2];
#pragma unroll
    for (int s = -2; s <= 2; ++s) g[s + 2] = f[k * P + ((j + s + 2 * ny) % ny) * nx + i];
    const double dy = eno_2h(g[0], g[1], g[2], g[3], g[4], u[1]);
    const double ly = g[1] + g[3] - 2.0 * g[2];
    const int col = j * nx + i;
#pragma unroll
    for (int s = -2; s <= 2; ++s) {
      const int e = k + s;
      g[s + 2] = e < 0 ? 2.0 * f[col] - f[P + col]
                       : (e > nz ? 2.0 * f[nz * P + col] - f[(nz - 1) * P + col] : f[e * P + col]);
    }
    const double dz = eno_2h(g[0], g[1], g[2], g[3], g[4], u[2]);
    const double lz = g[3] + g[1] - 2.0 * g[2];
    const double adv = u[0] * (dx / h2) + u[1] * (dy / h2) + u[2] * (dz / h2);
    const double lap = (lx + ly + lz) / (h * h);
    const double acc = (div[a] * (0.25 / h)) / rho - adv + kappa * lap;
    vout[a * C + o] = g[2] + dt * acc;
  }
}

// b = scale * D_h sigma* at the interior nodes (staggered divergence, the
// node form of Eq. stag_stenc).  Each thread marches up a z-segment of one
// (i, j) column: the cell plane below a node is the one above the previous
// node, kept in registers, so every cell plane is read once per segment.
__global__ __launch_bounds__(256) void k_rhs(const double* __restrict__ sstar,
                                               double* __restrict__ b, int nx, int ny, int nz,
                                               int seg, int blocks, int blocks_per_xcd,
                                               double scale) {
  // workgroup w runs on XCD w mod 8; each XCD takes a contiguous range of
  // column blocks (rows, for 256-wide rows) of one segment after the other, so
  // the cells of row j-1 that a node of row j reads were just read by the
  // workgroup of row j-1 on the same XCD and come from its L2
  const int w = blockIdx.x;
  const int slot = w >> 3;
  const int blk = (w & 7) * blocks_per_xcd + slot % blocks_per_xcd;
  if (blk >= blocks) return;
  const int P = nx * ny;
  const int t = blk * blockDim.x + threadIdx.x;
  if (t >= P) return;
  const int k0 = 1 + (slot / blocks_per_xcd) * seg;
  if (k0 > nz - 1) return;
  const int k1 = min(k0 + seg, nz);  // nodes k0 .. k1-1
  const int i = t % nx, j = t / nx;
  const int N = P * nz, C = (nz + 1) * P;
  const int xs[2] = {i == 0 ? nx - 1 : i - 1, i};
  const int ys[2] = {j == 0 ? ny - 1 : j - 1, j};
  double lo[6][2][2];
#pragma unroll
  for (int n = 0; n < 6; ++n)
#pragma unroll
    for (int ey = 0; ey < 2; ++ey)
#pragma unroll
      for (int ex = 0; ex < 2; ++ex)
        lo[n][ey][ex] = sstar[n * N + ((k0 - 1) * ny + ys[ey]) * nx + xs[ex]];
  for (int k = k0; k < k1; ++k) {
    double acc[3] = {0.0, 0.0, 0.0};
#pragma unroll
    for (int n = 0; n < 6; ++n) {
      double g[2][2][2];
#pragma unroll
      for (int ey = 0; ey < 2; ++ey)
#pragma unroll
        for (int ex = 0; ex < 2; ++ex) {
          g[0][ey][ex] = lo[n][ey][ex];
          g[1][ey][ex] = sstar[n * N + (k * ny + ys[ey]) * nx + xs[ex]];
          lo[n][ey][ex] = g[1][ey][ex];
        }
      const int p = VA[n], q = VB[n];
      acc[p] += node_diff(g, q);
      if (p != q) acc[q] += node_diff(g, p);
    }
    const int o = k * P + j * nx + i;
#pragma unroll
    for (int a = 0; a < 3; ++a) b[a * C + o] = acc[a] * scale;
  }
}

__global__ void k_zero_walls(double* __restrict__ b, int nx, int ny, int nz) {
  const int t = blockIdx.x * blockDim.x + threadIdx.x;
  const int P = nx * ny;
  if (t >= 6 * P) return;
  const int c = t / (2 * P), rem = t % (2 * P);
  const int plane = rem < P ? 0 : nz;
  b[(static_cast<size_t>(c) * (nz + 1) + plane) * P + rem % P] = 0.0;
}

__global__ __launch_bounds__(256) void k_stress_update(const double* __restrict__ sstar,
                                                       const double* __restrict__ v,
                                                       double* __restrict__ out, int nx, int ny,
                                                       int nz, double h, double dt, double lam,
                                                       double mu) {
  CellIdx c;
  const int t = blockIdx.x * blockDim.x + threadIdx.x;
  if (!cell_of(t, nx, ny, nz, &c)) return;
  const int N = nx * ny * nz;
  double L[3][3];
  cell_gradient(v, nx, ny, nz, c, 0.25 / h, L);
  const double tr = L[0][0] + L[1][1] + L[2][2];
#pragma unroll
  for (int n = 0; n < 6; ++n) {
    const int p = VA[n], q = VB[n];
    const double D = 0.5 * (L[p][q] + L[q][p]);
    out[n * N + t] = sstar[n * N + t] + dt * ((p == q ? lam * tr : 0.0) + 2.0 * mu * D);
  }
}

__global__ void k_set_walls(double* __restrict__ v, int nx, int ny, int nz, double U) {
  const int t = blockIdx.x * blockDim.x + threadIdx.x;
  const int P = nx * ny;
  if (t >= 2 * P) return;
  const int plane = t < P ? 0 : nz;
  const size_t o = static_cast<size_t>(plane) * P + (t % P);
  const size_t C = static_cast<size_t>(nz + 1) * P;
  v[o] = plane == 0 ? -U : U;
  v[C + o] = 0.0;
  v[2 * C + o] = 0.0;
}

// Wall planes k = 0 and k = nz of v from per-node data lo, hi [3][ny][nx].
__global__ void k_copy_walls(double* __restrict__ v, const double* __restrict__ lo,
                             const double* __restrict__ hi, int nx, int ny, int nz) {
  const int t = blockIdx.x * blockDim.x + threadIdx.x;
  const int P = nx * ny;
  if (t >= 3 * P) return;
  const int a = t / P, q = t - a * P;
  const size_t C = static_cast<size_t>(nz + 1) * P;
  v[a * C + q] = lo[t];
  v[a * C + static_cast<size_t>(nz) * P + q] = hi[t];
}

// ---------------------------------------------------------------------------
// Reverse mode.  All cotangents are derivatives with respect to the stored
// numbers (Euclidean inner product on the arrays).
// ---------------------------------------------------------------------------

// Per cell: cotangents of sigma (Voigt), chi and the velocity gradient L
// (9 values, [a][b] row-major, stored as [9][cells]) from those of sigma*
// and chi'.
__global__ __launch_bounds__(256) void k_stz_step_vjp(
    const double* __restrict__ v, const double* __restrict__ sigma, const double* __restrict__ chi,
    const double* __restrict__ g_sstar, const double* __restrict__ g_chi1,
    double* __restrict__ g_sigma, double* __restrict__ g_chi, double* __restrict__ g_L, int nx,
    int ny, int nz, StzArgs a) {
  CellIdx c;
  const int t = blockIdx.x * blockDim.x + threadIdx.x;
  if (!cell_of(t, nx, ny, nz, &c)) return;
  const int N = nx * ny * nz;
  double L[3][3], S[3][3], S0[3][3], sbar, W[3][3];
  cell_gradient(v, nx, ny, nz, c, 0.25 / a.h, L);
  load_voigt(sigma, N, t, S);
  deviator(S, S0, &sbar);
  // f = sum_n g_n sigma*_n = W : S* with W symmetric, W_ab = g_n (a==b) or g_n/2
#pragma unroll
  for (int n = 0; n < 6; ++n) {
    const double g = g_sstar[n * N + t];
    const int p = VA[n], q = VB[n];
    if (p == q) {
      W[p][p] = g;
    } else {
      W[p][q] = 0.5 * g;
      W[q][p] = 0.5 * g;
    }
  }
  const double x = chi[t];
  const double gc = g_chi1[t];
  const Plastic pl = plastic_rate(sbar, x, a);
  const bool act = pl.D > 0.0;
  const double rho = act ? pl.D / sbar : 0.0;
  const double trL = L[0][0] + L[1][1] + L[2][2];
  double WS[3][3], WdotS = 0.0;
#pragma unroll
  for (int p = 0; p < 3; ++p)
#pragma unroll
    for (int q = 0; q < 3; ++q) {
      double s = 0.0;
#pragma unroll
      for (int m = 0; m < 3; ++m) s += W[p][m] * S[m][q];
      WS[p][q] = s;
      WdotS += W[p][q] * S[p][q];
    }
  // dL: dt (2 (W S) - tr(W:S) I)
#pragma unroll
  for (int p = 0; p < 3; ++p)
#pragma unroll
    for (int q = 0; q < 3; ++q)
      g_L[(p * 3 + q) * N + t] = a.dt * (2.0 * WS[p][q] - (p == q ? WdotS : 0.0));
  // H = df/dS over all nine entries
  const double trW = W[0][0] + W[1][1] + W[2][2];
  double W0[3][3], W0dotS = 0.0;
#pragma unroll
  for (int p = 0; p < 3; ++p)
#pragma unroll
    for (int q = 0; q < 3; ++q) {
      W0[p][q] = W[p][q] - (p == q ? trW / 3.0 : 0.0);
      W0dotS += W0[p][q] * S[p][q];
    }
  double H[3][3];
  // coefficient multiplying S0 / (2 sbar) from the sbar-dependence
  double dsb = 0.0;
  double gchi = 0.0;
  const double kq = 2.0 * a.dt / (a.c0 * a.s_y);
  if (act) {
    const double drho = pl.dD_ds / sbar - pl.D / (sbar * sbar);
    dsb += -2.0 * a.mu * a.dt * W0dotS * drho;
    dsb += gc * kq * (a.chi_inf - x) * (pl.D + sbar * pl.dD_ds);
    gchi += -2.0 * a.mu * a.dt * W0dotS * pl.dD_dchi / sbar;
    gchi += gc * kq * (sbar * pl.dD_dchi * (a.chi_inf - x) - sbar * pl.D);
  }
  gchi += gc;
#pragma unroll
  for (int p = 0; p < 3; ++p)
#pragma unroll
    for (int q = 0; q < 3; ++q) {
      double LtW = 0.0, WL = 0.0;
#pragma unroll
      for (int m = 0; m < 3; ++m) {
        LtW += L[m][p] * W[m][q];
        WL += W[p][m] * L[m][q];
      }
      double hpq = W[p][q] + a.dt * (LtW + WL - trL * W[p][q]);
      if (act) hpq += -2.0 * a.mu * a.dt * rho * W0[p][q] + dsb * S0[p][q] / (2.0 * sbar);
      H[p][q] = hpq;
    }
#pragma unroll
  for (int n = 0; n < 6; ++n) {
    const int p = VA[n], q = VB[n];
    g_sigma[n * N + t] = p == q ? H[p][p] : H[p][q] + H[q][p];
  }
  g_chi[t] = gchi;
}

// g_v_a(node) += scale * (G_h^T T)_a = -scale * sum_b d_b T_ab at interior
// nodes, T a full 3x3 cell tensor stored [9][cells].
__global__ __launch_bounds__(256) void k_grad_transpose_add(const double* __restrict__ T,
                                                            double* __restrict__ g_v, int nx,
                                                            int ny, int nz, double ih4,
                                                            double scale) {
  int i, j, k;
  NodeCells nc;
  const int t = blockIdx.x * blockDim.x + threadIdx.x;
  if (!node_of(t, nx, ny, nz, &i, &j, &k, &nc)) return;
  const int N = nx * ny * nz, P = nx * ny, C = (nz + 1) * P;
  const int o = k * P + j * nx + i;
#pragma unroll
  for (int p = 0; p < 3; ++p) {
    double acc = 0.0;
#pragma unroll
    for (int q = 0; q < 3; ++q) {
      double g[2][2][2];
#pragma unroll
      for (int ez = 0; ez < 2; ++ez)
#pragma unroll
        for (int ey = 0; ey < 2; ++ey)
#pragma unroll
          for (int ex = 0; ex < 2; ++ex) g[ez][ey][ex] = T[(p * 3 + q) * N + nc.cell[ez][ey][ex]];
      acc += node_diff(g, q);
    }
    g_v[p * C + o] -= scale * ih4 * acc;
  }
}

// g_sstar_n += -(1/dt) (G or G + G^T)_n with G = G_h g_b (walls of g_b as 0).
__global__ __launch_bounds__(256) void k_rhs_vjp(const double* __restrict__ g_b,
                                                 double* __restrict__ g_sstar, int nx, int ny,
                                                 int nz, double ih4, double scale) {
  CellIdx c;
  const int t = blockIdx.x * blockDim.x + threadIdx.x;
  if (!cell_of(t, nx, ny, nz, &c)) return;
  const int N = nx * ny * nz, P = nx * ny, C = (nz + 1) * P;
  const int xs[2] = {c.i, c.ip}, ys[2] = {c.j, c.jp};
  double G[3][3];
#pragma unroll
  for (int a = 0; a < 3; ++a) {
    double f[2][2][2];
#pragma unroll
    for (int dz = 0; dz < 2; ++dz) {
      const int kk = c.k + dz;
      const bool wall = (kk == 0 || kk == nz);
#pragma unroll
      for (int dy = 0; dy < 2; ++dy)
#pragma unroll
        for (int dx = 0; dx < 2; ++dx)
          f[dz][dy][dx] = wall ? 0.0 : g_b[a * C + kk * P + ys[dy] * nx + xs[dx]];
    }
    double gx = 0.0, gy = 0.0, gz = 0.0;
#pragma unroll
    for (int p = 0; p < 2; ++p)
#pragma unroll
      for (int q = 0; q < 2; ++q) {
        gx += f[p][q][1] - f[p][q][0];
        gy += f[p][1][q] - f[p][0][q];
        gz += f[1][p][q] - f[0][p][q];
      }
    G[a][0] = gx * ih4;
    G[a][1] = gy * ih4;
    G[a][2] = gz * ih4;
  }
#pragma unroll
  for (int n = 0; n < 6; ++n) {
    const int p = VA[n], q = VB[n];
    const double val = p == q ? G[p][p] : G[p][q] + G[q][p];
    g_sstar[n * N + t] -= scale * val;
  }
}

// g_v += G_h^T T(g_sigma), T_cd = dt (lam tr(g) delta_cd + mu (2 g_cc or g_{cd})),
// evaluated per node from the 8 surrounding cells.
__global__ __launch_bounds__(256) void k_stress_update_vjp(const double* __restrict__ gs,
                                                           double* __restrict__ g_v, int nx, int ny,
                                                           int nz, double ih4, double dt,
                                                           double lam, double mu) {
  int i, j, k;
  NodeCells nc;
  const int t = blockIdx.x * blockDim.x + threadIdx.x;
  if (!node_of(t, nx, ny, nz, &i, &j, &k, &nc)) return;
  const int N = nx * ny * nz, P = nx * ny, C = (nz + 1) * P;
  const int o = k * P + j * nx + i;
  double acc[3] = {0.0, 0.0, 0.0};
  // T[p][q] per cell is linear in the Voigt cotangent: accumulate d_q T[p][q]
  // directly from each Voigt component's node derivatives.
#pragma unroll
  for (int n = 0; n < 6; ++n) {
    double g[2][2][2];
#pragma unroll
    for (int ez = 0; ez < 2; ++ez)
#pragma unroll
      for (int ey = 0; ey < 2; ++ey)
#pragma unroll
        for (int ex = 0; ex < 2; ++ex) g[ez][ey][ex] = gs[n * N + nc.cell[ez][ey][ex]];
    const int p = VA[n], q = VB[n];
    if (p == q) {
      // lam * g_pp enters T_aa for every a; 2 mu g_pp enters T_pp
#pragma unroll
      for (int aa = 0; aa < 3; ++aa) acc[aa] += lam * node_diff(g, aa);
      acc[p] += 2.0 * mu * node_diff(g, p);
    } else {
      // mu g_pq enters T_pq and T_qp
      acc[p] += mu * node_diff(g, q);
      acc[q] += mu * node_diff(g, p);
    }
  }
#pragma unroll
  for (int a = 0; a < 3; ++a) g_v[a * C + o] -= dt * ih4 * acc[a];
}

inline int blocks_for(long long n, int bs) { return static_cast<int>((n + bs - 1) / bs); }

}  // namespace

void launch_stz_step(const double* v, const double* sigma, const double* chi, double* sstar,
                     double* chi1, double* dcell, Dims d, const StzArgs& a, hipStream_t s) {
  const long long n = static_cast<long long>(d.nx) * d.ny * d.nz;
  const dim3 grid(blocks_for(n, 256)), block(256);
  // the diffusion term reads D^pl of the six face neighbours: one pass first
  if (a.l2 > 0.0)
    hipLaunchKernelGGL(k_dpl_cells, grid, block, 0, s, sigma, chi, dcell, static_cast<int>(n), a);
  if (a.advect) {
    // z-segments of 32 cell planes, fewer when that leaves too few workgroups
    // one workgroup per (16 x 16 tile, plane); bands of 16 rows dealt
    // round-robin to the eight XCDs, each band plane by plane on its XCD
    const int ntx = (d.nx + kTile - 1) / kTile, bands = (d.ny + kTile - 1) / kTile;
    const long long wgs = 8LL * ((bands + 7) / 8) * d.nz * ntx;
    const dim3 g2(static_cast<unsigned>(wgs)), b2(kTile * kTile);
    if (a.l2 > 0.0)
      hipLaunchKernelGGL((k_stz_step_adv<true>), g2, b2, 0, s, v, sigma, chi, sstar, chi1, dcell,
                         d.nx, d.ny, d.nz, ntx, bands, a);
    else
      hipLaunchKernelGGL((k_stz_step_adv<false>), g2, b2, 0, s, v, sigma, chi, sstar, chi1, dcell,
                         d.nx, d.ny, d.nz, ntx, bands, a);
  } else if (a.l2 > 0.0) {
    hipLaunchKernelGGL((k_stz_step<true>), grid, block, 0, s, v, sigma, chi, sstar, chi1, dcell,
                       d.nx, d.ny, d.nz, a);
  } else {
    hipLaunchKernelGGL((k_stz_step<false>), grid, block, 0, s, v, sigma, chi, sstar, chi1, dcell,
                       d.nx, d.ny, d.nz, a);
  }
}

void launch_rhs(const double* sstar, double* b, Dims d, double h, double dt, hipStream_t s) {
  // z-segments of 16 node planes, fewer planes when that leaves too few workgroups
  const int P = d.nx * d.ny, interior = d.nz - 1;
  const int wgs = static_cast<int>(blocks_for(P, 256));
  int seg = 16;
  while (seg > 1 && wgs * ((interior + seg - 1) / seg) < 2048) seg /= 2;
  const int nseg = (interior + seg - 1) / seg;
  const int bpx = (wgs + 7) / 8;
  hipLaunchKernelGGL(k_rhs, dim3(8 * bpx * nseg), dim3(256), 0, s, sstar, b, d.nx, d.ny, d.nz, seg,
                     wgs, bpx, 0.25 / (h * dt));
  hipLaunchKernelGGL(k_zero_walls, dim3(blocks_for(6LL * d.plane(), 256)), dim3(256), 0, s, b,
                     d.nx, d.ny, d.nz);
}

void launch_stress_update(const double* sstar, const double* v, double* out, Dims d, double h,
                          double dt, double lam, double mu, hipStream_t s) {
  const long long n = static_cast<long long>(d.nx) * d.ny * d.nz;
  hipLaunchKernelGGL(k_stress_update, dim3(blocks_for(n, 256)), dim3(256), 0, s, sstar, v, out,
                     d.nx, d.ny, d.nz, h, dt, lam, mu);
}

void launch_explicit_velocity(const double* v, const double* sigma, double* vout, Dims d, double h,
                              double dt, double rho, double kappa, hipStream_t s) {
  const long long n = static_cast<long long>(d.nx) * d.ny * (d.nz - 1);
  hipLaunchKernelGGL(k_explicit_velocity, dim3(blocks_for(n, 256)), dim3(256), 0, s, v, sigma, vout,
                     d.nx, d.ny, d.nz, h, dt, rho, kappa);
}

void launch_set_walls(double* v, Dims d, double U, hipStream_t s) {
  hipLaunchKernelGGL(k_set_walls, dim3(blocks_for(2LL * d.plane(), 256)), dim3(256), 0, s, v, d.nx,
                     d.ny, d.nz, U);
}

void launch_copy_walls(double* v, const double* lo, const double* hi, Dims d, hipStream_t s) {
  hipLaunchKernelGGL(k_copy_walls, dim3(blocks_for(3LL * d.plane(), 256)), dim3(256), 0, s, v, lo,
                     hi, d.nx, d.ny, d.nz);
}

void launch_stz_step_vjp(const double* v, const double* sigma, const double* chi,
                         const double* g_sstar, const double* g_chi1, double* g_sigma,
                         double* g_chi, double* g_L, Dims d, const StzArgs& a, hipStream_t s) {
  const long long n = static_cast<long long>(d.nx) * d.ny * d.nz;
  hipLaunchKernelGGL(k_stz_step_vjp, dim3(blocks_for(n, 256)), dim3(256), 0, s, v, sigma, chi,
                     g_sstar, g_chi1, g_sigma, g_chi, g_L, d.nx, d.ny, d.nz, a);
}

void launch_grad_transpose_add(const double* g_L, double* g_v, Dims d, double h, double scale,
                               hipStream_t s) {
  const long long n = static_cast<long long>(d.nx) * d.ny * (d.nz - 1);
  hipLaunchKernelGGL(k_grad_transpose_add, dim3(blocks_for(n, 256)), dim3(256), 0, s, g_L, g_v,
                     d.nx, d.ny, d.nz, 0.25 / h, scale);
}

void launch_rhs_vjp(const double* g_b, double* g_sstar, Dims d, double h, double dt,
                    hipStream_t s) {
  const long long n = static_cast<long long>(d.nx) * d.ny * d.nz;
  hipLaunchKernelGGL(k_rhs_vjp, dim3(blocks_for(n, 256)), dim3(256), 0, s, g_b, g_sstar, d.nx,
                     d.ny, d.nz, 0.25 / h, 1.0 / dt);
}

void launch_stress_update_vjp(const double* g_sigma, double* g_v, Dims d, double h, double dt,
                              double lam, double mu, hipStream_t s) {
  const long long n = static_cast<long long>(d.nx) * d.ny * (d.nz - 1);
  hipLaunchKernelGGL(k_stress_update_vjp, dim3(blocks_for(n, 256)), dim3(256), 0, s, g_sigma, g_v,
                     d.nx, d.ny, d.nz, 0.25 / h, dt, lam, mu);
}

}  // namespace qs
