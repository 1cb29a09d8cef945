// Internal launcher declarations shared by the HIP translation units.
#pragma once
#include <hip/hip_runtime.h>

#include <cstddef>

namespace qs {

// Level geometry: node arrays are [3][nz+1][ny][nx], x fastest.
struct Dims {
  int nx, ny, nz;
  int plane() const { return nx * ny; }
  int comp() const { return (nz + 1) * nx * ny; }  // elements per component
  size_t elems() const { return 3ull * comp(); }
};

// Fine-operator coefficients in the form the fine smoother uses:
//   x_c = (h2 b_c + sum_a kap_ca (x_c(+e_a) + x_c(-e_a)) + m4 * mixed) * inv_diag
template <typename T>
struct FineCoef {
  T h2;        // h^2
  T p, q;      // lambda + 2 mu (along the component), mu (across it)
  T m4;        // (lambda + mu) / 4
  T inv_diag;  // 1 / (2 (lambda + 4 mu))
  T ih2;       // 1 / h^2 (residual form)
};

constexpr int kReduceBlock = 256;

// Two-wide loads and stores with the non-temporal hint, for data a launch
// touches once (so that L2 keeps what neighbouring workgroups share).  V is
// the two-wide HIP type of T (float2, double2).
template <typename T>
struct NT2 {
  typedef T E __attribute__((ext_vector_type(2)));
  template <typename V>
  __device__ static __forceinline__ V load(const T* p) {
    const E e = __builtin_nontemporal_load(reinterpret_cast<const E*>(p));
    V v;
    v.x = e.x;
    v.y = e.y;
    return v;
  }
  template <typename V>
  __device__ static __forceinline__ void store(T* p, const V& v) {
    E e;
    e.x = v.x;
    e.y = v.y;
    __builtin_nontemporal_store(e, reinterpret_cast<E*>(p));
  }
};

// --- multigrid kernels (kernels_mg.hip) -----------------------------------
template <typename T>
void launch_colour_fine(T* x, const T* b, Dims d, int colour, const FineCoef<T>& c, hipStream_t s);
template <typename T>
void launch_colour_gen(T* x, const T* b, Dims d, int colour, const T* S, const T* Dinv,
                       hipStream_t s);
// Colours c and c ^ 1 (c first) in one launch on a level with the generic
// stencil, given in packed form (packed_stencil.h); needs an even row length
// of at most 512.
template <typename T>
void launch_colour_pair_gen(T* x, const T* b, Dims d, int colour, const T* Pst, hipStream_t s);
bool colour_pair_supported(Dims d);
// The column pairs of a row fill a power-of-two run of at most 64 lanes, so
// the pair kernels take the outer window columns by lane shuffles.
bool pair_rows_in_lanes(Dims d);
// Coarse residual r = b - A x on the interior, two nodes per thread (even nx,
// 16-byte aligned vectors), packed stencil.
template <typename T>
void launch_residual_pair_gen(const T* x, const T* b, T* r, Dims d, const T* Pst, hipStream_t s);

// Fine-level row-parity half sweep (kernels_sweep.hip): updates every node
// of the rows with parity row_par, reading own rows from own_src, neighbour
// rows from nbr_src and writing dst.  zero = 1: own rows are known to be 0
// and not read; zero = 2: own and neighbour rows (x_first = 0 only).
// zero = 3: own and neighbour rows are read as x + T ec (the coarse
// correction ec prolongated on the fly); zero = 4: own rows only (both
// x_first = 1, row_par 1 and 0, the two halves of the first post-smoothing
// sweep; ec is the coarse level's correction, null otherwise).
template <typename T>
void launch_sweep_half(const T* own_src, const T* nbr_src, T* dst, const T* b, const T* ec, Dims d,
                       int row_par, int plane_first, int x_first, const FineCoef<T>& cf, int seg,
                       int seg_major, int zero, hipStream_t s);
int sweep_rows_per_group(int nx);  // rows of one parity per workgroup
int sweep_segment_length(Dims d, int bytes_per_value);  // z planes per workgroup
int sweep_lds_bytes(Dims d, int bytes_per_value);
bool sweep_supported(Dims d, size_t lds_limit, int bytes_per_value);
void sweep_set_lds_limit(size_t bytes);

// r = b - A x on interior nodes (walls of r = 0).  If `zero_interior`, x's
// interior is treated as 0 (r = b - A_IB x_B).  If `partial` is non-null,
// per-block sums of r^2 (in double) go to partial[blockIdx].  `r` may be
// null (norm only).  Returns the number of blocks used (for the reduction).
// The output may be scaled: r_out = (b - A x) * out_scale.
template <typename Tin, typename Tout>
int launch_residual_fine(const Tin* x, const Tin* b, Tout* r, Dims d, const FineCoef<double>& c,
                         double out_scale, bool zero_interior, double* partial, hipStream_t s);
template <typename T>
int launch_residual_gen(const T* x, const T* b, T* r, Dims d, const T* Pst, bool zero_interior,
                        double* partial, hipStream_t s);
int residual_blocks(Dims d);  // upper bound on the partial sums any residual kernel writes

// Fine-operator residual by z-marching tiles (kernels_resid.hip): same
// contract as launch_residual_fine with zero_interior = false; b may be null
// (treated as 0).  Returns the number of partial sums written.
template <typename Tin, typename Tout>
int launch_residual_fine_zm(const Tin* x, const Tin* b, Tout* r, Dims d, const FineCoef<double>& c,
                            double out_scale, double* partial, hipStream_t s);
int resid_zmarch_blocks(Dims d);
// The same for the refinement loop: x_out = x + es * e on the interior (x_out
// must not be x), r = (b - K x_out) * out_scale in FP32, partial sums of the
// unscaled r^2.  Returns the number of partial sums.
int launch_update_residual_zm(const double* x, const float* e, double es, double* x_out,
                              const double* b, float* r, Dims d, const FineCoef<double>& c,
                              double out_scale, double* partial, hipStream_t s);
// Fine level: bc = T^T (b - K x) on the interior coarse nodes, without
// writing the fine residual (kernels_resid.hip).  nx, ny, nz even.  With xc
// non-null, the coarse correction is cleared at the same interior nodes.
template <typename T>
void launch_resid_restrict(const T* x, const T* b, T* bc, T* xc, Dims d,
                           const FineCoef<double>& c, hipStream_t s);

// bc = T^T r; with xc non-null, also xc = 0 at the interior coarse nodes.
template <typename T>
void launch_restrict(const T* r, T* bc, T* xc, Dims fine, hipStream_t s);
template <typename T>
void launch_prolong_add(T* x, const T* ec, Dims fine, hipStream_t s);

// Deterministic sum of partial[0..n) into out[0].
// Sum of n partials in a fixed order into out[0] (device) and, if given,
// out_host[0] (device address of pinned host memory).
void launch_reduce_sum(const double* partial, int n, double* out, double* out_host,
                       hipStream_t s);

template <typename T>
void launch_fill(T* x, size_t n, T value, hipStream_t s);
// Zero the interior planes of a node vector.
template <typename T>
void launch_zero_interior(T* x, Dims d, hipStream_t s);

// Coarsest level: x_interior = Ainv b_interior, computed in double in one
// launch (interior unknowns ordered by component, plane, row, column).
template <typename T>
void launch_coarse_solve(const double* Ainv, int n, const T* b, T* x, Dims d, hipStream_t s);

// --- STZ / projection kernels (kernels_stz.hip) -----------------------------
struct StzArgs {
  double s_y, tau0, beta, delta_over_T, c0, chi_inf, dt;
  double lam, mu, h;
  double l2;  // squared diffusion length of Eq. chi_evo (0: no diffusion term)
  int n_sub;  // plastic sub-steps: 1 single step, > 1 fixed count, -1 per cell, -2 backward Euler
  int advect; // 1: sigma* carries the advection -(v . grad) sigma (Eq. ENO)
  int chi_wall;  // 1: no chi diffusion flux through the wall faces
};
// dcell: device scratch of nx*ny*nz doubles, used when a.l2 > 0 (may be null otherwise)
void launch_stz_step(const double* v, const double* sigma, const double* chi, double* sstar,
                     double* chi1, double* dcell, Dims d, const StzArgs& a, hipStream_t s);
void launch_rhs(const double* sstar, double* b, Dims d, double h, double dt, hipStream_t s);
void launch_stress_update(const double* sstar, const double* v, double* out, Dims d, double h,
                          double dt, double lam, double mu, hipStream_t s);
void launch_set_walls(double* v, Dims d, double U, hipStream_t s);
void launch_explicit_velocity(const double* v, const double* sigma, double* vout, Dims d, double h,
                              double dt, double rho, double kappa, hipStream_t s);
void launch_copy_walls(double* v, const double* lo, const double* hi, Dims d, hipStream_t s);
void launch_stz_step_vjp(const double* v, const double* sigma, const double* chi,
                         const double* g_sstar, const double* g_chi1, double* g_sigma,
                         double* g_chi, double* g_L, Dims d, const StzArgs& a, hipStream_t s);
void launch_grad_transpose_add(const double* g_L, double* g_v, Dims d, double h, double scale,
                               hipStream_t s);
void launch_rhs_vjp(const double* g_b, double* g_sstar, Dims d, double h, double dt,
                    hipStream_t s);
void launch_stress_update_vjp(const double* g_sigma, double* g_v, Dims d, double h, double dt,
                              double lam, double mu, hipStream_t s);

}  // namespace qs
