// Row-parity Gauss-Seidel sweep for gfx950 (smoother of Sec. 3.6).
//
// Colour order.  With colour c = (i&1) + 2(j&1) + 4(k&1), the pre-smoothing
// order 0,1,4,5,2,3,6,7 visits all nodes of even rows j first (colours 0,1,4,5)
// and then all nodes of odd rows (2,3,6,7); post-smoothing runs the reverse.
// A node of an even row couples only to nodes of its own row and of the two
// odd rows next to it, so while even rows are updated the odd rows are
// read-only, and the whole half-sweep is one launch: every row of the active
// parity is an independent (x, z) problem with four colours
//   (first x parity, first z parity), (second x, first z),
//   (first x, second z),              (second x, second z).
//
// Work split.  One workgroup takes R rows of one parity (all of x, so the
// periodic wrap in x stays inside the workgroup) over a segment of z planes
// and marches up the segment: each first-parity plane f is updated (two
// x-parity phases with a barrier between them), then the second-parity plane
// f-1, which needs the new planes f-2 and f.  Planes f-2..f+1 of the row and
// of its two neighbour rows sit in an LDS ring of four planes; every global
// value is loaded once per workgroup.  The second-parity planes at the
// segment ends need first-parity planes just outside the segment: the
// workgroup recomputes those (one plane per end) from old values, so the
// sweep reads `own_src` / `nbr_src` and writes `dst` (ping-pong buffers):
//   even-row half: own rows and neighbour rows from the old vector,
//   odd-row half:  own rows from the old vector, neighbour rows from the new.
// Workgroups are mapped so that each XCD (round-robin dispatch over 8) gets a
// contiguous block of (row, segment) pairs: the segments of one row and the
// rows next to each other then run on the same XCD and share halo planes and
// neighbour rows through its L2.
#include <hip/hip_runtime.h>

#include "device.h"

namespace qs {

namespace {

struct SweepArgs {
  int nx, ny, nz;
  int row_par;      // parity of the rows updated
  int plane_first;  // parity of the planes updated first
  int x_first;      // parity of the columns updated first in each plane
  int seg;          // planes per segment
  int nseg;         // segments
  int rows_per_wg;  // rows of this parity per workgroup
  int ngroups;      // workgroups per segment column
  int real_wgs;     // ngroups * nseg
  int grid_per_xcd; // padded grid / 8
};


// Per-thread context of the sweep: indices and pointers that every helper
// needs, passed by value so that everything stays in registers.
template <typename T>
struct SweepCtx {
  T* ring;           // LDS ring [4][rows][3 rows][3 comps][nx]
  int nx, rows, r, i, im, ip;
  int j, jm, jp;
  size_t P, C;
  bool active;
};

template <typename T>
__device__ __forceinline__ int ring_idx(const SweepCtx<T>& c, int plane, int rr, int comp, int col) {
  return ((((plane & 3) * c.rows + c.r) * 3 + rr) * 3 + comp) * c.nx + col;
}

template <typename T>
__device__ __forceinline__ T rget(const SweepCtx<T>& c, int plane, int rr, int comp, int col) {
  return c.ring[ring_idx(c, plane, rr, comp, col)];
}

template <typename T>
__device__ __forceinline__ void load_plane(const SweepCtx<T>& c, const T* __restrict__ own_src,
                                           const T* __restrict__ nbr_src, int p) {
  if (!c.active) return;
  const size_t o = static_cast<size_t>(p) * c.P + c.i;
  const size_t om = o + static_cast<size_t>(c.jm) * c.nx;
  const size_t oo = o + static_cast<size_t>(c.j) * c.nx;
  const size_t op = o + static_cast<size_t>(c.jp) * c.nx;
#pragma unroll
  for (int k = 0; k < 3; ++k) {
    const T vm = nbr_src[k * c.C + om];
    const T vo = own_src[k * c.C + oo];
    const T vp = nbr_src[k * c.C + op];
    c.ring[ring_idx(c, p, 0, k, c.i)] = vm;
    c.ring[ring_idx(c, p, 1, k, c.i)] = vo;
    c.ring[ring_idx(c, p, 2, k, c.i)] = vp;
  }
}

// Values of one plane (three rows, three components) held in registers
// between the global load and the store into the ring.
template <typename T>
struct PlaneRegs {
  T v[9];
};

template <typename T>
__device__ __forceinline__ void fetch_plane(const SweepCtx<T>& c, const T* __restrict__ own_src,
                                            const T* __restrict__ nbr_src, int p, PlaneRegs<T>& out) {
  if (!c.active) return;
  const size_t o = static_cast<size_t>(p) * c.P + c.i;
  const size_t om = o + static_cast<size_t>(c.jm) * c.nx;
  const size_t oo = o + static_cast<size_t>(c.j) * c.nx;
  const size_t op = o + static_cast<size_t>(c.jp) * c.nx;
#pragma unroll
  for (int k = 0; k < 3; ++k) {
    out.v[3 * k] = nbr_src[k * c.C + om];
    out.v[3 * k + 1] = own_src[k * c.C + oo];
    out.v[3 * k + 2] = nbr_src[k * c.C + op];
  }
}

template <typename T>
__device__ __forceinline__ void store_plane(const SweepCtx<T>& c, int p, const PlaneRegs<T>& in) {
  if (!c.active) return;
#pragma unroll
  for (int k = 0; k < 3; ++k) {
    c.ring[ring_idx(c, p, 0, k, c.i)] = in.v[3 * k];
    c.ring[ring_idx(c, p, 1, k, c.i)] = in.v[3 * k + 1];
    c.ring[ring_idx(c, p, 2, k, c.i)] = in.v[3 * k + 2];
  }
}

// Gauss-Seidel value of the node (row j, plane p, column i) from the ring:
// x = D^-1 (b - sum_{q != p} A_pq x_q).  Rows in the ring: 0 = j-1, 1 = j, 2 = j+1.
template <typename T>
__device__ __forceinline__ void gs_fine(const SweepCtx<T>& c, int p, T b0, T b1, T b2,
                                        const FineCoef<T> cf, T& o0, T& o1, T& o2) {
  const int i = c.i, im = c.im, ip = c.ip;
#define RX(rr, k, dz, col) rget(c, p + (dz), rr, k, col)
  const T fx0 = RX(1, 0, 0, ip) + RX(1, 0, 0, im);
  const T fy0 = RX(2, 0, 0, i) + RX(0, 0, 0, i);
  const T fz0 = RX(1, 0, 1, i) + RX(1, 0, -1, i);
  const T fx1 = RX(1, 1, 0, ip) + RX(1, 1, 0, im);
  const T fy1 = RX(2, 1, 0, i) + RX(0, 1, 0, i);
  const T fz1 = RX(1, 1, 1, i) + RX(1, 1, -1, i);
  const T fx2 = RX(1, 2, 0, ip) + RX(1, 2, 0, im);
  const T fy2 = RX(2, 2, 0, i) + RX(0, 2, 0, i);
  const T fz2 = RX(1, 2, 1, i) + RX(1, 2, -1, i);
  // mixed differences f(+,+) - f(+,-) - f(-,+) + f(-,-)
  const T mxy0 = RX(2, 0, 0, ip) - RX(0, 0, 0, ip) - RX(2, 0, 0, im) + RX(0, 0, 0, im);
  const T mxy1 = RX(2, 1, 0, ip) - RX(0, 1, 0, ip) - RX(2, 1, 0, im) + RX(0, 1, 0, im);
  const T mxz0 = RX(1, 0, 1, ip) - RX(1, 0, -1, ip) - RX(1, 0, 1, im) + RX(1, 0, -1, im);
  const T mxz2 = RX(1, 2, 1, ip) - RX(1, 2, -1, ip) - RX(1, 2, 1, im) + RX(1, 2, -1, im);
  const T myz1 = RX(2, 1, 1, i) - RX(2, 1, -1, i) - RX(0, 1, 1, i) + RX(0, 1, -1, i);
  const T myz2 = RX(2, 2, 1, i) - RX(2, 2, -1, i) - RX(0, 2, 1, i) + RX(0, 2, -1, i);
#undef RX
  o0 = (cf.h2 * b0 + cf.p * fx0 + cf.q * (fy0 + fz0) + cf.m4 * (mxy1 + mxz2)) * cf.inv_diag;
  o1 = (cf.h2 * b1 + cf.p * fy1 + cf.q * (fx1 + fz1) + cf.m4 * (mxy0 + myz2)) * cf.inv_diag;
  o2 = (cf.h2 * b2 + cf.p * fz2 + cf.q * (fx2 + fy2) + cf.m4 * (mxz0 + myz1)) * cf.inv_diag;
}

// Generic 27-point block stencil; K holds the plane's 243 stencil entries
// followed by the 9 entries of the inverse centre block (staged in LDS).
template <typename T>
__device__ __forceinline__ void gs_gen(const SweepCtx<T>& c, int p, T b0, T b1, T b2,
                                       const T* K, T& o0, T& o1, T& o2) {
  T a0 = b0, a1 = b1, a2 = b2;
#pragma unroll 3
  for (int q = 0; q < 27; ++q) {
    if (q == 13) continue;
    const int oz = q / 9 - 1, oy = (q / 3) % 3, ox = q % 3;
    const int col = ox == 0 ? c.im : (ox == 1 ? c.i : c.ip);
    const T n0 = rget(c, p + oz, oy, 0, col);
    const T n1 = rget(c, p + oz, oy, 1, col);
    const T n2 = rget(c, p + oz, oy, 2, col);
    const T* B = K + q * 9;
    a0 -= B[0] * n0 + B[1] * n1 + B[2] * n2;
    a1 -= B[3] * n0 + B[4] * n1 + B[5] * n2;
    a2 -= B[6] * n0 + B[7] * n1 + B[8] * n2;
  }
  const T* Di = K + 243;
  o0 = Di[0] * a0 + Di[1] * a1 + Di[2] * a2;
  o1 = Di[3] * a0 + Di[4] * a1 + Di[5] * a2;
  o2 = Di[6] * a0 + Di[7] * a1 + Di[8] * a2;
}

constexpr int kCoef = 252;  // 243 stencil + 9 inverse centre block, per plane

// Update all nodes of plane p whose column parity is xp; write them to the
// ring and, for planes of this segment, to dst.  bv: b at this node.
template <typename T, bool FINE>
__device__ __forceinline__ void update_phase(const SweepCtx<T>& c, int p, int xp, int z0, int z1,
                                             const T bv[3], T* __restrict__ dst,
                                             const FineCoef<T> cf, const T* K) {
  if (!c.active || (c.i & 1) != xp) return;
  T o0, o1, o2;
  if (FINE)
    gs_fine<T>(c, p, bv[0], bv[1], bv[2], cf, o0, o1, o2);
  else
    gs_gen<T>(c, p, bv[0], bv[1], bv[2], K, o0, o1, o2);
  c.ring[ring_idx(c, p, 1, 0, c.i)] = o0;
  c.ring[ring_idx(c, p, 1, 1, c.i)] = o1;
  c.ring[ring_idx(c, p, 1, 2, c.i)] = o2;
  if (p >= z0 && p < z1) {
    const size_t bo = static_cast<size_t>(p) * c.P + static_cast<size_t>(c.j) * c.nx + c.i;
    dst[bo] = o0;
    dst[c.C + bo] = o1;
    dst[2 * c.C + bo] = o2;
  }
}

template <typename T>
__device__ __forceinline__ void fetch_b(const SweepCtx<T>& c, const T* __restrict__ b, int p, int nz,
                                        T out[3]) {
  if (!c.active || p < 1 || p > nz - 1) return;
  const size_t bo = static_cast<size_t>(p) * c.P + static_cast<size_t>(c.j) * c.nx + c.i;
  out[0] = b[bo];
  out[1] = b[c.C + bo];
  out[2] = b[2 * c.C + bo];
}

// Coefficients of planes pa and pb (kCoef each), split over the workgroup's
// threads: at most 3 values per thread for workgroups of >= 168 threads.
template <typename T>
__device__ __forceinline__ void fetch_coef(const T* __restrict__ S, const T* __restrict__ Dinv,
                                           int pa, int pb, int nz, T out[3]) {
  const int nt = blockDim.x;
#pragma unroll
  for (int u = 0; u < 3; ++u) {
    const int idx = threadIdx.x + u * nt;
    if (idx < 2 * kCoef) {
      const int pl = idx < kCoef ? pa : pb;
      const int k = idx < kCoef ? idx : idx - kCoef;
      T v = T(0);
      if (pl >= 0 && pl <= nz)
        v = k < 243 ? S[static_cast<size_t>(pl) * 243 + k] : Dinv[static_cast<size_t>(pl) * 9 + k - 243];
      out[u] = v;
    }
  }
}

template <typename T>
__device__ __forceinline__ void store_coef(T* set, const T in[3]) {
  const int nt = blockDim.x;
#pragma unroll
  for (int u = 0; u < 3; ++u) {
    const int idx = threadIdx.x + u * nt;
    if (idx < 2 * kCoef) set[idx] = in[u];
  }
}

template <typename T, bool FINE>
__global__ __launch_bounds__(512) void k_sweep_rows(const T* __restrict__ own_src,
                                                    const T* __restrict__ nbr_src,
                                                    T* __restrict__ dst, const T* __restrict__ b,
                                                    SweepArgs a, FineCoef<T> cf,
                                                    const T* __restrict__ S,
                                                    const T* __restrict__ Dinv) {
  extern __shared__ __align__(16) unsigned char smem[];
  // XCD-aware mapping of the (padded) grid onto (row group, segment)
  const int wg = blockIdx.x;
  const int L = (wg & 7) * a.grid_per_xcd + (wg >> 3);
  if (L >= a.real_wgs) return;  // whole workgroup leaves before any barrier
  const int group = L / a.nseg, sgi = L - group * a.nseg;
  SweepCtx<T> c;
  c.ring = reinterpret_cast<T*>(smem);
  c.nx = a.nx;
  c.rows = a.rows_per_wg;
  c.r = threadIdx.x / a.nx;
  c.i = threadIdx.x - c.r * a.nx;
  c.im = c.i == 0 ? a.nx - 1 : c.i - 1;
  c.ip = c.i + 1 == a.nx ? 0 : c.i + 1;
  const int rowidx = group * a.rows_per_wg + c.r;
  c.j = 2 * rowidx + a.row_par;
  c.active = (c.r < a.rows_per_wg) && (c.j < a.ny);
  c.jm = c.j == 0 ? a.ny - 1 : c.j - 1;
  c.jp = c.j + 1 >= a.ny ? c.j + 1 - a.ny : c.j + 1;
  c.P = static_cast<size_t>(a.nx) * a.ny;
  c.C = static_cast<size_t>(a.nz + 1) * c.P;

  const int nz = a.nz;
  const int z0 = 1 + sgi * a.seg;
  const int z1 = min(z0 + a.seg, nz);  // segment = interior planes [z0, z1)
  const int pf = a.plane_first, x1 = a.x_first, x2 = 1 - a.x_first;
  // first-parity planes: parity pf, interior, in [z0-1, z1]
  int f0 = max(z0 - 1, 1);
  if ((f0 & 1) != pf) ++f0;
  int flast = min(z1, nz - 1);
  if ((flast & 1) != pf) --flast;
  if (f0 > flast) return;  // uniform over the workgroup

  // The ring holds planes f-2 .. f+1 while planes f and f-1 are updated;
  // planes f+2 and f+3, b at planes f+2 and f+1 and (generic stencil) the
  // coefficients of planes f+2 and f+1 are fetched into registers before
  // those updates and stored once the slots they replace are no longer read.
  // Coefficients sit in two sets [plane f | plane f-1], alternating per step.
  T* coef = c.ring + 4 * a.rows_per_wg * 9 * a.nx;
  if (f0 - 1 >= z0) load_plane<T>(c, own_src, nbr_src, f0 - 2);  // bottom segment: wall below
  load_plane<T>(c, own_src, nbr_src, f0 - 1);
  load_plane<T>(c, own_src, nbr_src, f0);
  load_plane<T>(c, own_src, nbr_src, f0 + 1);  // f0 + 1 <= nz
  T bf[3] = {T(0), T(0), T(0)}, bs[3] = {T(0), T(0), T(0)};
  fetch_b<T>(c, b, f0, nz, bf);
  fetch_b<T>(c, b, f0 - 1, nz, bs);
  if (!FINE) {
    T cv[3] = {T(0), T(0), T(0)};
    fetch_coef<T>(S, Dinv, f0, f0 - 1, nz, cv);
    store_coef<T>(coef, cv);
  }
  __syncthreads();
  // Drain the prologue loads here.  Memory counters complete in order, so a
  // wait for a prologue load that the compiler would otherwise place inside
  // the loop (it cannot tell iterations apart) would also wait for every
  // prefetch issued in that iteration.
  __builtin_amdgcn_s_waitcnt(0);
  PlaneRegs<T> pa, pb;
  int set = 0;
  for (int f = f0; f <= flast; f += 2) {
    const bool more_a = f + 2 <= nz, more_b = f + 3 <= nz;
    if (more_a) fetch_plane<T>(c, own_src, nbr_src, f + 2, pa);
    if (more_b) fetch_plane<T>(c, own_src, nbr_src, f + 3, pb);
    T bf_n[3] = {T(0), T(0), T(0)}, bs_n[3] = {T(0), T(0), T(0)};
    fetch_b<T>(c, b, f + 2, nz, bf_n);
    fetch_b<T>(c, b, f + 1, nz, bs_n);
    T cv[3] = {T(0), T(0), T(0)};
    if (!FINE) fetch_coef<T>(S, Dinv, f + 2, f + 1, nz, cv);
    const T* Kf = coef + set * 2 * kCoef;
    const T* Ks = Kf + kCoef;
    update_phase<T, FINE>(c, f, x1, z0, z1, bf, dst, cf, Kf);
    __syncthreads();
    update_phase<T, FINE>(c, f, x2, z0, z1, bf, dst, cf, Kf);
    __syncthreads();
    const int sp = f - 1;  // second-parity plane below f
    if (sp >= z0 && sp <= z1 - 1 && sp >= 1) {
      update_phase<T, FINE>(c, sp, x1, z0, z1, bs, dst, cf, Ks);
      __syncthreads();
      update_phase<T, FINE>(c, sp, x2, z0, z1, bs, dst, cf, Ks);
      __syncthreads();
    }
    if (more_a) store_plane<T>(c, f + 2, pa);
    if (more_b) store_plane<T>(c, f + 3, pb);
    set ^= 1;
    if (!FINE) store_coef<T>(coef + set * 2 * kCoef, cv);
#pragma unroll
    for (int k = 0; k < 3; ++k) {
      bf[k] = bf_n[k];
      bs[k] = bs_n[k];
    }
    __syncthreads();
  }
  const int sp = flast + 1;  // only when flast + 2 is the top wall (already in the ring)
  if (sp >= z0 && sp <= z1 - 1 && sp <= nz - 1) {
    const T* Ks = coef + set * 2 * kCoef + kCoef;  // plane flast + 1, fetched as "f + 1"
    update_phase<T, FINE>(c, sp, x1, z0, z1, bs, dst, cf, Ks);
    __syncthreads();
    update_phase<T, FINE>(c, sp, x2, z0, z1, bs, dst, cf, Ks);
  }
}

}  // namespace

int sweep_lds_bytes(Dims d, int bytes_per_value, bool fine) {
  // ring of four planes x rows x 3 rows x 3 components; the generic stencil
  // adds two double-buffered coefficient sets of two planes each
  const int rpw = d.nx >= 256 ? 1 : 256 / d.nx;
  return (4 * rpw * 9 * d.nx + (fine ? 0 : 4 * kCoef)) * bytes_per_value;
}

template <typename T>
void launch_sweep_half(const T* own_src, const T* nbr_src, T* dst, const T* b, Dims d, int row_par,
                       int plane_first, int x_first, const FineCoef<T>& cf, const T* S,
                       const T* Dinv, bool fine, int seg, hipStream_t s) {
  SweepArgs a;
  a.nx = d.nx;
  a.ny = d.ny;
  a.nz = d.nz;
  a.row_par = row_par;
  a.plane_first = plane_first;
  a.x_first = x_first;
  a.seg = seg;
  a.nseg = (d.nz - 1 + seg - 1) / seg;
  a.rows_per_wg = d.nx >= 256 ? 1 : 256 / d.nx;
  const int rows = (d.ny - row_par + 1) / 2;
  a.ngroups = (rows + a.rows_per_wg - 1) / a.rows_per_wg;
  a.real_wgs = a.ngroups * a.nseg;
  a.grid_per_xcd = (a.real_wgs + 7) / 8;
  const int threads = a.rows_per_wg * d.nx;
  const size_t lds = static_cast<size_t>(sweep_lds_bytes(d, sizeof(T), fine));
  if (fine)
    hipLaunchKernelGGL((k_sweep_rows<T, true>), dim3(8 * a.grid_per_xcd), dim3(threads), lds, s,
                       own_src, nbr_src, dst, b, a, cf, S, Dinv);
  else
    hipLaunchKernelGGL((k_sweep_rows<T, false>), dim3(8 * a.grid_per_xcd), dim3(threads), lds, s,
                       own_src, nbr_src, dst, b, a, cf, S, Dinv);
}

void sweep_set_lds_limit(size_t bytes) {
  (void)hipFuncSetAttribute(reinterpret_cast<const void*>(&k_sweep_rows<double, true>),
                            hipFuncAttributeMaxDynamicSharedMemorySize, static_cast<int>(bytes));
  (void)hipFuncSetAttribute(reinterpret_cast<const void*>(&k_sweep_rows<double, false>),
                            hipFuncAttributeMaxDynamicSharedMemorySize, static_cast<int>(bytes));
  (void)hipFuncSetAttribute(reinterpret_cast<const void*>(&k_sweep_rows<float, true>),
                            hipFuncAttributeMaxDynamicSharedMemorySize, static_cast<int>(bytes));
  (void)hipFuncSetAttribute(reinterpret_cast<const void*>(&k_sweep_rows<float, false>),
                            hipFuncAttributeMaxDynamicSharedMemorySize, static_cast<int>(bytes));
}

template void launch_sweep_half<double>(const double*, const double*, double*, const double*, Dims,
                                        int, int, int, const FineCoef<double>&, const double*,
                                        const double*, bool, int, hipStream_t);
template void launch_sweep_half<float>(const float*, const float*, float*, const float*, Dims, int,
                                       int, int, const FineCoef<float>&, const float*,
                                       const float*, bool, int, hipStream_t);

}  // namespace qs
