// Multigrid kernels for gfx950 (paper Sec. 3.6).
//
// Node vectors are structure-of-arrays [3][nz+1][ny][nx] with x fastest, so
// consecutive lanes of a 64-wide wavefront touch consecutive x addresses.
// x and y wrap periodically; planes k = 0 and k = nz are walls and are never
// written by any kernel here.
//
// Smoothing is multicolour block Gauss-Seidel: colour c = (i&1) + 2(j&1) +
// 4(k&1).  Nodes of one colour are never coupled by the 3x3x3 stencil, so a
// colour pass updates them in place in any order without races.
#include <algorithm>
#include <type_traits>

#include "device.h"
#include "packed_stencil.h"

namespace qs {

namespace {

struct ColourRange {
  int a, bb, kfirst, hx, hy, nk;
  __host__ __device__ int total() const { return hx * hy * nk; }
};

ColourRange colour_range(Dims d, int colour) {
  ColourRange r;
  r.a = colour & 1;
  r.bb = (colour >> 1) & 1;
  const int e = (colour >> 2) & 1;
  r.kfirst = e ? 1 : 2;
  r.hx = (d.nx - r.a + 1) / 2;
  r.hy = (d.ny - r.bb + 1) / 2;
  r.nk = (d.nz - 1 - r.kfirst) >= 0 ? (d.nz - 1 - r.kfirst) / 2 + 1 : 0;
  return r;
}

__device__ __forceinline__ int wrap_m(int i, int n) { return i == 0 ? n - 1 : i - 1; }
__device__ __forceinline__ int wrap_p(int i, int n) { return i == n - 1 ? 0 : i + 1; }

// Sum of the off-diagonal part of the fine operator (times h^2, sign moved
// to the right-hand side) for component c at node (i, j, k):
//   sum_a kap_ca (x_c(+e_a) + x_c(-e_a)) + (lam+mu)/4 sum_{d!=c} sum_{s,t} s t x_d(p + s e_c + t e_d)
template <typename T>
struct FineNbr {
  const T* __restrict__ x;
  int C, P, nx;
  int k, j, i, im, ip, jm, jp;
  __device__ T at(int c, int kk, int jj, int ii) const { return x[c * C + kk * P + jj * nx + ii]; }
  // mixed difference f(+,+) - f(+,-) - f(-,+) + f(-,-) in the (x, y) plane
  __device__ T mxy(int c) const {
    return at(c, k, jp, ip) - at(c, k, jm, ip) - at(c, k, jp, im) + at(c, k, jm, im);
  }
  __device__ T mxz(int c) const {
    return at(c, k + 1, j, ip) - at(c, k - 1, j, ip) - at(c, k + 1, j, im) + at(c, k - 1, j, im);
  }
  __device__ T myz(int c) const {
    return at(c, k + 1, jp, i) - at(c, k - 1, jp, i) - at(c, k + 1, jm, i) + at(c, k - 1, jm, i);
  }
  __device__ T fx(int c) const { return at(c, k, j, ip) + at(c, k, j, im); }
  __device__ T fy(int c) const { return at(c, k, jp, i) + at(c, k, jm, i); }
  __device__ T fz(int c) const { return at(c, k + 1, j, i) + at(c, k - 1, j, i); }
  __device__ T offdiag(int c, T p, T q, T m4) const {
    if (c == 0) return p * fx(0) + q * (fy(0) + fz(0)) + m4 * (mxy(1) + mxz(2));
    if (c == 1) return p * fy(1) + q * (fx(1) + fz(1)) + m4 * (mxy(0) + myz(2));
    return p * fz(2) + q * (fx(2) + fy(2)) + m4 * (mxz(0) + myz(1));
  }
};

template <typename T>
__global__ __launch_bounds__(256) void k_colour_fine(T* __restrict__ x, const T* __restrict__ b,
                                                     int nx, int ny, int nz, ColourRange cr,
                                                     FineCoef<T> cf) {
  const int t = blockIdx.x * blockDim.x + threadIdx.x;
  if (t >= cr.total()) return;
  const int ii = t % cr.hx;
  const int rest = t / cr.hx;
  const int jj = rest % cr.hy;
  const int kk = rest / cr.hy;
  FineNbr<T> n;
  n.x = x;
  n.P = nx * ny;
  n.C = (nz + 1) * n.P;
  n.nx = nx;
  n.i = 2 * ii + cr.a;
  n.j = 2 * jj + cr.bb;
  n.k = cr.kfirst + 2 * kk;
  n.im = wrap_m(n.i, nx);
  n.ip = wrap_p(n.i, nx);
  n.jm = wrap_m(n.j, ny);
  n.jp = wrap_p(n.j, ny);
  const int o = n.k * n.P + n.j * nx + n.i;
  T v[3];
#pragma unroll
  for (int c = 0; c < 3; ++c) v[c] = (cf.h2 * b[c * n.C + o] + n.offdiag(c, cf.p, cf.q, cf.m4)) * cf.inv_diag;
#pragma unroll
  for (int c = 0; c < 3; ++c) x[c * n.C + o] = v[c];
}

template <typename T>
__global__ __launch_bounds__(256) void k_colour_gen(T* __restrict__ x, const T* __restrict__ b,
                                                    int nx, int ny, int nz, ColourRange cr,
                                                    const T* __restrict__ S,
                                                    const T* __restrict__ Dinv) {
  // blockIdx.y selects the plane; its stencil S[k][oz][y][x][c][d] and
  // inverse centre block are uniform over the workgroup and read with scalar
  // loads.  The three neighbour planes are visited in a loop that is not
  // unrolled; each visit issues its 27 loads together (the centre node's are
  // unused), so a thread waits for three rounds of memory latency.
  const int t = blockIdx.x * blockDim.x + threadIdx.x;
  const bool active = t < cr.hx * cr.hy;
  const int tt = active ? t : 0;
  const int ii = tt % cr.hx;
  const int jj = tt / cr.hx;
  const int k = cr.kfirst + 2 * static_cast<int>(blockIdx.y);
  const T* __restrict__ Sk = S + static_cast<size_t>(k) * 243;
  const T* __restrict__ Di = Dinv + static_cast<size_t>(k) * 9;
  const int i = 2 * ii + cr.a, j = 2 * jj + cr.bb;
  const int P = nx * ny, C = (nz + 1) * P;
  const int xs[3] = {wrap_m(i, nx), i, wrap_p(i, nx)};
  const int ys[3] = {wrap_m(j, ny), j, wrap_p(j, ny)};
  const int o = k * P + j * nx + i;
  T acc[3];
#pragma unroll
  for (int c = 0; c < 3; ++c) acc[c] = b[c * C + o];
  if (!active) return;
#pragma unroll 1
  for (int oz = 0; oz < 3; ++oz) {
    const int kk = k + oz - 1;
    T nb[9][3];
#pragma unroll
    for (int q = 0; q < 9; ++q) {
      const int off = kk * P + ys[q / 3] * nx + xs[q % 3];
#pragma unroll
      for (int c = 0; c < 3; ++c) nb[q][c] = x[c * C + off];
    }
#pragma unroll
    for (int q = 0; q < 9; ++q) {
      if (oz == 1 && q == 4) continue;  // centre block
      const T* B = Sk + (oz * 9 + q) * 9;
#pragma unroll
      for (int c = 0; c < 3; ++c)
        acc[c] -= B[c * 3] * nb[q][0] + B[c * 3 + 1] * nb[q][1] + B[c * 3 + 2] * nb[q][2];
    }
  }
#pragma unroll
  for (int c = 0; c < 3; ++c)
    x[c * C + o] = Di[c * 3] * acc[0] + Di[c * 3 + 1] * acc[1] + Di[c * 3 + 2] * acc[2];
}

// Block-level sum of one double per thread; result valid in thread 0.
__device__ __forceinline__ double block_sum(double v) {
  __shared__ double red[kReduceBlock / 64];
#pragma unroll
  for (int off = 32; off > 0; off >>= 1) v += __shfl_down(v, off, 64);
  const int lane = threadIdx.x & 63, wid = threadIdx.x >> 6;
  if (lane == 0) red[wid] = v;
  __syncthreads();
  double s = 0.0;
  if (threadIdx.x == 0) {
    for (int w = 0; w < kReduceBlock / 64; ++w) s += red[w];
  }
  return s;
}

template <typename Tin, typename Tout, bool ZERO_INT>
__global__ __launch_bounds__(kReduceBlock) void k_residual_fine(
    const Tin* __restrict__ x, const Tin* __restrict__ b, Tout* __restrict__ r, int nx, int ny,
    int nz, FineCoef<Tin> cf, Tin out_scale, double* __restrict__ partial) {
  const int t = blockIdx.x * blockDim.x + threadIdx.x;
  const int total = nx * ny * (nz - 1);
  double sq = 0.0;
  if (t < total) {
    FineNbr<Tin> n;
    n.x = x;
    n.P = nx * ny;
    n.C = (nz + 1) * n.P;
    n.nx = nx;
    n.i = t % nx;
    n.j = (t / nx) % ny;
    n.k = 1 + t / n.P;
    n.im = wrap_m(n.i, nx);
    n.ip = wrap_p(n.i, nx);
    n.jm = wrap_m(n.j, ny);
    n.jp = wrap_p(n.j, ny);
    const int o = n.k * n.P + n.j * nx + n.i;
#pragma unroll
    for (int c = 0; c < 3; ++c) {
      Tin off;
      if (ZERO_INT) {
        // only the wall planes contribute: nodes of plane k-1 or k+1 that are walls
        off = Tin(0);
        // only couplings into the wall planes remain: the face neighbour
        // across the wall and the mixed differences reaching it
#pragma unroll
        for (int side = 0; side < 2; ++side) {
          const bool touches = side == 0 ? (n.k == 1) : (n.k == nz - 1);
          if (!touches) continue;
          const int w = side == 0 ? 0 : nz;
          const Tin sg = side == 0 ? Tin(-1) : Tin(1);
          const Tin fz = n.at(c, w, n.j, n.i);
          Tin mix;
          if (c == 0)
            mix = sg * (n.at(2, w, n.j, n.ip) - n.at(2, w, n.j, n.im));
          else if (c == 1)
            mix = sg * (n.at(2, w, n.jp, n.i) - n.at(2, w, n.jm, n.i));
          else
            mix = sg * (n.at(0, w, n.j, n.ip) - n.at(0, w, n.j, n.im) + n.at(1, w, n.jp, n.i) -
                        n.at(1, w, n.jm, n.i));
          off += (c == 2 ? cf.p : cf.q) * fz + cf.m4 * mix;
        }
        const Tin bv = b ? b[c * n.C + o] : Tin(0);
        const Tin res = bv + off * cf.ih2;
        sq += static_cast<double>(res) * static_cast<double>(res);
        if (r) r[c * n.C + o] = static_cast<Tout>(res * out_scale);
      } else {
        off = n.offdiag(c, cf.p, cf.q, cf.m4);
        const Tin diag = Tin(2) * (cf.p + Tin(2) * cf.q);
        const Tin bv = b ? b[c * n.C + o] : Tin(0);
        const Tin res = bv - (diag * n.at(c, n.k, n.j, n.i) - off) * cf.ih2;
        sq += static_cast<double>(res) * static_cast<double>(res);
        if (r) r[c * n.C + o] = static_cast<Tout>(res * out_scale);
      }
    }
  }
  if (partial) {
    const double s = block_sum(sq);
    if (threadIdx.x == 0) partial[blockIdx.x] = s;
  }
}

// r = b - A x on a coarse level, one node per thread.  blockIdx.y selects the
// plane; its packed stencil (entries that vanish by symmetry left out, see
// packed_stencil.h) is uniform over the workgroup and read with scalar loads.
// All 81 neighbour loads are issued before the first is used.  ZERO_INT: x's
// interior is taken as zero, so only the couplings into the wall planes
// remain (a plane next to a wall).
template <typename T, bool ZERO_INT>
__global__ __launch_bounds__(kReduceBlock) void k_residual_gen(const T* __restrict__ x,
                                                               const T* __restrict__ b,
                                                               T* __restrict__ r, int nx, int ny,
                                                               int nz, const T* __restrict__ Pst,
                                                               double* __restrict__ partial) {
  const int t = blockIdx.x * blockDim.x + threadIdx.x;
  const int k = 1 + static_cast<int>(blockIdx.y);
  const T* __restrict__ Pk = Pst + static_cast<size_t>(k) * kPackedStencil;
  const bool active = t < nx * ny;
  const int tt = active ? t : 0;
  const unsigned P = static_cast<unsigned>(nx * ny), C = static_cast<unsigned>(nz + 1) * P;
  const int i = tt % nx, j = tt / nx;
  const unsigned xs[3] = {static_cast<unsigned>(wrap_m(i, nx)), static_cast<unsigned>(i),
                          static_cast<unsigned>(wrap_p(i, nx))};
  const unsigned ys[3] = {static_cast<unsigned>(wrap_m(j, ny)) * nx, static_cast<unsigned>(j) * nx,
                          static_cast<unsigned>(wrap_p(j, ny)) * nx};
  const unsigned o = k * P + j * nx + i;
  T acc[3];
#pragma unroll
  for (int c = 0; c < 3; ++c) acc[c] = b[c * C + o];
  // the three neighbour planes in a loop that is not unrolled, each visit
  // issuing its 27 loads together and running the body of that plane (see
  // k_colour_pair_gen)
#pragma unroll 1
  for (int oz = 0; oz < 3; ++oz) {
    const int kk = k + oz - 1;
    if (ZERO_INT && kk != 0 && kk != nz) continue;  // interior plane, taken as zero
    T nb[9][3];
#pragma unroll
    for (int q = 0; q < 9; ++q) {
      const unsigned off = kk * P + ys[q / 3] + xs[q % 3];
#pragma unroll
      for (int c = 0; c < 3; ++c) nb[q][c] = x[c * C + off];
    }
    auto apply = [&](auto OZ) {
      constexpr int ozc = decltype(OZ)::value;
      int n = packed_plane_start(ozc);
#pragma unroll
      for (int y = 0; y < 3; ++y)
#pragma unroll
        for (int q = 0; q < 3; ++q) {
          if (ozc == 1 && y == 1 && q == 1) {  // centre block: diagonal
#pragma unroll
            for (int c = 0; c < 3; ++c) acc[c] = fma(-Pk[kPackedCentre + c], nb[4][c], acc[c]);
            continue;
          }
#pragma unroll
          for (int c = 0; c < 3; ++c)
#pragma unroll
            for (int d = 0; d < 3; ++d) {
              if (!packed_used(ozc, y, q, c, d)) continue;
              acc[c] = fma(-Pk[n++], nb[y * 3 + q][d], acc[c]);
            }
        }
    };
    if (oz == 0)
      apply(std::integral_constant<int, 0>());
    else if (oz == 1)
      apply(std::integral_constant<int, 1>());
    else
      apply(std::integral_constant<int, 2>());
  }
  double sq = 0.0;
  if (active) {
#pragma unroll
    for (int c = 0; c < 3; ++c) {
      sq += static_cast<double>(acc[c]) * static_cast<double>(acc[c]);
      if (r) r[c * C + o] = acc[c];
    }
  }
  if (partial) {
    const double s = block_sum(sq);
    if (threadIdx.x == 0) partial[blockIdx.y * gridDim.x + blockIdx.x] = s;
  }
}

template <typename T>
struct Pair;
template <>
struct Pair<float> {
  using type = float2;
};
template <>
struct Pair<double> {
  using type = double2;
};

// Two colours that differ only in the x parity, (a, b) = (c, c ^ 1) with c
// first, in one launch on a coarse level.  Nodes of colour a couple to nodes
// of colour b only along x within their row and plane, so a thread owns the
// column pair (2p, 2p+1) of one row and plane: it updates its a-node from the
// old values, then its b-node once both x neighbours of colour a (its own and
// the one of pair p+1 or p-1) are new.  Where the column pairs of a row fill
// a power-of-two run of at most 64 lanes, that neighbour's new a-node comes by
// a lane shuffle; otherwise it comes through LDS.  Either way a workgroup
// holds whole rows, so the periodic neighbour in x is always present.  Every
// other term of the b-node uses values that neither update changes, and is
// summed while the a-node is.  Neighbour values of both nodes are read as
// pairs plus the two outer columns (four columns per row; the outer two, too,
// come by shuffles where the row fits that run of lanes), so a launch issues
// half the loads of two single-colour launches.
//
// A workgroup lies in one plane, so the plane's packed stencil (150 entries
// and the inverse centre block) is the same for all its lanes: it is read
// with scalar loads and enters the multiply-adds as a scalar operand.  The
// three neighbour planes differ in which entries are packed, so each has a
// body of its own in which the running index into the packed stencil is a
// constant; a body is entered through a branch on the plane, so that the
// scalar loads of one plane are not scheduled with those of the others.

// Where a thread's column pair and rows lie.
template <typename T>
struct PairSite {
  int W, rr, p, j, i0;
  bool active;
  unsigned P, C, il, ir, o;
  unsigned ys[3];
  // rb: the workgroup's block of rows_per_block rows of the colour
  __device__ PairSite(int tid, int nx, int ny, int nz, const ColourRange& cr, int rows_per_block,
                      int rb, int k) {
    W = nx / 2;  // column pairs per row
    rr = tid / W;
    p = tid - rr * W;
    const int jj = rb * rows_per_block + rr;
    active = rr < rows_per_block && jj < cr.hy;
    j = 2 * (active ? jj : 0) + cr.bb;
    i0 = 2 * p;
    P = static_cast<unsigned>(nx * ny);
    C = static_cast<unsigned>(nz + 1) * P;
    il = i0 == 0 ? nx - 1 : i0 - 1;  // column i0-1
    ir = i0 + 2 == nx ? 0 : i0 + 2;  // column i0+2
    ys[0] = static_cast<unsigned>(wrap_m(j, ny)) * nx;
    ys[1] = static_cast<unsigned>(j) * nx;
    ys[2] = static_cast<unsigned>(wrap_p(j, ny)) * nx;
    o = k * P + j * nx + i0;
  }
};

// The four-wide window of the rows j-1, j, j+1 of plane kk: w[y][0] = column
// i0-1, [1] = i0, [2] = i0+1, [3] = i0+2; the node at column i0 + s uses
// columns s .. s+2.  SHFL: the pairs of a row lie in W consecutive lanes of
// one wavefront (W a power of two dividing 64), so the outer columns i0-1
// and i0+2 are the neighbouring lanes' pair values (the periodic wrap is a
// rotation within the row's lanes) and only the pairs are loaded: a third of
// the load instructions.
template <typename T, bool SHFL>
__device__ __forceinline__ void pair_window(const T* __restrict__ x, const PairSite<T>& st,
                                            unsigned kk, T w[3][4][3]) {
  using V = typename Pair<T>::type;
  V v[3][3];
#pragma unroll
  for (int y = 0; y < 3; ++y) {
    const unsigned row = kk * st.P + st.ys[y];
#pragma unroll
    for (int c = 0; c < 3; ++c) {
      v[y][c] = *reinterpret_cast<const V*>(x + (c * st.C + row + st.i0));
      if (!SHFL) {
        w[y][0][c] = x[c * st.C + row + st.il];
        w[y][3][c] = x[c * st.C + row + st.ir];
      }
    }
  }
  int lm = 0, lp = 0;  // lanes of the pairs p-1 and p+1 in the row
  if (SHFL) {
    const int lane = static_cast<int>(__lane_id());
    const int base = lane & ~(st.W - 1);
    lm = base + ((st.p + st.W - 1) & (st.W - 1));
    lp = base + ((st.p + 1) & (st.W - 1));
  }
#pragma unroll
  for (int y = 0; y < 3; ++y)
#pragma unroll
    for (int c = 0; c < 3; ++c) {
      w[y][1][c] = v[y][c].x;
      w[y][2][c] = v[y][c].y;
      if (SHFL) {
        w[y][0][c] = __shfl(v[y][c].y, lm);
        w[y][3][c] = __shfl(v[y][c].x, lp);
      }
    }
}

// Terms of neighbour plane OZ (0, 1, 2 for k-1, k, k+1) subtracted from the
// a-node sum and the b-node sum; the b-node's blocks (1,1,0) and (1,1,2) wait
// for the new a values (pair_side), the centre block is the inverse's.
template <typename T, int OZ, int SA, int SB>
__device__ __forceinline__ void pair_plane(const T* __restrict__ Pk, const T w[3][4][3],
                                           T acca[3], T accb[3]) {
  int n = packed_plane_start(OZ);
#pragma unroll
  for (int y = 0; y < 3; ++y)
#pragma unroll
    for (int q = 0; q < 3; ++q) {
      if (OZ == 1 && y == 1 && q == 1) continue;  // centre block
      const bool later = OZ == 1 && y == 1;
#pragma unroll
      for (int c = 0; c < 3; ++c)
#pragma unroll
        for (int d = 0; d < 3; ++d) {
          if (!packed_used(OZ, y, q, c, d)) continue;
          const T co = Pk[n++];
          acca[c] = fma(-co, w[y][q + SA][d], acca[c]);
          if (!later) accb[c] = fma(-co, w[y][q + SB][d], accb[c]);
        }
    }
}

template <typename T, int SA, int SB>
__device__ __forceinline__ void pair_plane_rt(int oz, const T* __restrict__ Pk, const T w[3][4][3],
                                              T acca[3], T accb[3]) {
  if (oz == 0)
    pair_plane<T, 0, SA, SB>(Pk, w, acca, accb);
  else if (oz == 1)
    pair_plane<T, 1, SA, SB>(Pk, w, acca, accb);
  else
    pair_plane<T, 2, SA, SB>(Pk, w, acca, accb);
}

// D^-1 times a sum
template <typename T>
__device__ __forceinline__ void apply_inv(const T* __restrict__ Di, const T acc[3], T out[3]) {
#pragma unroll
  for (int c = 0; c < 3; ++c) out[c] = Di[c * 3] * acc[0] + Di[c * 3 + 1] * acc[1] + Di[c * 3 + 2] * acc[2];
}

// The b-node's x neighbours of colour a (the own a-node na and that of the
// pair on the side away from it, by a shuffle or from LDS xa), its last terms,
// its new value, and the store of the pair.
template <typename T, int XF, bool SHFL>
__device__ __forceinline__ void pair_finish(T* __restrict__ x, const PairSite<T>& st,
                                            const T* __restrict__ Pk, const T (*xa)[256], int tid,
                                            const T na[3], T accb[3]) {
  using V = typename Pair<T>::type;
  const int pn = XF ? (st.p == 0 ? st.W - 1 : st.p - 1) : (st.p == st.W - 1 ? 0 : st.p + 1);
  const int tn = st.active ? st.rr * st.W + pn : tid;
  // SHFL: the neighbour pair is the lane pn of the row's run of lanes, and
  // its new a-node comes by a shuffle (xa is not used)
  const int ln = SHFL ? (static_cast<int>(__lane_id()) & ~(st.W - 1)) + pn : 0;
  T side[2][3];
#pragma unroll
  for (int c = 0; c < 3; ++c) {
    side[XF][c] = na[c];  // XF = 0: left neighbour (i0) is own; XF = 1: right (i0+1)
    side[1 - XF][c] = SHFL ? __shfl(na[c], ln) : xa[c][tn];
  }
#pragma unroll
  for (int s2 = 0; s2 < 2; ++s2) {
    int m = packed_block_start(1, 1, 2 * s2);
#pragma unroll
    for (int c = 0; c < 3; ++c)
#pragma unroll
      for (int d = 0; d < 3; ++d) {
        if (!packed_used(1, 1, 2 * s2, c, d)) continue;
        accb[c] = fma(-Pk[m++], side[s2][d], accb[c]);
      }
  }
  if (!st.active) return;
  T nb[3];
  apply_inv<T>(Pk + kPackedInv, accb, nb);
#pragma unroll
  for (int c = 0; c < 3; ++c) {
    V v;
    v.x = XF ? nb[c] : na[c];
    v.y = XF ? na[c] : nb[c];
    *reinterpret_cast<V*>(x + c * st.C + st.o) = v;
  }
}

// One thread per column pair: the three neighbour planes in a loop that is
// not unrolled, each visit issuing its loads together (128^3 and larger).
// SHFL: the outer window columns and the neighbour pair's new a-node come by
// lane shuffles, with no LDS exchange and no barrier.
// The grid is one-dimensional, gx row blocks times the colour's planes, in
// an XCD-aware order: workgroups are dealt round-robin to the 8 XCDs, and XCD
// x takes the contiguous range [x per_xcd, (x+1) per_xcd) of (plane, row
// block) pairs, so that the neighbour rows and planes a workgroup reads are
// mostly fetched into the same L2 by the workgroups next to it.
template <typename T, int XF, bool SHFL>
__global__ __launch_bounds__(256) void k_colour_pair_gen(T* __restrict__ x, const T* __restrict__ b,
                                                         int nx, int ny, int nz, ColourRange cr,
                                                         int rows_per_block, int gx, int per_xcd,
                                                         const T* __restrict__ Pst) {
  using V = typename Pair<T>::type;
  __shared__ T xa[3][256];
  const int wg = blockIdx.x;
  const int L = (wg & 7) * per_xcd + (wg >> 3);
  if (L >= gx * cr.nk) return;  // the whole workgroup, before any barrier
  const int tid = threadIdx.x;
  const int k = cr.kfirst + 2 * (L / gx);
  const T* __restrict__ Pk = Pst + static_cast<size_t>(k) * kPackedStencil;  // uniform
  const PairSite<T> st(tid, nx, ny, nz, cr, rows_per_block, L % gx, k);
  T acca[3], accb[3];
  {
    V bv[3];
#pragma unroll
    for (int c = 0; c < 3; ++c) bv[c] = *reinterpret_cast<const V*>(b + c * st.C + st.o);
#pragma unroll
    for (int c = 0; c < 3; ++c) {
      acca[c] = XF ? bv[c].y : bv[c].x;
      accb[c] = XF ? bv[c].x : bv[c].y;
    }
  }
#pragma unroll 1
  for (int oz = 0; oz < 3; ++oz) {
    T w[3][4][3];
    pair_window<T, SHFL>(x, st, k + oz - 1, w);
    pair_plane_rt<T, XF, 1 - XF>(oz, Pk, w, acca, accb);
  }
  T na[3];
  apply_inv<T>(Pk + kPackedInv, acca, na);
  if (!SHFL) {
#pragma unroll
    for (int c = 0; c < 3; ++c) xa[c][tid] = na[c];
    __syncthreads();
  }
  pair_finish<T, XF, SHFL>(x, st, Pk, xa, tid, na, accb);
}

// The same two colours with three threads per column pair, one per
// neighbour plane (threadIdx.y), on the small levels (64^3 and below), where
// a launch is a few waves and each round of memory latency shows: every
// neighbour load of the pair is issued at once, across the three threads.
// The partial sums of planes k-1 and k+1 meet the middle thread's in LDS;
// the middle thread finishes the pair as above.
template <typename T, int XF, bool SHFL>
__global__ __launch_bounds__(384) void k_colour_pair_split(T* __restrict__ x,
                                                           const T* __restrict__ b, int nx,
                                                           int ny, int nz, ColourRange cr,
                                                           int rows_per_block,
                                                           const T* __restrict__ Pst) {
  using V = typename Pair<T>::type;
  __shared__ T xa[3][256];
  __shared__ T part[2][2][3][128];  // [plane k-1, k+1][a, b][component][pair]
  const int tid = threadIdx.x, oz = threadIdx.y;
  const int k = cr.kfirst + 2 * static_cast<int>(blockIdx.y);
  const T* __restrict__ Pk = Pst + static_cast<size_t>(k) * kPackedStencil;  // uniform
  const PairSite<T> st(tid, nx, ny, nz, cr, rows_per_block, blockIdx.x, k);
  T acca[3] = {T(0), T(0), T(0)}, accb[3] = {T(0), T(0), T(0)};
  V bv[3];
  if (oz == 1) {
#pragma unroll
    for (int c = 0; c < 3; ++c) bv[c] = *reinterpret_cast<const V*>(b + c * st.C + st.o);
  }
  {
    T w[3][4][3];
    pair_window<T, SHFL>(x, st, k + oz - 1, w);
    pair_plane_rt<T, XF, 1 - XF>(oz, Pk, w, acca, accb);
  }
  if (oz != 1) {
#pragma unroll
    for (int c = 0; c < 3; ++c) {
      part[oz >> 1][0][c][tid] = acca[c];
      part[oz >> 1][1][c][tid] = accb[c];
    }
  }
  __syncthreads();
  T na[3];
  if (oz == 1) {
#pragma unroll
    for (int c = 0; c < 3; ++c) {
      const T ba = XF ? bv[c].y : bv[c].x, bb = XF ? bv[c].x : bv[c].y;
      acca[c] = ba + part[0][0][c][tid] + acca[c] + part[1][0][c][tid];
      accb[c] = bb + part[0][1][c][tid] + accb[c] + part[1][1][c][tid];
    }
    apply_inv<T>(Pk + kPackedInv, acca, na);
    if (!SHFL) {
#pragma unroll
      for (int c = 0; c < 3; ++c) xa[c][tid] = na[c];
    }
  }
  if (!SHFL) __syncthreads();
  if (oz == 1) pair_finish<T, XF, SHFL>(x, st, Pk, xa, tid, na, accb);
}

// Coarse residual r = b - A x (V-cycle form: no norm) for the column pair
// (2p, 2p+1) of one row and plane per thread.  The four-column window of each
// neighbour row serves both nodes, so a launch issues half the neighbour
// loads of one thread per node; each node's terms are summed in the order of
// k_residual_gen, so the two kernels give the same values.
template <typename T, bool SHFL>
__global__ __launch_bounds__(256) void k_residual_pair_gen(const T* __restrict__ x,
                                                           const T* __restrict__ b,
                                                           T* __restrict__ r, int nx, int ny,
                                                           int nz, const T* __restrict__ Pst) {
  using V = typename Pair<T>::type;
  const int W = nx / 2;
  const int t = blockIdx.x * blockDim.x + threadIdx.x;
  const int k = 1 + static_cast<int>(blockIdx.y);
  const T* __restrict__ Pk = Pst + static_cast<size_t>(k) * kPackedStencil;  // uniform
  const bool active = t < W * ny;
  const int tt = active ? t : 0;
  const int p = tt % W, j = tt / W;
  const int i0 = 2 * p;
  const unsigned P = static_cast<unsigned>(nx * ny), C = static_cast<unsigned>(nz + 1) * P;
  const unsigned il = i0 == 0 ? nx - 1 : i0 - 1;  // column i0-1
  const unsigned ir = i0 + 2 == nx ? 0 : i0 + 2;  // column i0+2
  const unsigned ys[3] = {static_cast<unsigned>(wrap_m(j, ny)), static_cast<unsigned>(j),
                          static_cast<unsigned>(wrap_p(j, ny))};
  const unsigned o = k * P + j * nx + i0;
  T acc0[3], acc1[3];
#pragma unroll
  for (int c = 0; c < 3; ++c) {
    const V bv = *reinterpret_cast<const V*>(b + c * C + o);
    acc0[c] = bv.x;
    acc1[c] = bv.y;
  }
#pragma unroll 1
  for (int oz = 0; oz < 3; ++oz) {
    const unsigned kk = k + oz - 1;
    T w[3][4][3];  // rows j-1, j, j+1; columns i0-1 .. i0+2
    V v[3][3];
#pragma unroll
    for (int y = 0; y < 3; ++y) {
      const unsigned row = kk * P + ys[y] * nx;
#pragma unroll
      for (int c = 0; c < 3; ++c) {
        v[y][c] = *reinterpret_cast<const V*>(x + (c * C + row + i0));
        if (!SHFL) {
          w[y][0][c] = x[c * C + row + il];
          w[y][3][c] = x[c * C + row + ir];
        }
      }
    }
    // SHFL: a row's W pairs fill W consecutive lanes (W a power of two
    // dividing 64); the outer columns come from the neighbouring lanes
    const int lane = static_cast<int>(__lane_id()), base = lane & ~(W - 1);
    const int lm = base + ((p + W - 1) & (W - 1)), lp = base + ((p + 1) & (W - 1));
#pragma unroll
    for (int y = 0; y < 3; ++y)
#pragma unroll
      for (int c = 0; c < 3; ++c) {
        w[y][1][c] = v[y][c].x;
        w[y][2][c] = v[y][c].y;
        if (SHFL) {
          w[y][0][c] = __shfl(v[y][c].y, lm);
          w[y][3][c] = __shfl(v[y][c].x, lp);
        }
      }
    // the planes differ in which entries are packed: one body per plane
    auto apply = [&](auto OZ) {
      constexpr int ozc = decltype(OZ)::value;
      int n = packed_plane_start(ozc);
#pragma unroll
      for (int y = 0; y < 3; ++y)
#pragma unroll
        for (int q = 0; q < 3; ++q) {
          if (ozc == 1 && y == 1 && q == 1) {  // centre block: diagonal
#pragma unroll
            for (int c = 0; c < 3; ++c) {
              acc0[c] = fma(-Pk[kPackedCentre + c], w[1][1][c], acc0[c]);
              acc1[c] = fma(-Pk[kPackedCentre + c], w[1][2][c], acc1[c]);
            }
            continue;
          }
#pragma unroll
          for (int c = 0; c < 3; ++c)
#pragma unroll
            for (int d = 0; d < 3; ++d) {
              if (!packed_used(ozc, y, q, c, d)) continue;
              const T co = Pk[n++];
              acc0[c] = fma(-co, w[y][q][d], acc0[c]);
              acc1[c] = fma(-co, w[y][q + 1][d], acc1[c]);
            }
        }
    };
    if (oz == 0)
      apply(std::integral_constant<int, 0>());
    else if (oz == 1)
      apply(std::integral_constant<int, 1>());
    else
      apply(std::integral_constant<int, 2>());
  }
  if (!active) return;
#pragma unroll
  for (int c = 0; c < 3; ++c) {
    V v;
    v.x = acc0[c];
    v.y = acc1[c];
    *reinterpret_cast<V*>(r + c * C + o) = v;
  }
}

// b_c(I) = sum over the 27 fine nodes around 2I of w * r(f), w = prod (1 or 1/2).
// One thread per coarse node; per fine row it loads the pair (2I, 2I+1) as one
// two-wide access and 2I-1 on its own, or (SHFL: the nxc coarse nodes of a row
// are a power-of-two run of at most 64 lanes) takes 2I-1 from the lane of
// node I-1 once all loads of the component are issued.  Rows of lanes are
// whole (the total is a multiple of nxc), so lanes that leave early never
// serve as a shuffle source.
template <typename T, bool SHFL>
__global__ __launch_bounds__(256) void k_restrict(const T* __restrict__ r, T* __restrict__ bc,
                                                  T* __restrict__ xc, int nxf, int nyf, int nzf) {
  using V = typename Pair<T>::type;
  const int nxc = nxf / 2, nyc = nyf / 2, nzc = nzf / 2;
  const int t = blockIdx.x * blockDim.x + threadIdx.x;
  const int total = nxc * nyc * (nzc - 1);
  if (total <= 0) return;
  if (t >= total) return;
  const int I = t % nxc, J = (t / nxc) % nyc, K = 1 + t / (nxc * nyc);
  const int il = I == 0 ? nxf - 1 : 2 * I - 1;
  const int Pf = nxf * nyf, Cf = (nzf + 1) * Pf;
  const int Pc = nxc * nyc, Cc = (nzc + 1) * Pc;
  const int ys[3] = {wrap_m(2 * J, nyf), 2 * J, 2 * J + 1};
  const T w[3] = {T(0.5), T(1), T(0.5)};
  // the 54 loads of a component are all issued before any value is used, so
  // the thread waits for one round of memory latency per component
#pragma unroll
  for (int c = 0; c < 3; ++c) {
    V v[3][3];
    T left[3][3];
#pragma unroll
    for (int dz = 0; dz < 3; ++dz)
#pragma unroll
      for (int dy = 0; dy < 3; ++dy) {
        const T* row = r + c * Cf + (2 * K + dz - 1) * Pf + ys[dy] * nxf;
        v[dz][dy] = *reinterpret_cast<const V*>(row + 2 * I);
        if (!SHFL) left[dz][dy] = row[il];
      }
    if (SHFL) {
      const int lane = static_cast<int>(__lane_id());
      const int src = (lane & ~(nxc - 1)) + ((I + nxc - 1) & (nxc - 1));
#pragma unroll
      for (int dz = 0; dz < 3; ++dz)
#pragma unroll
        for (int dy = 0; dy < 3; ++dy) left[dz][dy] = __shfl(v[dz][dy].y, src);
    }
    T acc = T(0);
#pragma unroll
    for (int dz = 0; dz < 3; ++dz) {
      T az = T(0);
#pragma unroll
      for (int dy = 0; dy < 3; ++dy) {
        const T ax = T(0.5) * left[dz][dy] + v[dz][dy].x + T(0.5) * v[dz][dy].y;
        az += w[dy] * ax;
      }
      acc += w[dz] * az;
    }
    {
      bc[c * Cc + K * Pc + J * nxc + I] = acc;
      if (xc) xc[c * Cc + K * Pc + J * nxc + I] = T(0);
    }
  }
}

// x(f) += sum_J w(f - 2J) e(J) over the (up to 8) coarse nodes around f.  One
// thread per pair of fine columns (2I, 2I+1) of a row, which use the coarse
// columns I and I+1, marching up a segment of coarse planes: for each coarse
// plane it combines the (up to) four coarse values of the pair's x-y
// neighbourhood once, then adds plane K alone to fine plane 2K and the mean
// of planes K and K+1 to fine plane 2K+1.  Each coarse value is loaded by the
// threads of the rows next to it, not by every fine node around it; the fine
// pair is read and written as one two-wide access.  SHFL: the nxc pairs of a
// fine row are a power-of-two run of at most 64 lanes, and the values of
// coarse column I+1 come from the lane of pair I+1 (whole rows of lanes leave
// together).
template <typename T, bool SHFL>
__global__ __launch_bounds__(256) void k_prolong_add(T* __restrict__ x, const T* __restrict__ ec,
                                                     int nxf, int nyf, int nzf, int kseg) {
  using V = typename Pair<T>::type;
  const int nxc = nxf / 2, nyc = nyf / 2, nzc = nzf / 2;
  const int t = blockIdx.x * blockDim.x + threadIdx.x;
  const int per = nxc * nyf;  // threads per segment
  const int nseg = (nzc + kseg - 1) / kseg;
  if (t >= per * nseg) return;
  const int i0 = t % nxc, j = (t / nxc) % nyf, sg = t / per;
  const int Ks = sg * kseg, Ke = min(Ks + kseg, nzc);  // coarse planes K: fine 2K, 2K+1
  const int Pf = nxf * nyf, Cf = (nzf + 1) * Pf;
  const int Pc = nxc * nyc, Cc = (nzc + 1) * Pc;
  const int i1 = i0 + 1 == nxc ? 0 : i0 + 1;
  const int j0 = j >> 1;
  const int j1 = (j & 1) ? (j0 + 1 == nyc ? 0 : j0 + 1) : j0;
  const bool oy = j & 1;
  const T wy = oy ? T(0.5) : T(1), wz = T(0.5);
  // x-y combination of coarse plane K for the even and the odd fine column
  // (the row j1 is loaded on even fine rows too, where it is j0, so that all
  // twelve loads are issued before any is used)
  const int src1 = SHFL ? (static_cast<int>(__lane_id()) & ~(nxc - 1)) + ((i0 + 1) & (nxc - 1)) : 0;
  auto coarse = [&](int K, T pe[3], T po[3]) {
    T a0[3], a1[3], b0[3], b1[3];
#pragma unroll
    for (int c = 0; c < 3; ++c) {
      const T* p0 = ec + c * Cc + K * Pc + j0 * nxc;
      const T* p1 = ec + c * Cc + K * Pc + j1 * nxc;
      a0[c] = p0[i0];
      b0[c] = p1[i0];
      if (!SHFL) {
        a1[c] = p0[i1];
        b1[c] = p1[i1];
      }
    }
    if (SHFL) {
#pragma unroll
      for (int c = 0; c < 3; ++c) {
        a1[c] = __shfl(a0[c], src1);
        b1[c] = __shfl(b0[c], src1);
      }
    }
#pragma unroll
    for (int c = 0; c < 3; ++c) {
      if (oy) {
        pe[c] = wy * (a0[c] + b0[c]);
        po[c] = wy * (T(0.5) * (a0[c] + a1[c]) + T(0.5) * (b0[c] + b1[c]));
      } else {
        pe[c] = a0[c];
        po[c] = T(0.5) * (a0[c] + a1[c]);
      }
    }
  };
  T pe0[3], po0[3], pe1[3], po1[3];
  coarse(Ks, pe0, po0);
  const size_t orow = static_cast<size_t>(j) * nxf + 2 * i0;
  for (int K = Ks; K < Ke; ++K) {
    coarse(K + 1, pe1, po1);  // K + 1 <= nzc (the top coarse wall is zero)
#pragma unroll
    for (int c = 0; c < 3; ++c) {
      if (K >= 1) {  // fine plane 2K (plane 0 is the wall)
        T* px = x + c * Cf + static_cast<size_t>(2 * K) * Pf + orow;
        V v = NT2<T>::template load<V>(px);
        v.x += pe0[c];
        v.y += po0[c];
        NT2<T>::store(px, v);
      }
      T* qx = x + c * Cf + static_cast<size_t>(2 * K + 1) * Pf + orow;
      V v = NT2<T>::template load<V>(qx);
      v.x += wz * (pe0[c] + pe1[c]);
      v.y += wz * (po0[c] + po1[c]);
      NT2<T>::store(qx, v);
    }
#pragma unroll
    for (int c = 0; c < 3; ++c) {
      pe0[c] = pe1[c];
      po0[c] = po1[c];
    }
  }
}

__global__ __launch_bounds__(1024) void k_reduce_sum(const double* __restrict__ partial, int n,
                                                     double* __restrict__ out,
                                                     double* __restrict__ out_host) {
  __shared__ double red[16];
  double s = 0.0;
  for (int q = threadIdx.x; q < n; q += blockDim.x) s += partial[q];
#pragma unroll
  for (int off = 32; off > 0; off >>= 1) s += __shfl_down(s, off, 64);
  const int lane = threadIdx.x & 63, wid = threadIdx.x >> 6;
  if (lane == 0) red[wid] = s;
  __syncthreads();
  if (threadIdx.x == 0) {
    double t = 0.0;
    for (int w = 0; w < (int)(blockDim.x >> 6); ++w) t += red[w];
    out[0] = t;
    if (out_host) out_host[0] = t;
  }
}

template <typename T>
__global__ void k_fill(T* __restrict__ x, size_t n, T v) {
  size_t t = blockIdx.x * static_cast<size_t>(blockDim.x) + threadIdx.x;
  const size_t stride = static_cast<size_t>(gridDim.x) * blockDim.x;
  for (; t < n; t += stride) x[t] = v;
}

// The coarsest solve in one launch: x_interior = A^-1 b_interior with the
// interior unknowns in the order (component, plane, row, column); each lane
// reads its b entries straight from the node vector (in double) and the row's
// result goes straight to x, so no gathered copy of b is made.
template <typename T>
__global__ __launch_bounds__(256) void k_coarse_apply(const double* __restrict__ A,
                                                      const T* __restrict__ b, T* __restrict__ x,
                                                      int n, int P, int nz) {
  const int row = blockIdx.x * 4 + (threadIdx.x >> 6);
  const int lane = threadIdx.x & 63;
  if (row >= n) return;
  const int per = P * (nz - 1);              // interior unknowns per component
  const size_t C = static_cast<size_t>(nz + 1) * P;
  auto at = [&](int q) -> size_t {            // node-vector index of unknown q
    const int c = (q >= per) + (q >= 2 * per);
    return c * C + P + (q - c * per);
  };
  const double* a = A + static_cast<size_t>(row) * n;
  double s0 = 0.0, s1 = 0.0, s2 = 0.0, s3 = 0.0;
  int q = lane;
  for (; q + 192 < n; q += 256) {
    const double a0 = a[q], a1 = a[q + 64], a2 = a[q + 128], a3 = a[q + 192];
    const double v0 = static_cast<double>(b[at(q)]), v1 = static_cast<double>(b[at(q + 64)]);
    const double v2 = static_cast<double>(b[at(q + 128)]), v3 = static_cast<double>(b[at(q + 192)]);
    s0 += a0 * v0;
    s1 += a1 * v1;
    s2 += a2 * v2;
    s3 += a3 * v3;
  }
  for (; q < n; q += 64) s0 += a[q] * static_cast<double>(b[at(q)]);
  double s = (s0 + s1) + (s2 + s3);
#pragma unroll
  for (int off = 32; off > 0; off >>= 1) s += __shfl_down(s, off, 64);
  if (lane == 0) x[at(row)] = static_cast<T>(s);
}

inline int blocks_for(long long n, int bs) { return static_cast<int>((n + bs - 1) / bs); }

}  // namespace

template <typename T>
void launch_colour_fine(T* x, const T* b, Dims d, int colour, const FineCoef<T>& c, hipStream_t s) {
  const ColourRange cr = colour_range(d, colour);
  if (cr.total() <= 0) return;
  hipLaunchKernelGGL(k_colour_fine<T>, dim3(blocks_for(cr.total(), 256)), dim3(256), 0, s, x, b,
                     d.nx, d.ny, d.nz, cr, c);
}

template <typename T>
void launch_colour_gen(T* x, const T* b, Dims d, int colour, const T* S, const T* Dinv,
                       hipStream_t s) {
  const ColourRange cr = colour_range(d, colour);
  if (cr.total() <= 0) return;
  hipLaunchKernelGGL(k_colour_gen<T>, dim3(blocks_for(cr.hx * cr.hy, 256), cr.nk), dim3(256), 0, s, x, b,
                     d.nx, d.ny, d.nz, cr, S, Dinv);
}

bool pair_rows_in_lanes(Dims d) {
  const int W = d.nx / 2;
  return d.nx % 2 == 0 && W >= 1 && W <= 64 && (W & (W - 1)) == 0;
}

bool colour_pair_supported(Dims d) { return d.nx % 2 == 0 && d.nx >= 2 && d.nx <= 512; }

template <typename T>
void launch_colour_pair_gen(T* x, const T* b, Dims d, int colour, const T* Pst, hipStream_t s) {
  // colour is the one updated first; its partner is colour ^ 1
  const ColourRange cr = colour_range(d, colour);
  if (cr.total() <= 0) return;
  const int W = d.nx / 2;
  // whole rows in workgroups of about 128 column pairs: more, smaller
  // workgroups than 256-pair ones (measured: 5.3 against 6.3 us at 64^3, same
  // at 128^3)
  const int rpb = std::max(1, std::min(cr.hy, 128 / W));
  const dim3 grid(blocks_for(cr.hy, rpb), cr.nk);
  // outer window columns by lane shuffles where a row's pairs fill a power-of-two
  // run of lanes of one wavefront
  const bool shfl = pair_rows_in_lanes(d);
#define QS_PAIR(KERNEL, XF, SH, G, B, ...)                                                   \
  hipLaunchKernelGGL((KERNEL<T, XF, SH>), G, B, 0, s, x, b, d.nx, d.ny, d.nz, cr, rpb, __VA_ARGS__)
  if (d.nx <= 64) {  // small levels: three threads per pair
    const dim3 block(rpb * W, 3);
    if (cr.a && shfl)
      QS_PAIR(k_colour_pair_split, 1, true, grid, block, Pst);
    else if (cr.a)
      QS_PAIR(k_colour_pair_split, 1, false, grid, block, Pst);
    else if (shfl)
      QS_PAIR(k_colour_pair_split, 0, true, grid, block, Pst);
    else
      QS_PAIR(k_colour_pair_split, 0, false, grid, block, Pst);
    return;
  }
  const int threads = (rpb * W + 63) / 64 * 64;
  const int gx = static_cast<int>(grid.x), per_xcd = (gx * cr.nk + 7) / 8;
  const dim3 g1(8 * per_xcd), b1(threads);
  if (cr.a && shfl)
    QS_PAIR(k_colour_pair_gen, 1, true, g1, b1, gx, per_xcd, Pst);
  else if (cr.a)
    QS_PAIR(k_colour_pair_gen, 1, false, g1, b1, gx, per_xcd, Pst);
  else if (shfl)
    QS_PAIR(k_colour_pair_gen, 0, true, g1, b1, gx, per_xcd, Pst);
  else
    QS_PAIR(k_colour_pair_gen, 0, false, g1, b1, gx, per_xcd, Pst);
#undef QS_PAIR
}

template <typename T>
void launch_residual_pair_gen(const T* x, const T* b, T* r, Dims d, const T* Pst, hipStream_t s) {
  const dim3 grid(blocks_for(static_cast<long long>(d.nx / 2) * d.ny, 256), d.nz - 1);
  if (d.nz - 1 <= 0) return;
  if (pair_rows_in_lanes(d))
    hipLaunchKernelGGL((k_residual_pair_gen<T, true>), grid, dim3(256), 0, s, x, b, r, d.nx, d.ny,
                       d.nz, Pst);
  else
    hipLaunchKernelGGL((k_residual_pair_gen<T, false>), grid, dim3(256), 0, s, x, b, r, d.nx, d.ny,
                       d.nz, Pst);
}

int residual_blocks(Dims d) {
  const int flat = blocks_for(static_cast<long long>(d.nx) * d.ny * (d.nz - 1), kReduceBlock);
  const int planes = blocks_for(static_cast<long long>(d.nx) * d.ny, kReduceBlock) * (d.nz - 1);
  const int zm = resid_zmarch_blocks(d);
  return std::max(flat, std::max(planes, zm));
}

template <typename Tin, typename Tout>
int launch_residual_fine(const Tin* x, const Tin* b, Tout* r, Dims d, const FineCoef<double>& c,
                         double out_scale, bool zero_interior, double* partial, hipStream_t s) {
  FineCoef<Tin> cf;
  cf.h2 = static_cast<Tin>(c.h2);
  cf.p = static_cast<Tin>(c.p);
  cf.q = static_cast<Tin>(c.q);
  cf.m4 = static_cast<Tin>(c.m4);
  cf.inv_diag = static_cast<Tin>(c.inv_diag);
  cf.ih2 = static_cast<Tin>(c.ih2);
  const int nb = residual_blocks(d);
  if (zero_interior)
    hipLaunchKernelGGL((k_residual_fine<Tin, Tout, true>), dim3(nb), dim3(kReduceBlock), 0, s, x, b,
                       r, d.nx, d.ny, d.nz, cf, static_cast<Tin>(out_scale), partial);
  else
    hipLaunchKernelGGL((k_residual_fine<Tin, Tout, false>), dim3(nb), dim3(kReduceBlock), 0, s, x,
                       b, r, d.nx, d.ny, d.nz, cf, static_cast<Tin>(out_scale), partial);
  return nb;
}

template <typename T>
int launch_residual_gen(const T* x, const T* b, T* r, Dims d, const T* Pst, bool zero_interior,
                        double* partial, hipStream_t s) {
  const dim3 grid(blocks_for(static_cast<long long>(d.nx) * d.ny, kReduceBlock), d.nz - 1);
  if (zero_interior)
    hipLaunchKernelGGL((k_residual_gen<T, true>), grid, dim3(kReduceBlock), 0, s, x, b, r, d.nx,
                       d.ny, d.nz, Pst, partial);
  else
    hipLaunchKernelGGL((k_residual_gen<T, false>), grid, dim3(kReduceBlock), 0, s, x, b, r, d.nx,
                       d.ny, d.nz, Pst, partial);
  return static_cast<int>(grid.x * grid.y);
}

template <typename T>
void launch_restrict(const T* r, T* bc, T* xc, Dims f, hipStream_t s) {
  const long long total = static_cast<long long>(f.nx / 2) * (f.ny / 2) * (f.nz / 2 - 1);
  if (total <= 0) return;
  if (pair_rows_in_lanes(f))
    hipLaunchKernelGGL((k_restrict<T, true>), dim3(blocks_for(total, 256)), dim3(256), 0, s, r, bc, xc,
                       f.nx, f.ny, f.nz);
  else
    hipLaunchKernelGGL((k_restrict<T, false>), dim3(blocks_for(total, 256)), dim3(256), 0, s, r, bc,
                       xc, f.nx, f.ny, f.nz);
}

template <typename T>
void launch_prolong_add(T* x, const T* ec, Dims f, hipStream_t s) {
  // march just far enough that the launch keeps about 512K threads: a long
  // march reloads fewer coarse values, a short one exposes less latency per
  // thread (small levels)
  const int nzc = f.nz / 2;
  if (nzc <= 0) return;
  const long long per = static_cast<long long>(f.nx / 2) * f.ny;
  const long long want = std::max<long long>(1, (512 * 1024 + per - 1) / per);
  const int kseg = static_cast<int>(std::max<long long>(1, (nzc + want - 1) / want));
  const long long total = per * ((nzc + kseg - 1) / kseg);
  if (total <= 0) return;
  if (pair_rows_in_lanes(f))
    hipLaunchKernelGGL((k_prolong_add<T, true>), dim3(blocks_for(total, 256)), dim3(256), 0, s, x, ec,
                       f.nx, f.ny, f.nz, kseg);
  else
    hipLaunchKernelGGL((k_prolong_add<T, false>), dim3(blocks_for(total, 256)), dim3(256), 0, s, x,
                       ec, f.nx, f.ny, f.nz, kseg);
}

void launch_reduce_sum(const double* partial, int n, double* out, double* out_host,
                       hipStream_t s) {
  hipLaunchKernelGGL(k_reduce_sum, dim3(1), dim3(1024), 0, s, partial, n, out, out_host);
}

template <typename T>
void launch_fill(T* x, size_t n, T value, hipStream_t s) {
  if (n == 0) return;
  const int nb = static_cast<int>(std::min<size_t>((n + 255) / 256, 65536));
  hipLaunchKernelGGL(k_fill<T>, dim3(nb), dim3(256), 0, s, x, n, value);
}


template <typename T>
void launch_zero_interior(T* x, Dims d, hipStream_t s) {
  for (int c = 0; c < 3; ++c)
    launch_fill<T>(x + static_cast<size_t>(c) * d.comp() + d.plane(),
                   static_cast<size_t>(d.plane()) * (d.nz - 1), T(0), s);
}

template <typename T>
void launch_coarse_solve(const double* Ainv, int n, const T* b, T* x, Dims d, hipStream_t s) {
  if (n <= 0) return;
  hipLaunchKernelGGL(k_coarse_apply<T>, dim3(blocks_for(n, 4)), dim3(256), 0, s, Ainv, b, x, n,
                     d.plane(), d.nz);
}

#define QS_INST(T)                                                                               \
  template void launch_colour_fine<T>(T*, const T*, Dims, int, const FineCoef<T>&, hipStream_t); \
  template void launch_colour_gen<T>(T*, const T*, Dims, int, const T*, const T*, hipStream_t);  \
  template void launch_colour_pair_gen<T>(T*, const T*, Dims, int, const T*, hipStream_t);       \
  template void launch_residual_pair_gen<T>(const T*, const T*, T*, Dims, const T*, hipStream_t); \
  template int launch_residual_gen<T>(const T*, const T*, T*, Dims, const T*, bool, double*,     \
                                      hipStream_t);                                              \
  template void launch_restrict<T>(const T*, T*, T*, Dims, hipStream_t);                         \
  template void launch_prolong_add<T>(T*, const T*, Dims, hipStream_t);                          \
  template void launch_fill<T>(T*, size_t, T, hipStream_t);                                      \
  template void launch_zero_interior<T>(T*, Dims, hipStream_t);                                  \
  template void launch_coarse_solve<T>(const double*, int, const T*, T*, Dims, hipStream_t);
QS_INST(double)
QS_INST(float)
#undef QS_INST
template int launch_residual_fine<double, double>(const double*, const double*, double*, Dims,
                                                  const FineCoef<double>&, double, bool, double*,
                                                  hipStream_t);
template int launch_residual_fine<double, float>(const double*, const double*, float*, Dims,
                                                 const FineCoef<double>&, double, bool, double*,
                                                 hipStream_t);
template int launch_residual_fine<float, float>(const float*, const float*, float*, Dims,
                                                const FineCoef<double>&, double, bool, double*,
                                                hipStream_t);

}  // namespace qs
