// Row-parity Gauss-Seidel sweep of the fine level for gfx950 (smoother of
// Sec. 3.6 applied to the operator of Sec. 3.4).
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
// f-1, which needs the new planes f-2 and f.  Each thread owns one column pair
// (2t, 2t+1) of its row and updates the column of the active x parity in each
// phase, so every lane works in every phase; the pair moves between HBM and
// LDS as one two-wide access.
//
// LDS.  Planes f-2..f+1 of the row and of its two neighbour rows sit in a ring
// of four planes.  Each LDS row holds the nx columns plus a copy of column
// nx-1 before column 0 and of column 0 after column nx-1, so that the x
// neighbours of every column are at fixed offsets; with the row length a
// compile-time constant every stencil read is one base register plus an
// immediate offset.
//
// Segments.  The second-parity planes at the segment ends need first-parity
// planes just outside the segment: the workgroup recomputes those (one plane
// per end) from old values, so the sweep reads `own_src` / `nbr_src` and
// writes `dst` (ping-pong buffers):
//   even-row half: own rows and neighbour rows from the old vector,
//   odd-row half:  own rows from the old vector, neighbour rows from the new.
// Workgroups are mapped so that each XCD (round-robin dispatch over 8) gets a
// contiguous block of (row group, segment) pairs, by default neighbouring row
// groups of one segment: rows next to each other then run on the same XCD, at
// the same planes, and share their neighbour rows through its L2.  The
// segment length is chosen so that the whole launch is one round of resident
// workgroups.
#include <hip/hip_runtime.h>

#include <algorithm>

#include "device.h"

namespace qs {

namespace {

template <typename T>
struct V2;
template <>
struct V2<float> {
  using type = float2;
};
template <>
struct V2<double> {
  using type = double2;
};

struct SweepArgs {
  int nx, ny, nz;
  int row_par;       // parity of the rows updated
  int plane_first;   // parity of the planes updated first
  int x_first;       // parity of the columns updated first in each plane
  int seg;           // planes per segment
  int nseg;          // segments
  int rows;          // rows of this parity per workgroup
  int ngroups;       // workgroups per segment column
  int real_wgs;      // ngroups * nseg
  int grid_per_xcd;  // padded grid / 8
  int seg_major;     // 1: consecutive workgroups take consecutive row groups of one segment
  int xs;            // column segments per row (2 for FP64 rows of 768, else 1)
};

constexpr int kPad = 2;  // LDS row: [unused][copy of col nx-1][cols 0..nx-1][copy of col 0][unused]
// FP64 rows of 768 nodes do not fit the ring of one workgroup (223 KB of LDS):
// there two workgroups share a row, each holding its 384 columns and kHalo
// columns on either side, which it updates as well (from the same old values,
// so that its own columns see exact neighbours) but does not write.  Wrong
// values at a halo's outer edge travel inward one column per update phase,
// three columns within a step (the two x-parity phases of a first-parity
// plane, then of the second-parity plane below it); the next step starts
// again from old values, so four halo columns keep every written column exact.
constexpr int kHalo = 4;
constexpr int kSplitW = 384;

// rows of one parity per workgroup: two at 256 columns, more for shorter rows
// (at most 256 threads), one at 384, 512 and 768 (384 threads)
int rows_per_group(int nx) { return std::max(1, std::min(64, 512 / nx)); }

// Per-thread state of the sweep, passed by value so that it stays in registers.
template <typename T, int NX>
struct Ctx {
  T* ring;   // [4 planes][2 rows + 1][3 components][NXP]: rows j0-1 .. j0+2 rows-1
  int nx;    // row length (NX when NX > 0)
  int rows;  // rows per workgroup
  int r;     // row of this thread within the workgroup (ring rows 2r .. 2r+2)
  int c0;    // first column of this thread's pair
  int tpr;   // threads per row
  int j, jm, jp;
  size_t P, C;
  bool write;  // false for rows past the last one of this parity (last group)
  // rows of 768 FP64 values: split into two column segments (see kHalo)
  static constexpr bool kSplit = NX == 768 && sizeof(T) == 8;
  int gc0;       // global column of this thread's pair (c0 without the split)
  bool own_col;  // the pair is one the workgroup writes (not halo)
  // prolongation variants (Z = 3, 4): the coarse correction ec, its plane
  // and component strides, the coarse columns I, I+1 of this pair and the
  // coarse rows A (row j-1, or j for even j) and B (row j+1)
  const T* ec;
  size_t Pc, Cc;
  int nzc, I, I1, JA, JB;
  __device__ __forceinline__ int nxp() const {
    return (kSplit ? kSplitW + 2 * kHalo : (NX > 0 ? NX : nx)) + 2 * kPad;
  }
  // column 0 of LDS row q = 3 rr + component of this thread's rows
  // (rr 0, 1, 2 = j-1, j, j+1) in the plane held in ring slot (plane & 3);
  // the rows of a workgroup are consecutive, so the neighbour row between two
  // of its rows is stored once
  __device__ __forceinline__ T* row(int plane, int q) const {
    return ring + (((plane & 3) * (2 * rows + 1) + 2 * r) * 3 + q) * nxp() + kPad;
  }
};

// Values of one plane that a thread moves into the ring: its rows j-1 and j,
// and the row j+1 for the workgroup's last row (the other rows j+1 are the
// next thread row's j-1).
template <typename T>
struct PlaneRegs {
  typename V2<T>::type v[9];
};

// Z = 0: rows as stored; Z = 1: the thread's own row reads as zero; Z = 2:
// own and neighbour rows read as zero (a vector known to be zero is not
// fetched); Z = 3: own and neighbour rows read as x + T e_c, the coarse-grid
// correction prolongated on the fly (the first half of the first
// post-smoothing sweep, which thereby also applies the correction); Z = 4:
// the own rows read as x + T e_c (its second half: the neighbour rows come
// corrected from the first half's output).  The correction is added where the
// registers go into the ring (correct_plane).
template <typename T, int NX, int Z>
__device__ __forceinline__ void fetch_plane(const Ctx<T, NX>& c, const T* __restrict__ own_src,
                                            const T* __restrict__ nbr_src, int p,
                                            PlaneRegs<T>& out) {
  using V = typename V2<T>::type;
  const int nx = NX > 0 ? NX : c.nx;
  const size_t o = static_cast<size_t>(p) * c.P + c.gc0;
  const size_t om = o + static_cast<size_t>(c.jm) * nx;
  const size_t oo = o + static_cast<size_t>(c.j) * nx;
  const size_t op = o + static_cast<size_t>(c.jp) * nx;
  const bool top = c.r == c.rows - 1;  // uniform over a wavefront's row
  const V zero = V{T(0), T(0)};
#pragma unroll
  for (int k = 0; k < 3; ++k) {
    out.v[k] = Z == 2 ? zero : *reinterpret_cast<const V*>(nbr_src + k * c.C + om);
    out.v[3 + k] = (Z == 1 || Z == 2) ? zero : NT2<T>::template load<V>(own_src + k * c.C + oo);
  }
  if (top) {
#pragma unroll
    for (int k = 0; k < 3; ++k)
      out.v[6 + k] = Z == 2 ? zero : *reinterpret_cast<const V*>(nbr_src + k * c.C + op);
  }
}

// Coarse values behind the correction of two consecutive fine planes: coarse
// planes Ka and Ka + 1 (clamped to the top wall, whose values are zero), rows
// A and B (Z = 3) or A (Z = 4), columns I and I + 1, three components.
template <typename T>
struct CoarseRegs {
  T e[2][2][2][3];  // [plane Ka, Ka+1][row A, B][column I, I+1][component]
};

template <typename T, int NX, int Z>
__device__ __forceinline__ void fetch_coarse(const Ctx<T, NX>& c, int Ka, CoarseRegs<T>& out) {
  if (Z != 3 && Z != 4) return;
#pragma unroll
  for (int kp = 0; kp < 2; ++kp) {
    const size_t base = static_cast<size_t>(min(Ka + kp, c.nzc)) * c.Pc;
    const int nxc = NX > 0 ? NX / 2 : c.nx / 2;
#pragma unroll
    for (int rb = 0; rb < (Z == 3 ? 2 : 1); ++rb) {
      const size_t o = base + static_cast<size_t>(rb ? c.JB : c.JA) * nxc;
#pragma unroll
      for (int k = 0; k < 3; ++k) {
        out.e[kp][rb][0][k] = c.ec[k * c.Cc + o + c.I];
        out.e[kp][rb][1][k] = c.ec[k * c.Cc + o + c.I1];
      }
    }
  }
}

// x + T e_c for the fine plane p (coarse planes Ka, Ka+1 in ce) on the rows
// of `in` that need it, in the arithmetic of k_prolong_add: the x, y
// combination of each coarse plane, then the z mean on odd planes.
template <typename T, int NX, int Z>
__device__ __forceinline__ void correct_plane(const Ctx<T, NX>& c, int p, int Ka,
                                              const CoarseRegs<T>& ce, PlaneRegs<T>& in) {
  if (Z != 3 && Z != 4) return;
  const T h = T(0.5);
  const int k0 = (p >> 1) - Ka, k1 = min((p + 1) >> 1, c.nzc) - Ka;
  const bool oz = p & 1;
  // fine rows: q = 0 row j-1, 1 row j, 2 row j+1 (top thread only)
  const bool top = c.r == c.rows - 1;
#pragma unroll
  for (int q = 0; q < 3; ++q) {
    if (Z == 4 && q != 1) continue;      // own row only
    if (q == 2 && !top) continue;
    // Z = 3: j is odd, rows j-1 and j+1 even (coarse rows A and B), row j
    // between them; Z = 4: j is even, coarse row A
    const bool oy = Z == 3 && q == 1;
    const int ra = (Z == 3 && q == 2) ? 1 : 0;
#pragma unroll
    for (int k = 0; k < 3; ++k) {
      // x, y combination of both coarse planes (static indices, so that the
      // coarse values stay in registers), then the planes this fine plane uses
      T pe[2], po[2];
#pragma unroll
      for (int kp = 0; kp < 2; ++kp) {
        const T a0 = ce.e[kp][ra][0][k], a1 = ce.e[kp][ra][1][k];
        if (oy) {
          const T b0 = ce.e[kp][1][0][k], b1 = ce.e[kp][1][1][k];
          pe[kp] = h * (a0 + b0);
          po[kp] = h * (h * (a0 + a1) + h * (b0 + b1));
        } else {
          pe[kp] = a0;
          po[kp] = h * (a0 + a1);
        }
      }
      const T pe0 = k0 ? pe[1] : pe[0], po0 = k0 ? po[1] : po[0];
      const T pe1 = k1 ? pe[1] : pe[0], po1 = k1 ? po[1] : po[0];
      typename V2<T>::type& v = in.v[3 * q + k];
      if (oz) {
        v.x += h * (pe0 + pe1);
        v.y += h * (po0 + po1);
      } else {
        v.x += pe0;
        v.y += po0;
      }
    }
  }
}

template <typename T, int NX>
__device__ __forceinline__ void store_plane(const Ctx<T, NX>& c, int p, const PlaneRegs<T>& in) {
  using V = typename V2<T>::type;
  const int nx = NX > 0 ? NX : c.nx;
  // the pair holding column 0 also writes its copy after the row end, the
  // pair holding column nx-1 its copy before column 0; every other thread
  // writes its first value once more onto itself (no branch)
  const bool hi = !Ctx<T, NX>::kSplit && c.c0 == nx - 2;
  const int g = Ctx<T, NX>::kSplit ? c.c0 : (c.c0 == 0 ? nx : (hi ? -1 : c.c0));
  T* base = c.row(p, 0);
  const int nq = c.r == c.rows - 1 ? 9 : 6;
#pragma unroll
  for (int q = 0; q < 9; ++q) {
    if (q < nq) {
      T* rw = base + q * c.nxp();
      *reinterpret_cast<V*>(rw + c.c0) = in.v[q];
      rw[g] = hi ? in.v[q].y : in.v[q].x;
    }
  }
}

// b at plane p, the plane clamped into the interior (b is used only there).
template <typename T, int NX>
__device__ __forceinline__ void fetch_b(const Ctx<T, NX>& c, const T* __restrict__ b, int p, int nz,
                                        typename V2<T>::type out[3]) {
  using V = typename V2<T>::type;
  p = min(max(p, 1), nz - 1);
  const int nx = NX > 0 ? NX : c.nx;
  const size_t o = static_cast<size_t>(p) * c.P + static_cast<size_t>(c.j) * nx + c.gc0;
#pragma unroll
  for (int k = 0; k < 3; ++k) out[k] = NT2<T>::template load<V>(b + k * c.C + o);
}

// Gauss-Seidel value of the node (row j, plane p, column col):
// x = D^-1 (b - sum_{q != p} A_pq x_q) with the fine-operator stencil.
template <typename T, int NX>
__device__ __forceinline__ void gs_node(const Ctx<T, NX>& c, int p, int col, T b0, T b1, T b2,
                                        const FineCoef<T>& cf, T& o0, T& o1, T& o2) {
  const int W = c.nxp();
  // base pointers at column col-1 of row 0 (j-1) of planes p-1, p, p+1
  const T* zm = c.row(p - 1, 0) + col - 1;
  const T* z0 = c.row(p, 0) + col - 1;
  const T* zp = c.row(p + 1, 0) + col - 1;
#define RX(ptr, rr, k, dx) ptr[((rr) * 3 + (k)) * W + 1 + (dx)]
  const T fx0 = RX(z0, 1, 0, 1) + RX(z0, 1, 0, -1);
  const T fy0 = RX(z0, 2, 0, 0) + RX(z0, 0, 0, 0);
  const T fz0 = RX(zp, 1, 0, 0) + RX(zm, 1, 0, 0);
  const T fx1 = RX(z0, 1, 1, 1) + RX(z0, 1, 1, -1);
  const T fy1 = RX(z0, 2, 1, 0) + RX(z0, 0, 1, 0);
  const T fz1 = RX(zp, 1, 1, 0) + RX(zm, 1, 1, 0);
  const T fx2 = RX(z0, 1, 2, 1) + RX(z0, 1, 2, -1);
  const T fy2 = RX(z0, 2, 2, 0) + RX(z0, 0, 2, 0);
  const T fz2 = RX(zp, 1, 2, 0) + RX(zm, 1, 2, 0);
  // mixed differences f(+,+) - f(+,-) - f(-,+) + f(-,-)
  const T mxy0 = RX(z0, 2, 0, 1) - RX(z0, 0, 0, 1) - RX(z0, 2, 0, -1) + RX(z0, 0, 0, -1);
  const T mxy1 = RX(z0, 2, 1, 1) - RX(z0, 0, 1, 1) - RX(z0, 2, 1, -1) + RX(z0, 0, 1, -1);
  const T mxz0 = RX(zp, 1, 0, 1) - RX(zm, 1, 0, 1) - RX(zp, 1, 0, -1) + RX(zm, 1, 0, -1);
  const T mxz2 = RX(zp, 1, 2, 1) - RX(zm, 1, 2, 1) - RX(zp, 1, 2, -1) + RX(zm, 1, 2, -1);
  const T myz1 = RX(zp, 2, 1, 0) - RX(zm, 2, 1, 0) - RX(zp, 0, 1, 0) + RX(zm, 0, 1, 0);
  const T myz2 = RX(zp, 2, 2, 0) - RX(zm, 2, 2, 0) - RX(zp, 0, 2, 0) + RX(zm, 0, 2, 0);
#undef RX
  o0 = (cf.h2 * b0 + cf.p * fx0 + cf.q * (fy0 + fz0) + cf.m4 * (mxy1 + mxz2)) * cf.inv_diag;
  o1 = (cf.h2 * b1 + cf.p * fy1 + cf.q * (fx1 + fz1) + cf.m4 * (mxy0 + myz2)) * cf.inv_diag;
  o2 = (cf.h2 * b2 + cf.p * fz2 + cf.q * (fx2 + fy2) + cf.m4 * (mxz0 + myz1)) * cf.inv_diag;
}

// Update column c0 + xp of plane p and write it into the ring (and its copy
// past the row end when it is column 0 or nx-1).
template <typename T, int NX, int XP>
__device__ __forceinline__ void update_phase(const Ctx<T, NX>& c, int p,
                                             const typename V2<T>::type bv[3],
                                             const FineCoef<T>& cf, T o[3]) {
  const int nx = NX > 0 ? NX : c.nx;
  const int col = c.c0 + XP;
  const T b0 = XP ? bv[0].y : bv[0].x;
  const T b1 = XP ? bv[1].y : bv[1].x;
  const T b2 = XP ? bv[2].y : bv[2].x;
  gs_node<T, NX>(c, p, col, b0, b1, b2, cf, o[0], o[1], o[2]);
  T* own = c.row(p, 3);
  const int W = c.nxp();
  // copy of column 0 after the row end / of column nx-1 before column 0
  const int g = Ctx<T, NX>::kSplit ? col : (col == 0 ? nx : (col == nx - 1 ? -1 : col));
#pragma unroll
  for (int k = 0; k < 3; ++k) {
    own[k * W + col] = o[k];
    own[k * W + g] = o[k];
  }
}

// Both x-parity phases of plane p (barrier between them); the updated pair is
// written to dst if p lies in this workgroup's segment [z0, z1).
template <typename T, int NX, int X1>
__device__ __forceinline__ void update_plane(const Ctx<T, NX>& c, int p, int z0, int z1,
                                             const typename V2<T>::type bv[3],
                                             const FineCoef<T>& cf, T* __restrict__ dst) {
  using V = typename V2<T>::type;
  T oa[3], ob[3];
  update_phase<T, NX, X1>(c, p, bv, cf, oa);
  __syncthreads();
  update_phase<T, NX, 1 - X1>(c, p, bv, cf, ob);
  if (c.write && c.own_col && p >= z0 && p < z1) {
    const int nx = NX > 0 ? NX : c.nx;
    const size_t o = static_cast<size_t>(p) * c.P + static_cast<size_t>(c.j) * nx + c.gc0;
#pragma unroll
    for (int k = 0; k < 3; ++k) {
      V v;
      v.x = X1 ? ob[k] : oa[k];
      v.y = X1 ? oa[k] : ob[k];
      NT2<T>::store(dst + k * c.C + o, v);
    }
  }
}

// Registers of one step of the march at first-parity plane f: planes f+2
// and f+3 and b at planes f+2 and f+1.
template <typename T, int Z>
struct StepRegs {
  PlaneRegs<T> p2, p3;
  typename V2<T>::type bf[3], bs[3];
  CoarseRegs<T> ce[1];  // Z = 3, 4 only
};

// Issue the loads of the step whose planes are g = f+2 and g+1.
template <typename T, int NX, int Z>
__device__ __forceinline__ void fetch_step(const Ctx<T, NX>& c, const T* __restrict__ own_src,
                                           const T* __restrict__ nbr_src, const T* __restrict__ b,
                                           int g, int nz, StepRegs<T, Z>& s) {
  fetch_b<T, NX>(c, b, g, nz, s.bf);
  fetch_b<T, NX>(c, b, g - 1, nz, s.bs);
  fetch_plane<T, NX, Z>(c, own_src, nbr_src, min(g, nz), s.p2);
  fetch_plane<T, NX, Z>(c, own_src, nbr_src, min(g + 1, nz), s.p3);
  fetch_coarse<T, NX, Z>(c, min(g, nz) >> 1, s.ce[0]);
}

// One step of the march: issue the loads for two steps ahead into `nxt`,
// update planes f and f-1 from the ring, then move `cur` (planes f+2, f+3)
// into the slots of f-2 and f-1 and its b values into bf / bs.
template <typename T, int NX, int X1, int Z>
__device__ __forceinline__ void march_step(const Ctx<T, NX>& c, const T* __restrict__ own_src,
                                           const T* __restrict__ nbr_src, const T* __restrict__ b,
                                           T* __restrict__ dst, const FineCoef<T>& cf, int f,
                                           int z0, int z1, int nz, typename V2<T>::type bf[3],
                                           typename V2<T>::type bs[3], StepRegs<T, Z>& cur,
                                           StepRegs<T, Z>& nxt) {
  fetch_step<T, NX, Z>(c, own_src, nbr_src, b, f + 4, nz, nxt);
  update_plane<T, NX, X1>(c, f, z0, z1, bf, cf, dst);
  __syncthreads();
  const int sp = f - 1;  // second-parity plane below f
  if (sp >= z0 && sp <= z1 - 1 && sp >= 1) {
    update_plane<T, NX, X1>(c, sp, z0, z1, bs, cf, dst);
    __syncthreads();
  }
  {
    const int Ka = min(f + 2, nz) >> 1;  // as fetch_step
    correct_plane<T, NX, Z>(c, min(f + 2, nz), Ka, cur.ce[0], cur.p2);
    correct_plane<T, NX, Z>(c, min(f + 3, nz), Ka, cur.ce[0], cur.p3);
  }
  if (f + 2 <= nz) store_plane<T, NX>(c, f + 2, cur.p2);
  if (f + 3 <= nz) store_plane<T, NX>(c, f + 3, cur.p3);
#pragma unroll
  for (int k = 0; k < 3; ++k) {
    bf[k] = cur.bf[k];
    bs[k] = cur.bs[k];
  }
  __syncthreads();
}

// threads per workgroup: rows * nx/2, at most 256 except for 768-column rows
// (FP64 rows of 768 are split over two workgroups of 196 threads)
template <typename T>
constexpr int sweep_max_threads(int nx) { return nx == 768 && sizeof(T) == 4 ? 384 : 256; }

template <typename T, int NX, int X1, int Z>
__global__ __launch_bounds__(sweep_max_threads<T>(NX)) void k_sweep_rows(const T* __restrict__ own_src,
                                                    const T* __restrict__ nbr_src,
                                                    T* __restrict__ dst, const T* __restrict__ b,
                                                    const T* __restrict__ ec,
                                                    SweepArgs a, FineCoef<T> cf) {
  using V = typename V2<T>::type;
  extern __shared__ __align__(16) unsigned char smem[];
  // XCD-aware mapping of the (padded) grid onto (row group, segment)
  const int wg = blockIdx.x;
  const int L0 = (wg & 7) * a.grid_per_xcd + (wg >> 3);
  if (L0 >= a.real_wgs) return;  // whole workgroup leaves before any barrier
  const int xseg = L0 % a.xs, L = L0 / a.xs;  // the column segments of a row group are neighbours
  int group, sgi;
  if (a.seg_major) {
    sgi = L / a.ngroups;
    group = L - sgi * a.ngroups;
  } else {
    group = L / a.nseg;
    sgi = L - group * a.nseg;
  }
  Ctx<T, NX> c;
  c.ring = reinterpret_cast<T*>(smem);
  c.nx = NX > 0 ? NX : a.nx;
  c.rows = a.rows;
  c.tpr = (Ctx<T, NX>::kSplit ? kSplitW + 2 * kHalo : c.nx) >> 1;
  c.r = threadIdx.x / c.tpr;
  c.c0 = 2 * (threadIdx.x - c.r * c.tpr);
  if (Ctx<T, NX>::kSplit) {
    int g = xseg * kSplitW - kHalo + c.c0;
    g = g < 0 ? g + c.nx : (g >= c.nx ? g - c.nx : g);
    c.gc0 = g;
    c.own_col = c.c0 >= kHalo && c.c0 < kHalo + kSplitW;
  } else {
    c.gc0 = c.c0;
    c.own_col = true;
  }
  // threads = rows * tpr, so every thread has a row slot; rows past the last
  // row of this parity (last group only) are computed on the wrapped row
  // index, which keeps the shared neighbour rows consistent, and not written
  const int jr = 2 * (group * a.rows + c.r) + a.row_par;
  const int jlast = a.ny - 2 + a.row_par;
  c.write = jr <= jlast;
  c.j = jr % a.ny;
  c.jm = c.j == 0 ? a.ny - 1 : c.j - 1;
  c.jp = c.j + 1 >= a.ny ? c.j + 1 - a.ny : c.j + 1;
  c.P = static_cast<size_t>(c.nx) * a.ny;
  c.C = static_cast<size_t>(a.nz + 1) * c.P;
  if (Z == 3 || Z == 4) {
    const int nxc = c.nx / 2, nyc = a.ny / 2;
    c.ec = ec;
    c.nzc = a.nz / 2;
    c.Pc = static_cast<size_t>(nxc) * nyc;
    c.Cc = static_cast<size_t>(c.nzc + 1) * c.Pc;
    c.I = c.gc0 >> 1;
    c.I1 = c.I + 1 == nxc ? 0 : c.I + 1;
    c.JA = Z == 3 ? (c.jm >> 1) : (c.j >> 1);
    c.JB = c.jp >> 1;
  }

  const int nz = a.nz;
  const int z0 = 1 + sgi * a.seg;
  const int z1 = min(z0 + a.seg, nz);  // segment = interior planes [z0, z1)
  const int pf = a.plane_first;
  // first-parity planes: parity pf, interior, in [z0-1, z1]
  int f0 = max(z0 - 1, 1);
  if ((f0 & 1) != pf) ++f0;
  int flast = min(z1, nz - 1);
  if ((flast & 1) != pf) --flast;
  if (f0 > flast) return;  // uniform over the workgroup

  // The ring holds planes f-2 .. f+1 while planes f and f-1 are updated.
  // Loads run two steps ahead: while the step at f computes, the registers of
  // one set (planes f+2, f+3, b at f+2 and f+1, issued a step earlier) are in
  // flight or have landed, and the other set is being filled for the step at
  // f+2 (planes f+4, f+5).  At the end of the step the first set goes into
  // the ring slots of planes f-2 and f-1.  All plane indices are clamped into
  // the arrays, so every step issues the same loads (the compiler can then
  // count them exactly when it waits for a set) and values fetched past the
  // walls are never used.
  const int first = f0 - 1 >= z0 ? f0 - 2 : f0 - 1;  // bottom segment: the wall plane too
  V bf[3], bs[3];
  fetch_b<T, NX>(c, b, f0, nz, bf);
  fetch_b<T, NX>(c, b, f0 - 1, nz, bs);
  StepRegs<T, Z> ra, rb;
  {
    PlaneRegs<T> q0, q1, q2, q3;
    fetch_plane<T, NX, Z>(c, own_src, nbr_src, max(f0 - 2, 0), q0);
    fetch_plane<T, NX, Z>(c, own_src, nbr_src, f0 - 1, q1);
    fetch_plane<T, NX, Z>(c, own_src, nbr_src, f0, q2);
    fetch_plane<T, NX, Z>(c, own_src, nbr_src, f0 + 1, q3);  // f0 + 1 <= nz
    if (Z == 3 || Z == 4) {
      // coarse planes of the fine planes f0-2 .. f0+1 (first loads of the march)
      CoarseRegs<T> lo, hi;
      const int Klo = max(f0 - 2, 0) >> 1, Khi = f0 >> 1;
      fetch_coarse<T, NX, Z>(c, Klo, lo);
      fetch_coarse<T, NX, Z>(c, Khi, hi);
      correct_plane<T, NX, Z>(c, max(f0 - 2, 0), Klo, lo, q0);
      // plane f0 - 1 needs coarse planes (f0-1)>>1 and f0>>1: within [Klo, Klo + 1]
      correct_plane<T, NX, Z>(c, f0 - 1, Klo, lo, q1);
      correct_plane<T, NX, Z>(c, f0, Khi, hi, q2);
      correct_plane<T, NX, Z>(c, f0 + 1, Khi, hi, q3);
    }
    fetch_step<T, NX, Z>(c, own_src, nbr_src, b, f0 + 2, nz, ra);
    if (first == f0 - 2) store_plane<T, NX>(c, f0 - 2, q0);
    store_plane<T, NX>(c, f0 - 1, q1);
    store_plane<T, NX>(c, f0, q2);
    store_plane<T, NX>(c, f0 + 1, q3);
  }
  __syncthreads();
  for (int f = f0;; f += 4) {
    march_step<T, NX, X1, Z>(c, own_src, nbr_src, b, dst, cf, f, z0, z1, nz, bf, bs, ra, rb);
    if (f + 2 > flast) break;
    march_step<T, NX, X1, Z>(c, own_src, nbr_src, b, dst, cf, f + 2, z0, z1, nz, bf, bs, rb, ra);
    if (f + 4 > flast) break;
  }
  const int sp = flast + 1;  // only when flast + 2 is the top wall (already in the ring)
  if (sp >= z0 && sp <= z1 - 1 && sp <= nz - 1) update_plane<T, NX, X1>(c, sp, z0, z1, bs, cf, dst);
}

template <typename T, int NX>
void launch_nx(const T* own_src, const T* nbr_src, T* dst, const T* b, const T* ec,
               const SweepArgs& a, const FineCoef<T>& cf, int zero, int threads, size_t lds,
               hipStream_t s) {
  const dim3 grid(8 * a.grid_per_xcd), block(threads);
#define QS_SWEEP(X1, Z)                                                                        \
  hipLaunchKernelGGL((k_sweep_rows<T, NX, X1, Z>), grid, block, lds, s, own_src, nbr_src, dst, b, \
                     ec, a, cf)
  if (a.x_first && zero == 3)
    QS_SWEEP(1, 3);
  else if (a.x_first && zero == 4)
    QS_SWEEP(1, 4);
  else if (a.x_first)
    QS_SWEEP(1, 0);
  else if (zero == 2)
    QS_SWEEP(0, 2);
  else if (zero == 1)
    QS_SWEEP(0, 1);
  else
    QS_SWEEP(0, 0);
#undef QS_SWEEP
}

template <typename T, int NX>
void set_lds_limit_one(int bytes) {
  const void* k[6] = {reinterpret_cast<const void*>(&k_sweep_rows<T, NX, 0, 0>),
                      reinterpret_cast<const void*>(&k_sweep_rows<T, NX, 1, 0>),
                      reinterpret_cast<const void*>(&k_sweep_rows<T, NX, 0, 1>),
                      reinterpret_cast<const void*>(&k_sweep_rows<T, NX, 0, 2>),
                      reinterpret_cast<const void*>(&k_sweep_rows<T, NX, 1, 3>),
                      reinterpret_cast<const void*>(&k_sweep_rows<T, NX, 1, 4>)};
  for (const void* f : k)
    (void)hipFuncSetAttribute(f, hipFuncAttributeMaxDynamicSharedMemorySize, bytes);
}

template <typename T>
void set_lds_limit_all(int bytes) {
  set_lds_limit_one<T, 0>(bytes);
  set_lds_limit_one<T, 128>(bytes);
  set_lds_limit_one<T, 256>(bytes);
  set_lds_limit_one<T, 384>(bytes);
  set_lds_limit_one<T, 512>(bytes);
  set_lds_limit_one<T, 768>(bytes);
}

}  // namespace

int sweep_rows_per_group(int nx) { return rows_per_group(nx); }

// column segments per row and threads per row of the row sweep
int column_segments(int nx, int bytes_per_value) { return nx == 768 && bytes_per_value == 8 ? 2 : 1; }
int threads_per_row(int nx, int bytes_per_value) {
  return column_segments(nx, bytes_per_value) == 2 ? (kSplitW + 2 * kHalo) / 2 : nx / 2;
}

template <typename T>
int blocks_per_cu(Dims d, int threads, size_t lds) {
  int n = 0;
  const void* k = nullptr;
  switch (d.nx) {
    case 128: k = reinterpret_cast<const void*>(&k_sweep_rows<T, 128, 0, 0>); break;
    case 256: k = reinterpret_cast<const void*>(&k_sweep_rows<T, 256, 0, 0>); break;
    case 384: k = reinterpret_cast<const void*>(&k_sweep_rows<T, 384, 0, 0>); break;
    case 512: k = reinterpret_cast<const void*>(&k_sweep_rows<T, 512, 0, 0>); break;
    case 768: k = reinterpret_cast<const void*>(&k_sweep_rows<T, 768, 0, 0>); break;
    default: k = reinterpret_cast<const void*>(&k_sweep_rows<T, 0, 0, 0>); break;
  }
  if (hipOccupancyMaxActiveBlocksPerMultiprocessor(&n, k, threads, lds) != hipSuccess) n = 1;
  return std::max(n, 1);
}

// Planes per segment: as many segments as make the launch one round of
// resident workgroups on the current device (measured: a second, partial round
// or half-empty CUs cost more than the halo planes of shorter segments).
int sweep_segment_length(Dims d, int bytes_per_value) {
  int dev = 0, cus = 256;
  if (hipGetDevice(&dev) != hipSuccess ||
      hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev) != hipSuccess)
    cus = 256;
  const int R = rows_per_group(d.nx);
  const int threads = R * threads_per_row(d.nx, bytes_per_value);
  const size_t lds = static_cast<size_t>(sweep_lds_bytes(d, bytes_per_value));
  const int per_cu = bytes_per_value == 8 ? blocks_per_cu<double>(d, threads, lds)
                                          : blocks_per_cu<float>(d, threads, lds);
  const int groups = std::max(1, ((d.ny + 1) / 2 + R - 1) / R) * column_segments(d.nx, bytes_per_value);
  const int slots = per_cu * cus;
  int nseg = std::max(1, slots / groups);
  // more row groups than resident slots: split z so that the launch is a
  // whole number of rounds when two or four segments make it one
  if (groups > slots && groups % slots != 0)
    for (int k : {2, 4})
      if ((groups * k) % slots == 0) {
        nseg = k;
        break;
      }
  const int seg = (d.nz - 1 + nseg - 1) / nseg;
  return std::max(seg, 4);
}

int sweep_lds_bytes(Dims d, int bytes_per_value) {
  const int w = column_segments(d.nx, bytes_per_value) == 2 ? kSplitW + 2 * kHalo : d.nx;
  return 4 * (2 * rows_per_group(d.nx) + 1) * 3 * (w + 2 * kPad) * bytes_per_value;
}

bool sweep_supported(Dims d, size_t lds_limit, int bytes_per_value) {
  if (d.nx % 2 != 0 || d.ny % 2 != 0 || d.nx < 4 || d.nz < 2) return false;
  if (d.nx > 512 && d.nx != 768) return false;
  return static_cast<size_t>(sweep_lds_bytes(d, bytes_per_value)) <= lds_limit;
}

template <typename T>
void launch_sweep_half(const T* own_src, const T* nbr_src, T* dst, const T* b, const T* ec, Dims d,
                       int row_par, int plane_first, int x_first, const FineCoef<T>& cf, int seg,
                       int seg_major, int zero, hipStream_t s) {
  SweepArgs a;
  a.nx = d.nx;
  a.ny = d.ny;
  a.nz = d.nz;
  a.row_par = row_par;
  a.plane_first = plane_first;
  a.x_first = x_first;
  a.seg = seg;
  a.nseg = (d.nz - 1 + seg - 1) / seg;
  a.rows = rows_per_group(d.nx);
  const int rows = (d.ny - row_par + 1) / 2;
  a.ngroups = (rows + a.rows - 1) / a.rows;
  a.xs = column_segments(d.nx, sizeof(T));
  a.real_wgs = a.ngroups * a.nseg * a.xs;
  a.grid_per_xcd = (a.real_wgs + 7) / 8;
  a.seg_major = seg_major;
  const int threads = a.rows * threads_per_row(d.nx, sizeof(T));
  const size_t lds = static_cast<size_t>(sweep_lds_bytes(d, sizeof(T)));
  switch (d.nx) {
    case 128: launch_nx<T, 128>(own_src, nbr_src, dst, b, ec, a, cf, zero, threads, lds, s); break;
    case 256: launch_nx<T, 256>(own_src, nbr_src, dst, b, ec, a, cf, zero, threads, lds, s); break;
    case 384: launch_nx<T, 384>(own_src, nbr_src, dst, b, ec, a, cf, zero, threads, lds, s); break;
    case 512: launch_nx<T, 512>(own_src, nbr_src, dst, b, ec, a, cf, zero, threads, lds, s); break;
    case 768: launch_nx<T, 768>(own_src, nbr_src, dst, b, ec, a, cf, zero, threads, lds, s); break;
    default: launch_nx<T, 0>(own_src, nbr_src, dst, b, ec, a, cf, zero, threads, lds, s); break;
  }
}

void sweep_set_lds_limit(size_t bytes) {
  set_lds_limit_all<double>(static_cast<int>(bytes));
  set_lds_limit_all<float>(static_cast<int>(bytes));
}

template void launch_sweep_half<double>(const double*, const double*, double*, const double*,
                                        const double*, Dims, int, int, int,
                                        const FineCoef<double>&, int, int, int, hipStream_t);
template void launch_sweep_half<float>(const float*, const float*, float*, const float*,
                                       const float*, Dims, int, int, int, const FineCoef<float>&,
                                       int, int, int, hipStream_t);

}  // namespace qs
