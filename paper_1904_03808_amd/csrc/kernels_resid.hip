// Fine-level residual r = b - K x by z-marching tiles (gfx950).
//
// A workgroup of 64 x 4 threads owns a 64 x 4 column tile and a segment of
// z planes.  Planes k-1, k, k+1 of the tile plus a one-node halo in x and y
// sit in an LDS ring of three planes, so each value of x is loaded once per
// workgroup (the halo columns once more by the neighbouring tile, usually
// from L2); the next plane is fetched into registers while the current one
// is computed.  The squared residual is summed per workgroup in double for
// the convergence test.  b and the outputs are touched once and carry the
// non-temporal hint, which leaves L2 to the shared halo of x.  Tiles are
// ordered so that each XCD takes a contiguous block of them (neighbouring
// tiles share halos through its L2).
#include <hip/hip_runtime.h>

#include <algorithm>

#include "device.h"

namespace qs {

namespace {

constexpr int TX = 64, TY = 4, HX = TX + 2, HY = TY + 2, HALO = HX * HY;
constexpr int SEGZ = 32;

struct ZmArgs {
  int nx, ny, nz;
  int ntx, nty, nseg;
  int real_wgs, grid_per_xcd;
};

template <typename T>
__device__ __forceinline__ int slot_idx(int p, int c, int hy, int hx) {
  return (((p % 3) * 3 + c) * HY + hy) * HX + hx;
}

// UPD: the iterate is first advanced by a correction, x' = x + es * e (the
// refinement step of FP32 V-cycles inside FP64), x' is written to x_out on
// the interior nodes of the tile and segment, and the residual is that of x'.
// Every workgroup forms x' on its halo itself (same arithmetic), so x' must
// go to another buffer than x.
template <typename Tin, typename Tout, bool UPD>
__global__ __launch_bounds__(256) void k_residual_zm(const Tin* __restrict__ x,
                                                     const Tin* __restrict__ b,
                                                     Tout* __restrict__ r, ZmArgs a,
                                                     FineCoef<Tin> cf, Tin out_scale,
                                                     double* __restrict__ partial,
                                                     const float* __restrict__ e, double es,
                                                     Tin* __restrict__ x_out) {
  __shared__ Tin ring[3 * 3 * HALO];
  __shared__ double red[4];
  const int wg = blockIdx.x;
  const int L = (wg & 7) * a.grid_per_xcd + (wg >> 3);
  if (L >= a.real_wgs) return;
  const int tx = L % a.ntx;
  const int rest = L / a.ntx;
  const int ty = rest % a.nty;
  const int sg = rest / a.nty;
  const int nx = a.nx, ny = a.ny, nz = a.nz;
  const int i0 = tx * TX, j0 = ty * TY;
  const int lx = threadIdx.x % TX, ly = threadIdx.x / TX;
  const int i = i0 + lx, j = j0 + ly;
  const bool own = (i < nx) && (j < ny);
  const size_t P = static_cast<size_t>(nx) * ny, C = static_cast<size_t>(nz + 1) * P;
  const int z0 = 1 + sg * SEGZ, z1 = min(z0 + SEGZ, nz);

  // halo element e of the tile -> global column offset in a plane
  size_t hoff[2];
  int hcount = 0;
#pragma unroll
  for (int u = 0; u < 2; ++u) {
    const int e = threadIdx.x + u * 256;
    if (e < HALO) {
      const int hy = e / HX, hx = e - hy * HX;
      int gj = j0 + hy - 1, gi = i0 + hx - 1;
      gj = ((gj % ny) + ny) % ny;
      gi = ((gi % nx) + nx) % nx;
      hoff[u] = static_cast<size_t>(gj) * nx + gi;
      hcount = u + 1;
    }
  }
  Tin pre[2][3];
  auto fetch = [&](int p) {
#pragma unroll
    for (int u = 0; u < 2; ++u)
      if (u < hcount)
#pragma unroll
        for (int c = 0; c < 3; ++c) {
          const size_t q = c * C + static_cast<size_t>(p) * P + hoff[u];
          if constexpr (UPD)
            pre[u][c] = x[q] + es * static_cast<double>(e[q]);
          else
            pre[u][c] = x[q];
        }
  };
  auto store = [&](int p) {
#pragma unroll
    for (int u = 0; u < 2; ++u)
      if (u < hcount) {
        const int e = threadIdx.x + u * 256;
#pragma unroll
        for (int c = 0; c < 3; ++c) ring[((p % 3) * 3 + c) * HALO + e] = pre[u][c];
      }
  };
  const size_t oown = own ? static_cast<size_t>(j) * nx + i : 0;
  Tin bc[3] = {Tin(0), Tin(0), Tin(0)}, bn[3] = {Tin(0), Tin(0), Tin(0)};
  auto fetch_b = [&](int p, Tin out[3]) {
    if (b && own && p >= 1 && p <= nz - 1) {
#pragma unroll
      for (int c = 0; c < 3; ++c)
        out[c] = __builtin_nontemporal_load(b + c * C + static_cast<size_t>(p) * P + oown);
    }
  };

  fetch(z0 - 1);
  store(z0 - 1);
  fetch(z0);
  store(z0);
  fetch(z0 + 1);
  fetch_b(z0, bc);
  double sq = 0.0;
  const Tin diag = Tin(2) * (cf.p + Tin(2) * cf.q);
  const int hx = lx + 1, hy = ly + 1;
  // Memory counters complete in order: drain the prologue loads before the
  // loop (a wait for them inside it would also wait for the prefetch), and
  // issue b of the next plane before the prefetch of plane p + 2, so that
  // handing b over at the end of an iteration leaves the prefetch in flight.
  __builtin_amdgcn_s_waitcnt(0);
  for (int p = z0; p < z1; ++p) {
    store(p + 1);
    __syncthreads();
    fetch_b(p + 1, bn);
    if (p + 2 <= nz) fetch(p + 2);
    if (own) {
#define X(c, dz, dy, dx) ring[slot_idx<Tin>(p + (dz), c, hy + (dy), hx + (dx))]
      const Tin fx0 = X(0, 0, 0, 1) + X(0, 0, 0, -1), fy0 = X(0, 0, 1, 0) + X(0, 0, -1, 0),
                fz0 = X(0, 1, 0, 0) + X(0, -1, 0, 0);
      const Tin fx1 = X(1, 0, 0, 1) + X(1, 0, 0, -1), fy1 = X(1, 0, 1, 0) + X(1, 0, -1, 0),
                fz1 = X(1, 1, 0, 0) + X(1, -1, 0, 0);
      const Tin fx2 = X(2, 0, 0, 1) + X(2, 0, 0, -1), fy2 = X(2, 0, 1, 0) + X(2, 0, -1, 0),
                fz2 = X(2, 1, 0, 0) + X(2, -1, 0, 0);
      // mixed differences f(+,+) - f(+,-) - f(-,+) + f(-,-)
      const Tin mxy0 = X(0, 0, 1, 1) - X(0, 0, -1, 1) - X(0, 0, 1, -1) + X(0, 0, -1, -1);
      const Tin mxy1 = X(1, 0, 1, 1) - X(1, 0, -1, 1) - X(1, 0, 1, -1) + X(1, 0, -1, -1);
      const Tin mxz0 = X(0, 1, 0, 1) - X(0, -1, 0, 1) - X(0, 1, 0, -1) + X(0, -1, 0, -1);
      const Tin mxz2 = X(2, 1, 0, 1) - X(2, -1, 0, 1) - X(2, 1, 0, -1) + X(2, -1, 0, -1);
      const Tin myz1 = X(1, 1, 1, 0) - X(1, -1, 1, 0) - X(1, 1, -1, 0) + X(1, -1, -1, 0);
      const Tin myz2 = X(2, 1, 1, 0) - X(2, -1, 1, 0) - X(2, 1, -1, 0) + X(2, -1, -1, 0);
      const Tin off0 = cf.p * fx0 + cf.q * (fy0 + fz0) + cf.m4 * (mxy1 + mxz2);
      const Tin off1 = cf.p * fy1 + cf.q * (fx1 + fz1) + cf.m4 * (mxy0 + myz2);
      const Tin off2 = cf.p * fz2 + cf.q * (fx2 + fy2) + cf.m4 * (mxz0 + myz1);
      const Tin r0 = bc[0] - (diag * X(0, 0, 0, 0) - off0) * cf.ih2;
      const Tin r1 = bc[1] - (diag * X(1, 0, 0, 0) - off1) * cf.ih2;
      const Tin r2 = bc[2] - (diag * X(2, 0, 0, 0) - off2) * cf.ih2;
      if constexpr (UPD) {
        const size_t o = static_cast<size_t>(p) * P + oown;
        __builtin_nontemporal_store(X(0, 0, 0, 0), x_out + o);
        __builtin_nontemporal_store(X(1, 0, 0, 0), x_out + C + o);
        __builtin_nontemporal_store(X(2, 0, 0, 0), x_out + 2 * C + o);
      }
#undef X
      sq += static_cast<double>(r0) * r0 + static_cast<double>(r1) * r1 + static_cast<double>(r2) * r2;
      if (r) {
        const size_t o = static_cast<size_t>(p) * P + oown;
        __builtin_nontemporal_store(static_cast<Tout>(r0 * out_scale), r + o);
        __builtin_nontemporal_store(static_cast<Tout>(r1 * out_scale), r + C + o);
        __builtin_nontemporal_store(static_cast<Tout>(r2 * out_scale), r + 2 * C + o);
      }
    }
#pragma unroll
    for (int c = 0; c < 3; ++c) bc[c] = bn[c];
    __syncthreads();
  }
  if (partial) {
#pragma unroll
    for (int off = 32; off > 0; off >>= 1) sq += __shfl_down(sq, off, 64);
    if ((threadIdx.x & 63) == 0) red[threadIdx.x >> 6] = sq;
    __syncthreads();
    if (threadIdx.x == 0) partial[L] = red[0] + red[1] + red[2] + red[3];
  }
}

ZmArgs zm_args(Dims d) {
  ZmArgs a;
  a.nx = d.nx;
  a.ny = d.ny;
  a.nz = d.nz;
  a.ntx = (d.nx + TX - 1) / TX;
  a.nty = (d.ny + TY - 1) / TY;
  a.nseg = (d.nz - 1 + SEGZ - 1) / SEGZ;
  a.real_wgs = a.ntx * a.nty * a.nseg;
  a.grid_per_xcd = (a.real_wgs + 7) / 8;
  return a;
}

// Fused fine residual and restriction, b_c = R (b - K x) with R = T^T: the
// residual never leaves the chip.  A workgroup owns a 64 x 8 fine tile, i.e.
// the 32 x 4 coarse nodes at its even positions, over a segment of coarse
// planes, and marches up the fine planes 2 K0 - 1 .. 2 K1 - 1.  Per fine plane
// it computes the residual on the 65 x 9 patch those coarse nodes read (one
// extra column and row below the tile), from x staged in a 3-plane LDS ring
// with a 67 x 11 footprint, reduces the patch in x and y for each coarse node
// and adds the result, weighted for the plane's z offset, to the coarse
// node's running sum, which is written when its third plane is done.  Both the
// residual and the weighted sums are evaluated in the same order as the
// separate residual and restriction kernels, so the result is identical.
constexpr int FX = 64, FY = 8;                      // fine tile
constexpr int RXN = FX + 1, RYN = FY + 1, RN = RXN * RYN;  // residual patch
constexpr int XXN = FX + 3, XYN = FY + 3, XN = XXN * XYN;  // x patch
constexpr int CSEG = 16;                            // coarse planes per segment

struct RrArgs {
  int nx, ny, nz;
  int ntx, nty, nseg;
  int real_wgs, grid_per_xcd;
};

template <typename T>
__global__ __launch_bounds__(256) void k_resid_restrict(const T* __restrict__ x,
                                                        const T* __restrict__ b,
                                                        T* __restrict__ bc, T* __restrict__ xc,
                                                        RrArgs a, FineCoef<T> cf) {
  __shared__ T ring[3 * 3 * XN];  // [plane % 3][component][XYN][XXN]
  __shared__ T rp[3 * RN];        // residual of the current plane [component][RYN][RXN]
  const int wg = blockIdx.x;
  const int L = (wg & 7) * a.grid_per_xcd + (wg >> 3);
  if (L >= a.real_wgs) return;
  const int tx = L % a.ntx;
  const int rest = L / a.ntx;
  const int ty = rest % a.nty;
  const int sg = rest / a.nty;
  const int nx = a.nx, ny = a.ny, nz = a.nz;
  const int nxc = nx / 2, nyc = ny / 2, nzc = nz / 2;
  const int i0 = tx * FX, j0 = ty * FY;
  const int K0 = 1 + sg * CSEG, K1 = min(K0 + CSEG, nzc);  // coarse planes [K0, K1)
  const size_t P = static_cast<size_t>(nx) * ny, C = static_cast<size_t>(nz + 1) * P;
  const int tid = threadIdx.x;

  // x patch element e -> offset within a plane (columns i0-2.., rows j0-2..)
  size_t hoff[3];
#pragma unroll
  for (int u = 0; u < 3; ++u) {
    const int e = min(tid + u * 256, XN - 1);
    const int hy = e / XXN, hx = e - hy * XXN;
    const int gj = (j0 - 2 + hy + 2 * ny) % ny, gi = (i0 - 2 + hx + 2 * nx) % nx;
    hoff[u] = static_cast<size_t>(gj) * nx + gi;
  }
  // residual patch node e -> plane offset and position in the x patch
  size_t roff[3];
  int rpos[3];
#pragma unroll
  for (int u = 0; u < 3; ++u) {
    const int e = min(tid + u * 256, RN - 1);
    const int ry = e / RXN, rx = e - ry * RXN;
    const int gj = (j0 - 1 + ry + ny) % ny, gi = (i0 - 1 + rx + nx) % nx;
    roff[u] = static_cast<size_t>(gj) * nx + gi;
    rpos[u] = (ry + 1) * XXN + rx + 1;
  }
  T pre[3][3];
  auto fetch = [&](int p) {
#pragma unroll
    for (int u = 0; u < 3; ++u)
      if (tid + u * 256 < XN)
#pragma unroll
        for (int c = 0; c < 3; ++c) pre[u][c] = x[c * C + static_cast<size_t>(p) * P + hoff[u]];
  };
  auto store = [&](int p) {
#pragma unroll
    for (int u = 0; u < 3; ++u) {
      const int e = tid + u * 256;
      if (e < XN)
#pragma unroll
        for (int c = 0; c < 3; ++c) ring[((p % 3) * 3 + c) * XN + e] = pre[u][c];
    }
  };
  T bcur[3][3], bnext[3][3];
  auto fetch_b = [&](int p, T out[3][3]) {
#pragma unroll
    for (int u = 0; u < 3; ++u)
      if (tid + u * 256 < RN)
#pragma unroll
        for (int c = 0; c < 3; ++c)
          out[u][c] = __builtin_nontemporal_load(b + c * C + static_cast<size_t>(p) * P + roff[u]);
  };

  const int kf0 = 2 * K0 - 1, kf1 = 2 * K1 - 1;  // fine planes of the march
  fetch(kf0 - 1);
  store(kf0 - 1);
  fetch(kf0);
  store(kf0);
  fetch_b(kf0, bcur);
  fetch(kf0 + 1);
  // drain the prologue loads (memory counters complete in order; a wait for
  // them placed inside the loop would also wait for each prefetch)
  __builtin_amdgcn_s_waitcnt(0);
  const T diag = T(2) * (cf.p + T(2) * cf.q);
  // coarse node of this thread (threads < 128) and its running sums
  const int Il = tid & 31, Jl = tid >> 5;
  const int I = i0 / 2 + Il, J = j0 / 2 + Jl;
  const bool cown = tid < 128 && I < nxc && J < nyc;
  T acc[3] = {T(0), T(0), T(0)};
  for (int kf = kf0; kf <= kf1; ++kf) {
    store(kf + 1);
    __syncthreads();
    if (kf + 1 <= kf1) fetch_b(kf + 1, bnext);
    if (kf + 2 <= nz) fetch(kf + 2);
    // residual on the patch
#pragma unroll
    for (int u = 0; u < 3; ++u) {
      const int e = tid + u * 256;
      if (e < RN) {
        const int pc = kf % 3, pm = (kf + 2) % 3, pp = (kf + 1) % 3;
        const int q = rpos[u];
#define X(c, pl, dy, dx) ring[((pl) * 3 + (c)) * XN + q + (dy) * XXN + (dx)]
        const T fx0 = X(0, pc, 0, 1) + X(0, pc, 0, -1), fy0 = X(0, pc, 1, 0) + X(0, pc, -1, 0),
                fz0 = X(0, pp, 0, 0) + X(0, pm, 0, 0);
        const T fx1 = X(1, pc, 0, 1) + X(1, pc, 0, -1), fy1 = X(1, pc, 1, 0) + X(1, pc, -1, 0),
                fz1 = X(1, pp, 0, 0) + X(1, pm, 0, 0);
        const T fx2 = X(2, pc, 0, 1) + X(2, pc, 0, -1), fy2 = X(2, pc, 1, 0) + X(2, pc, -1, 0),
                fz2 = X(2, pp, 0, 0) + X(2, pm, 0, 0);
        // mixed differences f(+,+) - f(+,-) - f(-,+) + f(-,-)
        const T mxy0 = X(0, pc, 1, 1) - X(0, pc, -1, 1) - X(0, pc, 1, -1) + X(0, pc, -1, -1);
        const T mxy1 = X(1, pc, 1, 1) - X(1, pc, -1, 1) - X(1, pc, 1, -1) + X(1, pc, -1, -1);
        const T mxz0 = X(0, pp, 0, 1) - X(0, pm, 0, 1) - X(0, pp, 0, -1) + X(0, pm, 0, -1);
        const T mxz2 = X(2, pp, 0, 1) - X(2, pm, 0, 1) - X(2, pp, 0, -1) + X(2, pm, 0, -1);
        const T myz1 = X(1, pp, 1, 0) - X(1, pm, 1, 0) - X(1, pp, -1, 0) + X(1, pm, -1, 0);
        const T myz2 = X(2, pp, 1, 0) - X(2, pm, 1, 0) - X(2, pp, -1, 0) + X(2, pm, -1, 0);
        const T off0 = cf.p * fx0 + cf.q * (fy0 + fz0) + cf.m4 * (mxy1 + mxz2);
        const T off1 = cf.p * fy1 + cf.q * (fx1 + fz1) + cf.m4 * (mxy0 + myz2);
        const T off2 = cf.p * fz2 + cf.q * (fx2 + fy2) + cf.m4 * (mxz0 + myz1);
        rp[e] = bcur[u][0] - (diag * X(0, pc, 0, 0) - off0) * cf.ih2;
        rp[RN + e] = bcur[u][1] - (diag * X(1, pc, 0, 0) - off1) * cf.ih2;
        rp[2 * RN + e] = bcur[u][2] - (diag * X(2, pc, 0, 0) - off2) * cf.ih2;
#undef X
      }
    }
    __syncthreads();
    if (cown) {
      // x-y reduction around fine (2 Il, 2 Jl) of the tile = patch (2 Il + 1, 2 Jl + 1)
      const T w[3] = {T(0.5), T(1), T(0.5)};
      const bool odd = kf & 1;
      const int Kdone = (kf - 1) / 2;  // coarse plane completed by an odd fine plane
      const size_t ob = static_cast<size_t>(J) * nxc + I;
      const size_t Pc = static_cast<size_t>(nxc) * nyc, Cc = static_cast<size_t>(nzc + 1) * Pc;
#pragma unroll
      for (int c = 0; c < 3; ++c) {
        T az = T(0);
#pragma unroll
        for (int dy = 0; dy < 3; ++dy) {
          const T* row = rp + c * RN + (2 * Jl + dy) * RXN + 2 * Il;
          const T ax = T(0.5) * row[0] + row[1] + T(0.5) * row[2];
          az += w[dy] * ax;
        }
        if (odd) {
          if (kf > kf0) {
            acc[c] += w[2] * az;
            bc[c * Cc + static_cast<size_t>(Kdone) * Pc + ob] = acc[c];
            if (xc) xc[c * Cc + static_cast<size_t>(Kdone) * Pc + ob] = T(0);
          }
          acc[c] = T(0) + w[0] * az;
        } else {
          acc[c] += w[1] * az;
        }
      }
    }
#pragma unroll
    for (int u = 0; u < 3; ++u)
#pragma unroll
      for (int c = 0; c < 3; ++c) bcur[u][c] = bnext[u][c];
  }
}

RrArgs rr_args(Dims d) {
  RrArgs a;
  a.nx = d.nx;
  a.ny = d.ny;
  a.nz = d.nz;
  a.ntx = (d.nx + FX - 1) / FX;
  a.nty = (d.ny + FY - 1) / FY;
  a.nseg = (d.nz / 2 - 1 + CSEG - 1) / CSEG;
  a.real_wgs = a.ntx * a.nty * a.nseg;
  a.grid_per_xcd = (a.real_wgs + 7) / 8;
  return a;
}

}  // namespace

int resid_zmarch_blocks(Dims d) { return zm_args(d).real_wgs; }

template <typename Tin, typename Tout>
int launch_residual_fine_zm(const Tin* x, const Tin* b, Tout* r, Dims d, const FineCoef<double>& c,
                            double out_scale, double* partial, hipStream_t s) {
  FineCoef<Tin> cf;
  cf.h2 = static_cast<Tin>(c.h2);
  cf.p = static_cast<Tin>(c.p);
  cf.q = static_cast<Tin>(c.q);
  cf.m4 = static_cast<Tin>(c.m4);
  cf.inv_diag = static_cast<Tin>(c.inv_diag);
  cf.ih2 = static_cast<Tin>(c.ih2);
  const ZmArgs a = zm_args(d);
  hipLaunchKernelGGL((k_residual_zm<Tin, Tout, false>), dim3(8 * a.grid_per_xcd), dim3(256), 0, s,
                     x, b, r, a, cf, static_cast<Tin>(out_scale), partial, nullptr, 0.0, nullptr);
  return a.real_wgs;
}

int launch_update_residual_zm(const double* x, const float* e, double es, double* x_out,
                              const double* b, float* r, Dims d, const FineCoef<double>& c,
                              double out_scale, double* partial, hipStream_t s) {
  const ZmArgs a = zm_args(d);
  hipLaunchKernelGGL((k_residual_zm<double, float, true>), dim3(8 * a.grid_per_xcd), dim3(256), 0,
                     s, x, b, r, a, c, out_scale, partial, e, es, x_out);
  return a.real_wgs;
}

template <typename T>
void launch_resid_restrict(const T* x, const T* b, T* bc, T* xc, Dims d,
                           const FineCoef<double>& c, hipStream_t s) {
  if (d.nz / 2 - 1 <= 0) return;
  FineCoef<T> cf;
  cf.h2 = static_cast<T>(c.h2);
  cf.p = static_cast<T>(c.p);
  cf.q = static_cast<T>(c.q);
  cf.m4 = static_cast<T>(c.m4);
  cf.inv_diag = static_cast<T>(c.inv_diag);
  cf.ih2 = static_cast<T>(c.ih2);
  const RrArgs a = rr_args(d);
  hipLaunchKernelGGL((k_resid_restrict<T>), dim3(8 * a.grid_per_xcd), dim3(256), 0, s, x, b, bc, xc,
                     a, cf);
}

template void launch_resid_restrict<double>(const double*, const double*, double*, double*, Dims,
                                            const FineCoef<double>&, hipStream_t);
template void launch_resid_restrict<float>(const float*, const float*, float*, float*, Dims,
                                           const FineCoef<double>&, hipStream_t);
template int launch_residual_fine_zm<double, double>(const double*, const double*, double*, Dims,
                                                     const FineCoef<double>&, double, double*,
                                                     hipStream_t);
template int launch_residual_fine_zm<double, float>(const double*, const double*, float*, Dims,
                                                    const FineCoef<double>&, double, double*,
                                                    hipStream_t);
template int launch_residual_fine_zm<float, float>(const float*, const float*, float*, Dims,
                                                   const FineCoef<double>&, double, double*,
                                                   hipStream_t);

}  // namespace qs
