// C ABI of libqsmg: handle, workspace layout, V-cycle drivers and the solve
// loops (paper Sec. 3.6), plus the projection step of Sec. 3.3.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <cstdint>
#include <cstdio>
#include <cstring>
#include <mutex>
#include <new>
#include <vector>

#include "device.h"
#include "hierarchy.h"
#include "packed_stencil.h"
#include "qsmg.h"

using namespace qs;

namespace {

constexpr int kMaxLevels = 16;

struct LevelBufs {
  Dims d{0, 0, 0};
  double* x64 = nullptr;
  double* b64 = nullptr;
  double* r64 = nullptr;
  float* x32 = nullptr;
  float* b32 = nullptr;
  float* r32 = nullptr;
  double* y64 = nullptr;  // second smoother buffer (ping-pong), smoothed levels
  double* xalt64 = nullptr;  // FP32-IR, fine level: the other buffer of the FP64 iterate
  float* y32 = nullptr;
  int seg64 = 16, seg32 = 16;  // z planes per workgroup of the row sweep (fine level)
  double* S64 = nullptr;
  double* D64 = nullptr;
  float* S32 = nullptr;
  float* D32 = nullptr;
  double* P64 = nullptr;  // packed plane stencils (packed_stencil.h)
  float* P32 = nullptr;
};

// Assigns aligned sub-buffers of the workspace; with base == nullptr it only
// measures.
struct Carver {
  char* base;
  size_t off = 0;
  template <typename T>
  T* take(size_t n) {
    off = (off + 255) & ~static_cast<size_t>(255);
    T* p = base ? reinterpret_cast<T*>(base + off) : nullptr;
    off += n * sizeof(T);
    return p;
  }
};

bool valid_params(const qs_params* p) {
  if (!p) return false;
  if (p->precision != QS_FP64 && p->precision != QS_FP32_IR) return false;
  if (p->n_pre < 0 || p->n_post < 0 || p->n_pre > 16 || p->n_post > 16) return false;
  if (!(p->h > 0.0) || !(p->mu > 0.0) || !(p->lambda + p->mu > 0.0)) return false;
  int seen = 0;
  for (int q = 0; q < 8; ++q) {
    const int c = p->colour_order[q];
    if (c < 0 || c > 7 || (seen >> c) & 1) return false;
    seen |= 1 << c;
  }
  return true;
}

int plan(const qs_params* p, std::vector<int>* dims) {
  if (plan_levels(p->nx, p->ny, p->nz, p->min_coarse_nz, dims) != 0) return -2;
  // 32-bit element indexing inside the kernels: node vectors and cell tensors
  const long long nodes = 3LL * (p->nz + 1) * p->ny * p->nx;
  const long long cells = 6LL * p->nz * p->ny * p->nx;
  if (nodes >= (1LL << 31) || cells >= (1LL << 31) ||
      static_cast<int>(dims->size() / 3) > kMaxLevels)
    return -2;
  return 0;
}

}  // namespace

struct qs_handle {
  qs_params p;
  hipStream_t stream = nullptr;
  int nlev = 0;
  LevelBufs L[kMaxLevels];
  FineCoef<double> fc64;
  FineCoef<float> fc32;
  double* Ainv = nullptr;
  int ncoarse = 0;
  double* partial = nullptr;
  int partial_n = 0;
  double* dnorm = nullptr;   // device, 4 doubles
  double* pinned = nullptr;      // host pinned, 4 doubles
  double* pinned_dev = nullptr;  // the same memory as the device addresses it (null: copy instead)
  bool row_sweep = false;    // colour order allows the row-parity sweep kernel
  size_t lds_limit = 0;      // bytes of LDS a workgroup may use
  void* static_scratch = nullptr;  // device address of `scratch` on this handle's device (or null)
};

namespace {

void carve(const qs_params* p, const std::vector<int>& dims, char* base, qs_handle* hd,
           size_t* total) {
  Carver cv{base};
  const int nlev = static_cast<int>(dims.size() / 3);
  int maxblocks = 1;
  for (int l = 0; l < nlev; ++l) {
    LevelBufs lb;
    lb.d = Dims{dims[3 * l], dims[3 * l + 1], dims[3 * l + 2]};
    const size_t e = lb.d.elems();
    if (p->precision == QS_FP64) {
      if (l > 0) {
        lb.x64 = cv.take<double>(e);
        lb.b64 = cv.take<double>(e);
      }
      lb.r64 = cv.take<double>(e);
      if (l < nlev - 1) lb.y64 = cv.take<double>(e);
    } else {
      if (l == 0) lb.xalt64 = cv.take<double>(e);
      lb.x32 = cv.take<float>(e);
      lb.b32 = cv.take<float>(e);
      if (l < nlev - 1) {
        lb.r32 = cv.take<float>(e);
        lb.y32 = cv.take<float>(e);
      }
    }
    const size_t planes = static_cast<size_t>(lb.d.nz + 1);
    lb.S64 = cv.take<double>(planes * kStencil);
    lb.D64 = cv.take<double>(planes * 9);
    lb.S32 = cv.take<float>(planes * kStencil);
    lb.D32 = cv.take<float>(planes * 9);
    lb.P64 = cv.take<double>(planes * kPackedStencil);
    lb.P32 = cv.take<float>(planes * kPackedStencil);
    const int nb = residual_blocks(lb.d);
    if (nb > maxblocks) maxblocks = nb;
    if (hd) hd->L[l] = lb;
  }
  const Dims g{dims[3 * (nlev - 1)], dims[3 * (nlev - 1) + 1], dims[3 * (nlev - 1) + 2]};
  const int nc = 3 * g.nx * g.ny * (g.nz - 1);
  double* Ainv = cv.take<double>(static_cast<size_t>(nc) * nc);
  double* partial = cv.take<double>(maxblocks);
  double* dnorm = cv.take<double>(4);
  if (hd) {
    hd->nlev = nlev;
    hd->ncoarse = nc;
    hd->Ainv = Ainv;
    hd->partial = partial;
    hd->partial_n = maxblocks;
    hd->dnorm = dnorm;
  }
  *total = (cv.off + 255) & ~static_cast<size_t>(255);
}

thread_local char g_last_error[256] = "";

qs_status hip_fail(const char* what, hipError_t e) {
  std::snprintf(g_last_error, sizeof(g_last_error), "%s: %s", what, hipGetErrorString(e));
  return QS_ERR_HIP;
}

void set_error(const char* what) { std::snprintf(g_last_error, sizeof(g_last_error), "%s", what); }

#define QS_HIP(call)                                   \
  do {                                                 \
    const hipError_t e_ = (call);                      \
    if (e_ != hipSuccess) return hip_fail(#call, e_);  \
  } while (0)

qs_status launch_check() {
  const hipError_t e = hipGetLastError();
  return e == hipSuccess ? QS_OK : hip_fail("kernel launch", e);
}

// Read the reduced double written to hd->dnorm[0] (and, when the pinned
// buffer is device-addressable, by the reduction kernel straight into it).
// The host polls the stream rather than sleeping in a synchronisation, so the
// next cycle is enqueued as soon as the norm is there.
qs_status read_norm(qs_handle* hd, double* out) {
  QS_HIP(hipGetLastError());
  if (!hd->pinned_dev)
    QS_HIP(hipMemcpyAsync(hd->pinned, hd->dnorm, sizeof(double), hipMemcpyDeviceToHost, hd->stream));
  hipError_t q;
  while ((q = hipStreamQuery(hd->stream)) == hipErrorNotReady) {
  }
  QS_HIP(q);
  *out = static_cast<volatile double*>(hd->pinned)[0];
  return QS_OK;
}

// ---- level operations in working precision T ----------------------------
template <typename T>
struct Prec;
template <>
struct Prec<double> {
  static double* x(LevelBufs& l) { return l.x64; }
  static double* b(LevelBufs& l) { return l.b64; }
  static double* r(LevelBufs& l) { return l.r64; }
  static double* y(LevelBufs& l) { return l.y64; }
  static const double* S(LevelBufs& l) { return l.S64; }
  static const double* D(LevelBufs& l) { return l.D64; }
  static const double* Pk(LevelBufs& l) { return l.P64; }
  static const FineCoef<double>& fc(qs_handle* hd) { return hd->fc64; }
  static int seg(const LevelBufs& l) { return l.seg64; }
};
template <>
struct Prec<float> {
  static float* x(LevelBufs& l) { return l.x32; }
  static float* b(LevelBufs& l) { return l.b32; }
  static float* r(LevelBufs& l) { return l.r32; }
  static float* y(LevelBufs& l) { return l.y32; }
  static const float* S(LevelBufs& l) { return l.S32; }
  static const float* D(LevelBufs& l) { return l.D32; }
  static const float* Pk(LevelBufs& l) { return l.P32; }
  static const FineCoef<float>& fc(qs_handle* hd) { return hd->fc32; }
  static int seg(const LevelBufs& l) { return l.seg32; }
};

template <typename T>
void colour_pass(qs_handle* hd, int l, T* x, const T* b, int colour) {
  LevelBufs& lb = hd->L[l];
  if (l == 0)
    launch_colour_fine<T>(x, b, lb.d, colour, Prec<T>::fc(hd), hd->stream);
  else
    launch_colour_gen<T>(x, b, lb.d, colour, Prec<T>::S(lb), Prec<T>::D(lb), hd->stream);
}

// Kernels that move column pairs as one two-wide access need 16-byte aligned
// node vectors (every device allocation is; an offset view may not be).
static bool aligned16(const void* p) { return (reinterpret_cast<uintptr_t>(p) & 15) == 0; }

template <typename T>
void residual(qs_handle* hd, int l, const T* x, const T* b, T* r, bool zero_interior) {
  LevelBufs& lb = hd->L[l];
  if (l == 0 && !zero_interior)
    launch_residual_fine_zm<T, T>(x, b, r, lb.d, hd->fc64, 1.0, nullptr, hd->stream);
  else if (l == 0)
    launch_residual_fine<T, T>(x, b, r, lb.d, hd->fc64, 1.0, zero_interior, nullptr, hd->stream);
  else if ((sizeof(T) == 8 || pair_rows_in_lanes(lb.d)) && !zero_interior && lb.d.nx % 2 == 0 &&
           aligned16(x) && aligned16(b) && aligned16(r))
    // two nodes per thread; in FP32 only where a row's pairs fit the lanes of
    // one wavefront and the outer window columns come by lane shuffles
    // (128^3: 25 against 35 us for one node per thread, which stays faster
    // when the outer columns are loaded)
    launch_residual_pair_gen<T>(x, b, r, lb.d, Prec<T>::Pk(lb), hd->stream);
  else
    launch_residual_gen<T>(x, b, r, lb.d, Prec<T>::Pk(lb), zero_interior, nullptr, hd->stream);
}

// Coarsest level: x_interior = A^{-1} (b - A_IB x_B).  Only the FP64 fine
// level carries wall data; coarse levels and the FP32 correction equation
// have zero walls, and b is used directly.
template <typename T>
void coarse_solve(qs_handle* hd, int l, T* x, const T* b, T* tmp) {
  LevelBufs& lb = hd->L[l];
  const T* rhs = b;
  if (l == 0 && sizeof(T) == sizeof(double)) {
    residual<T>(hd, l, x, b, tmp, true);
    rhs = tmp;
  }
  launch_coarse_solve<T>(hd->Ainv, hd->ncoarse, rhs, x, lb.d, hd->stream);
}

// Copy the two wall planes of x into y (both buffers must carry them).
template <typename T>
void copy_walls(const T* x, T* y, Dims d, hipStream_t s) {
  const size_t P = static_cast<size_t>(d.plane());
  for (int c = 0; c < 3; ++c) {
    const size_t o0 = static_cast<size_t>(c) * d.comp();
    const size_t o1 = o0 + static_cast<size_t>(d.nz) * P;
    (void)hipMemcpyAsync(y + o0, x + o0, P * sizeof(T), hipMemcpyDeviceToDevice, s);
    (void)hipMemcpyAsync(y + o1, x + o1, P * sizeof(T), hipMemcpyDeviceToDevice, s);
  }
}

template <typename T>
void zero_walls(T* y, Dims d, hipStream_t s) {
  const size_t P = static_cast<size_t>(d.plane());
  for (int c = 0; c < 3; ++c) {
    launch_fill<T>(y + static_cast<size_t>(c) * d.comp(), P, T(0), s);
    launch_fill<T>(y + static_cast<size_t>(c) * d.comp() + static_cast<size_t>(d.nz) * P, P, T(0), s);
  }
}

template <typename T>
bool use_row_sweep(qs_handle* hd, int l) {
  // the row sweep pays off on the fine level; coarse levels are small enough
  // that one launch per colour (data in L2/MALL) is faster
  return l == 0 && hd->row_sweep && sweep_supported(hd->L[l].d, hd->lds_limit, sizeof(T));
}

// `sweeps` Gauss-Seidel sweeps on level l, in the colour order given at
// setup (forward) or its reverse.  The row-parity kernel ping-pongs between
// x and the level's second buffer; an odd sweep count ends with a copy back.
// x_zero: the interior of x is known to be zero (its walls are zero too), so
// the first forward sweep does not read it; the sweep writes every interior
// node of the other buffer, so x need not even hold zeros then.
// prolong: the coarse correction of level l + 1 (reverse sweeps on a level
// with the row sweep only): the first sweep adds x += T prolong on the fly
// instead of a separate prolongation.
template <typename T>
void smooth(qs_handle* hd, int l, T* x, const T* b, int sweeps, bool reverse,
            bool x_zero = false, const T* prolong = nullptr) {
  if (sweeps <= 0) return;
  LevelBufs& lb = hd->L[l];
  const int* ord = hd->p.colour_order;
  if (!use_row_sweep<T>(hd, l)) {
    // on the coarse levels, consecutive colours that differ only in the x
    // parity share one launch
    const bool pairs = l > 0 && colour_pair_supported(lb.d);
    for (int s = 0; s < sweeps; ++s)
      for (int q = 0; q < 8; ++q) {
        const int c = ord[reverse ? 7 - q : q];
        if (pairs && q % 2 == 0 && ord[reverse ? 6 - q : q + 1] == (c ^ 1)) {
          launch_colour_pair_gen<T>(x, b, lb.d, c, Prec<T>::Pk(lb), hd->stream);
          ++q;
          continue;
        }
        colour_pass<T>(hd, l, x, b, c);
      }
    return;
  }
  // y's wall planes are zero from setup (coarse levels, FP32 corrections) or
  // hold the Dirichlet data copied once per solve (FP64 fine level)
  T* y = Prec<T>::y(lb);
  const FineCoef<T>& cf = Prec<T>::fc(hd);
  T* cur = x;
  T* oth = y;
  const int rp0 = reverse ? 1 : 0, pf = reverse ? 1 : 0, xf = reverse ? 1 : 0;
  for (int s = 0; s < sweeps; ++s) {
    const bool z = x_zero && s == 0 && !reverse;
    const bool pro = prolong && s == 0 && reverse;
    const T* ec = pro ? prolong : nullptr;
    launch_sweep_half<T>(cur, cur, oth, b, ec, lb.d, rp0, pf, xf, cf, Prec<T>::seg(lb), 1,
                         z ? 2 : (pro ? 3 : 0), hd->stream);
    launch_sweep_half<T>(cur, oth, oth, b, ec, lb.d, 1 - rp0, pf, xf, cf, Prec<T>::seg(lb), 1,
                         z ? 1 : (pro ? 4 : 0), hd->stream);
    T* t = cur;
    cur = oth;
    oth = t;
  }
  if (cur != x)
    (void)hipMemcpyAsync(x, cur, lb.d.elems() * sizeof(T), hipMemcpyDeviceToDevice, hd->stream);
}

// x_zero: x is zero on entry and need not hold it (see smooth; only when the
// row sweep smooths level l and n_pre >= 1)
template <typename T>
void vcycle(qs_handle* hd, int l, T* x, const T* b, bool x_zero = false) {
  LevelBufs& lb = hd->L[l];
  if (l == hd->nlev - 1) {
    coarse_solve<T>(hd, l, x, b, Prec<T>::r(lb));
    return;
  }
  smooth<T>(hd, l, x, b, hd->p.n_pre, false, x_zero);
  LevelBufs& cb = hd->L[l + 1];
  // the restriction also clears the interior of the coarse correction (its
  // walls are zero from setup and never written)
  if (l == 0) {
    launch_resid_restrict<T>(x, b, Prec<T>::b(cb), Prec<T>::x(cb), lb.d, hd->fc64, hd->stream);
  } else {
    T* r = Prec<T>::r(lb);
    residual<T>(hd, l, x, b, r, false);
    launch_restrict<T>(r, Prec<T>::b(cb), Prec<T>::x(cb), lb.d, hd->stream);
  }
  vcycle<T>(hd, l + 1, Prec<T>::x(cb), Prec<T>::b(cb));
  if (hd->p.n_post >= 1 && use_row_sweep<T>(hd, l)) {
    // the first post-smoothing sweep applies the prolongated correction
    smooth<T>(hd, l, x, b, hd->p.n_post, true, false, Prec<T>::x(cb));
    return;
  }
  launch_prolong_add<T>(x, Prec<T>::x(cb), lb.d, hd->stream);
  smooth<T>(hd, l, x, b, hd->p.n_post, true);
}

// ||b - K x||^2 on level 0 in FP64 (optionally writing the residual, scaled,
// in FP32 for the refinement loop); result in hd->dnorm[0].
template <typename Tout>
int residual_norm0(qs_handle* hd, const double* x, const double* b, Tout* r, double scale,
                   bool zero_interior) {
  const int nb =
      zero_interior
          ? launch_residual_fine<double, Tout>(x, b, r, hd->L[0].d, hd->fc64, scale, true,
                                               hd->partial, hd->stream)
          : launch_residual_fine_zm<double, Tout>(x, b, r, hd->L[0].d, hd->fc64, scale,
                                                  hd->partial, hd->stream);
  launch_reduce_sum(hd->partial, nb, hd->dnorm, hd->pinned_dev, hd->stream);
  return nb;
}

double pow2_near(double v) {
  if (!(v > 0.0) || !std::isfinite(v)) return 1.0;
  return std::ldexp(1.0, static_cast<int>(std::lround(std::log2(v))));
}

// Step scratch for callers that cannot allocate (qs_projection_step_noalloc):
// a fixed device array of QS_NOALLOC_SCRATCH_BYTES that every GPU the library
// runs on holds until the process ends.  Host code never passes `scratch`
// itself to a kernel or copy (on the host it is only a stand-in for the
// symbol); it uses the device address resolved per device at setup.
static __device__ __align__(256) unsigned char scratch[QS_NOALLOC_SCRATCH_BYTES];

constexpr int kMaxDevices = 64;
std::mutex g_scratch_mutex;
void* g_scratch_addr[kMaxDevices] = {};
bool g_scratch_tried[kMaxDevices] = {};

// Device address of `scratch` on the current device, resolved once per
// device (null, with the reason in the last-error text, if that failed).
void* static_scratch_address() {
  int dev = -1;
  if (hipGetDevice(&dev) != hipSuccess || dev < 0 || dev >= kMaxDevices) {
    (void)hipGetLastError();
    return nullptr;
  }
  std::lock_guard<std::mutex> lock(g_scratch_mutex);
  if (!g_scratch_tried[dev]) {
    g_scratch_tried[dev] = true;
    void* ptr = nullptr;
    const hipError_t e = hipGetSymbolAddress(&ptr, HIP_SYMBOL(scratch));
    if (e == hipSuccess && ptr) {
      g_scratch_addr[dev] = ptr;
    } else {
      (void)hipGetLastError();
      std::snprintf(g_last_error, sizeof(g_last_error), "hipGetSymbolAddress(scratch): %s",
                    hipGetErrorString(e));
    }
  }
  return g_scratch_addr[dev];
}

}  // namespace

extern "C" {

const char* qs_last_error(void) { return g_last_error; }

const char* qs_status_string(int s) {
  switch (s) {
    case QS_OK: return "ok";
    case QS_ERR_ARG: return "invalid argument";
    case QS_ERR_SHAPE: return "grid shape not supported";
    case QS_ERR_HIP: return "HIP runtime error";
    case QS_ERR_NOT_CONVERGED: return "not converged";
    case QS_ERR_NONFINITE: return "non-finite residual";
    case QS_ERR_WORKSPACE: return "workspace missing, misaligned or too small";
    default: return "unknown status";
  }
}

qs_status qs_workspace_bytes(const qs_params* p, size_t* bytes) {
  if (!valid_params(p) || !bytes) return QS_ERR_ARG;
  std::vector<int> dims;
  if (plan(p, &dims) != 0) return QS_ERR_SHAPE;
  carve(p, dims, nullptr, nullptr, bytes);
  return QS_OK;
}

qs_status qs_level_dims(const qs_params* p, int level, int* nlev, int* nx, int* ny, int* nz) {
  if (!valid_params(p)) return QS_ERR_ARG;
  std::vector<int> dims;
  if (plan(p, &dims) != 0) return QS_ERR_SHAPE;
  const int n = static_cast<int>(dims.size() / 3);
  if (nlev) *nlev = n;
  if (level < 0 || level >= n) return QS_ERR_ARG;
  if (nx) *nx = dims[3 * level];
  if (ny) *ny = dims[3 * level + 1];
  if (nz) *nz = dims[3 * level + 2];
  return QS_OK;
}

qs_status qs_setup(const qs_params* p, void* workspace, size_t workspace_bytes, void* stream,
                   qs_handle** out) {
  if (!valid_params(p) || !out) return QS_ERR_ARG;
  *out = nullptr;
  std::vector<int> dims;
  if (plan(p, &dims) != 0) return QS_ERR_SHAPE;
  size_t need = 0;
  carve(p, dims, nullptr, nullptr, &need);
  if (!workspace || (reinterpret_cast<uintptr_t>(workspace) & 255) || workspace_bytes < need)
    return QS_ERR_WORKSPACE;
  HostHierarchy H;
  if (build_hierarchy(p->nx, p->ny, p->nz, p->h, p->lambda, p->mu, p->min_coarse_nz, &H) != 0)
    return QS_ERR_SHAPE;
  qs_handle* hd = new (std::nothrow) qs_handle();
  if (!hd) return QS_ERR_ARG;
  hd->p = *p;
  hd->stream = static_cast<hipStream_t>(stream);
  hd->static_scratch = static_scratch_address();
  carve(p, dims, static_cast<char*>(workspace), hd, &need);
  {
    const hipError_t e = hipHostMalloc(reinterpret_cast<void**>(&hd->pinned), 4 * sizeof(double));
    if (e != hipSuccess) {
      delete hd;
      return hip_fail("hipHostMalloc", e);
    }
    void* dp = nullptr;
    if (hipHostGetDevicePointer(&dp, hd->pinned, 0) == hipSuccess && dp)
      hd->pinned_dev = static_cast<double*>(dp);
    else
      (void)hipGetLastError();  // fall back to a copy per norm
  }
  const double lam = p->lambda, mu = p->mu, h = p->h;
  {
    static const int kRowOrder[8] = {0, 1, 4, 5, 2, 3, 6, 7};
    hd->row_sweep = std::memcmp(p->colour_order, kRowOrder, sizeof(kRowOrder)) == 0;
    int dev = 0, lds = 65536;
    if (hipGetDevice(&dev) == hipSuccess &&
        hipDeviceGetAttribute(&lds, hipDeviceAttributeMaxSharedMemoryPerBlock, dev) == hipSuccess &&
        lds > 0)
      hd->lds_limit = static_cast<size_t>(lds);
    else
      hd->lds_limit = 65536;
    sweep_set_lds_limit(hd->lds_limit);
  }
  hd->fc64.h2 = h * h;
  hd->fc64.p = lam + 2.0 * mu;
  hd->fc64.q = mu;
  hd->fc64.m4 = 0.25 * (lam + mu);
  hd->fc64.inv_diag = 1.0 / (2.0 * (lam + 4.0 * mu));
  hd->fc64.ih2 = 1.0 / (h * h);
  hd->fc32.h2 = static_cast<float>(hd->fc64.h2);
  hd->fc32.p = static_cast<float>(hd->fc64.p);
  hd->fc32.q = static_cast<float>(hd->fc64.q);
  hd->fc32.m4 = static_cast<float>(hd->fc64.m4);
  hd->fc32.inv_diag = static_cast<float>(hd->fc64.inv_diag);
  hd->fc32.ih2 = static_cast<float>(hd->fc64.ih2);
  for (int l = 0; l < hd->nlev; ++l) {
    LevelBufs& lb = hd->L[l];
    if (l == 0 && sweep_supported(lb.d, hd->lds_limit, 4)) {
      lb.seg32 = sweep_segment_length(lb.d, 4);
      if (sweep_supported(lb.d, hd->lds_limit, 8)) lb.seg64 = sweep_segment_length(lb.d, 8);
    }
    if (lb.y64) launch_fill<double>(lb.y64, lb.d.elems(), 0.0, hd->stream);
    if (lb.y32) launch_fill<float>(lb.y32, lb.d.elems(), 0.0f, hd->stream);
    // the FP32 correction of the fine level and the coarse-level corrections:
    // walls stay zero for good (the refinement loop may skip clearing the
    // fine interior, see solve_impl; the restriction clears coarse interiors)
    if (l == 0 && lb.x32) launch_fill<float>(lb.x32, lb.d.elems(), 0.0f, hd->stream);
    if (l > 0 && lb.x32) launch_fill<float>(lb.x32, lb.d.elems(), 0.0f, hd->stream);
    if (l > 0 && lb.x64) launch_fill<double>(lb.x64, lb.d.elems(), 0.0, hd->stream);
  }
  // upload stencils (FP64 and their FP32 roundings) and the coarse inverse;
  // the staging vectors live until the synchronisation below
  std::vector<std::vector<float>> stage32;
  std::vector<std::vector<double>> stage64;
  stage32.reserve(3 * hd->nlev);
  stage64.reserve(hd->nlev);
  qs_status st = QS_OK;
  for (int l = 0; l < hd->nlev && st == QS_OK; ++l) {
    const HostLevel& hl = H.levels[l];
    LevelBufs& lb = hd->L[l];
    stage32.emplace_back(hl.stencil.begin(), hl.stencil.end());
    const std::vector<float>& s32 = stage32.back();
    stage32.emplace_back(hl.dinv.begin(), hl.dinv.end());
    const std::vector<float>& d32 = stage32.back();
    stage64.emplace_back();
    if (!pack_level(hl, &stage64.back())) {
      set_error("setup: a stencil entry that vanishes by symmetry is not negligible");
      st = QS_ERR_ARG;
      break;
    }
    const std::vector<double>& p64 = stage64.back();
    stage32.emplace_back(p64.begin(), p64.end());
    const std::vector<float>& p32 = stage32.back();
    hipError_t e = hipMemcpyAsync(lb.S64, hl.stencil.data(), hl.stencil.size() * 8,
                                  hipMemcpyHostToDevice, hd->stream);
    if (e == hipSuccess)
      e = hipMemcpyAsync(lb.D64, hl.dinv.data(), hl.dinv.size() * 8, hipMemcpyHostToDevice,
                         hd->stream);
    if (e == hipSuccess)
      e = hipMemcpyAsync(lb.S32, s32.data(), s32.size() * 4, hipMemcpyHostToDevice, hd->stream);
    if (e == hipSuccess)
      e = hipMemcpyAsync(lb.D32, d32.data(), d32.size() * 4, hipMemcpyHostToDevice, hd->stream);
    if (e == hipSuccess)
      e = hipMemcpyAsync(lb.P64, p64.data(), p64.size() * 8, hipMemcpyHostToDevice, hd->stream);
    if (e == hipSuccess)
      e = hipMemcpyAsync(lb.P32, p32.data(), p32.size() * 4, hipMemcpyHostToDevice, hd->stream);
    if (e != hipSuccess) st = hip_fail("hipMemcpyAsync (stencil upload)", e);
  }
  if (st == QS_OK) {
    const hipError_t e = hipMemcpyAsync(hd->Ainv, H.coarse_inv.data(), H.coarse_inv.size() * 8,
                                        hipMemcpyHostToDevice, hd->stream);
    if (e != hipSuccess) st = hip_fail("hipMemcpyAsync (coarse inverse)", e);
  }
  {
    const hipError_t e = hipStreamSynchronize(hd->stream);
    if (e != hipSuccess) st = hip_fail("hipStreamSynchronize (setup)", e);
  }
  if (st != QS_OK) {
    (void)hipHostFree(hd->pinned);
    delete hd;
    return st;
  }
  *out = hd;
  return QS_OK;
}

qs_status qs_destroy(qs_handle* hd) {
  if (!hd) return QS_ERR_ARG;
  if (hd->pinned) (void)hipHostFree(hd->pinned);
  delete hd;
  return QS_OK;
}

qs_status qs_apply(qs_handle* hd, const double* x, double* y) {
  if (!hd || !x || !y || x == y) return QS_ERR_ARG;
  const Dims d = hd->L[0].d;
  // y = -(0 - K x) on the interior, walls zeroed
  launch_residual_fine_zm<double, double>(x, nullptr, y, d, hd->fc64, -1.0, nullptr, hd->stream);
  for (int c = 0; c < 3; ++c) {
    launch_fill<double>(y + static_cast<size_t>(c) * d.comp(), d.plane(), 0.0, hd->stream);
    launch_fill<double>(y + static_cast<size_t>(c) * d.comp() + static_cast<size_t>(d.nz) * d.plane(),
                        d.plane(), 0.0, hd->stream);
  }
  return launch_check();
}

static qs_status solve_impl(qs_handle* hd, const double* b, double* x, double rtol, int max_cycles,
                            qs_solve_info* info) {
  const Dims d0 = hd->L[0].d;
  const double nunk = 3.0 * d0.nx * d0.ny * (d0.nz - 1);
  qs_solve_info local;
  qs_solve_info* inf = info ? info : &local;
  std::memset(inf, 0, sizeof(*inf));
  inf->levels = hd->nlev;
  double nb2 = 0.0;
  residual_norm0<double>(hd, x, b, nullptr, 1.0, true);
  qs_status st = read_norm(hd, &nb2);
  if (st != QS_OK) return st;
  if (!std::isfinite(nb2)) return QS_ERR_NONFINITE;
  if (nb2 == 0.0) {
    launch_zero_interior<double>(x, d0, hd->stream);
    inf->rel_res = 0.0;
    inf->rel_res_hist[0] = 0.0;
    return launch_check();
  }
  const bool fixed = !(rtol > 0.0);
  const bool ir = hd->p.precision == QS_FP32_IR;
  if (!ir && hd->L[0].y64) copy_walls<double>(x, hd->L[0].y64, d0, hd->stream);
  // FP32-IR: the update x += s e of one cycle is made by the next residual
  // kernel, out of place, so the iterate alternates between x and xalt64
  // (whose wall planes take the Dirichlet data once per solve)
  LevelBufs& l0 = hd->L[0];
  double* xs = x;
  if (ir) copy_walls<double>(x, l0.xalt64, d0, hd->stream);
  bool pending = false;  // a correction in l0.x32 not yet added to xs
  double e_scale = 0.0;
  auto finish = [&](qs_status st) {
    if (xs != x)
      (void)hipMemcpyAsync(x, xs, d0.elems() * sizeof(double), hipMemcpyDeviceToDevice,
                           hd->stream);
    return st;
  };
  double scale = pow2_near(std::sqrt(nb2 / nunk));
  double scale_used = scale;
  int cycles = 0;
  double rel = 0.0;
  // FP32-IR: each refinement step runs up to kMaxInner FP32 V-cycles on the
  // scaled residual before the next FP64 residual, fewer when the contraction
  // per V-cycle seen in the previous step says fewer reach rtol.
  constexpr int kMaxInner = 6;
  double rel_prev = 0.0;
  int inner_prev = 0;
  for (;;) {
    const bool need_norm = !fixed || cycles == max_cycles;
    if (ir) {
      // FP64 residual, written as FP32 scaled by 1/scale for the inner cycle
      scale_used = scale;
      if (pending) {
        double* xn = xs == x ? l0.xalt64 : x;
        const int nb = launch_update_residual_zm(xs, l0.x32, e_scale, xn, b, l0.b32, d0, hd->fc64,
                                                 1.0 / scale_used, hd->partial, hd->stream);
        launch_reduce_sum(hd->partial, nb, hd->dnorm, hd->pinned_dev, hd->stream);
        xs = xn;
        pending = false;
      } else {
        residual_norm0<float>(hd, xs, b, l0.b32, 1.0 / scale_used, false);
      }
    } else if (need_norm) {
      residual_norm0<double>(hd, x, b, nullptr, 1.0, false);
    }
    if (need_norm) {
      double rn2 = 0.0;
      st = read_norm(hd, &rn2);
      if (st != QS_OK) return finish(st);
      rel_prev = cycles > 0 ? rel : 0.0;
      rel = std::sqrt(rn2 / nb2);
      if (cycles < QS_HIST) inf->rel_res_hist[cycles] = rel;
      inf->rel_res = rel;
      if (!std::isfinite(rel)) {
        inf->cycles = cycles;
        return finish(QS_ERR_NONFINITE);
      }
      if (!fixed && rel <= rtol) break;
      if (ir) scale = pow2_near(std::sqrt(rn2 / nunk));
    }
    if (cycles >= max_cycles) {
      inf->cycles = cycles;
      return finish(fixed ? QS_OK : QS_ERR_NOT_CONVERGED);
    }
    if (ir) {
      // correction e solves A e = r / scale_used in FP32; x += scale_used e
      // is made by the next residual
      int inner = std::min(kMaxInner, max_cycles - cycles);
      if (!fixed && inner_prev > 0 && rel_prev > 0.0) {
        const double rho = std::pow(rel / rel_prev, 1.0 / inner_prev);
        if (rho > 0.0 && rho < 1.0) {
          const double need = std::ceil(std::log(rtol / rel) / std::log(rho));
          if (need < inner) inner = std::max(1, static_cast<int>(need));
        }
      }
      const bool skip_fill = hd->p.n_pre >= 1 && hd->nlev > 1 && use_row_sweep<float>(hd, 0);
      if (!skip_fill) launch_fill<float>(l0.x32, l0.d.elems(), 0.0f, hd->stream);
      vcycle<float>(hd, 0, l0.x32, l0.b32, skip_fill);
      for (int v = 1; v < inner; ++v) vcycle<float>(hd, 0, l0.x32, l0.b32);
      pending = true;
      e_scale = scale_used;
      for (int v = 1; v < inner && cycles + v < QS_HIST; ++v)
        inf->rel_res_hist[cycles + v] = std::nan("");  // no FP64 residual after this V-cycle
      cycles += inner;
      inner_prev = inner;
    } else {
      vcycle<double>(hd, 0, x, b);
      ++cycles;
    }
  }
  inf->cycles = cycles;
  return finish(launch_check());
}

qs_status qs_mg_solve(qs_handle* hd, const double* b, double* x, double rtol, int max_cycles,
                      qs_solve_info* info) {
  if (!hd || !b || !x || max_cycles < 0 || b == x || !aligned16(b) || !aligned16(x))
    return QS_ERR_ARG;
  return solve_impl(hd, b, x, rtol, max_cycles, info);
}

}  // extern "C"

// ---------------------------------------------------------------------------
// STZ step, projection step and their reverse-mode pieces (Secs. 3.1, 3.3)
// ---------------------------------------------------------------------------
namespace {

bool valid_stz(const qs_stz_params* sp) {
  return sp && sp->tau0 > 0.0 && sp->s_y > 0.0 && sp->c0 > 0.0 && std::isfinite(sp->dt) &&
         sp->l_diff >= 0.0 && std::isfinite(sp->l_diff) && sp->n_sub >= -2 &&
         (sp->advect == 0 || sp->advect == 1) && (sp->chi_wall == 0 || sp->chi_wall == 1);
}

// Scratch for D^pl per cell during an STZ step: a fine-level FP64 buffer of
// the hierarchy that holds nothing between solves (the residual of an FP64
// handle, the second iterate buffer of an FP32-IR one; each solve rewrites
// them before reading), nx*ny*3*(nz+1) >= nx*ny*nz doubles.
double* stz_dcell(qs_handle* hd) {
  return hd->p.precision == QS_FP64 ? hd->L[0].r64 : hd->L[0].xalt64;
}

StzArgs stz_args(qs_handle* hd, const qs_stz_params* sp) {
  StzArgs a;
  a.s_y = sp->s_y;
  a.tau0 = sp->tau0;
  a.beta = sp->beta;
  a.delta_over_T = sp->delta_over_T;
  a.c0 = sp->c0;
  a.chi_inf = sp->chi_inf;
  a.dt = sp->dt;
  a.lam = hd->p.lambda;
  a.mu = hd->p.mu;
  a.h = hd->p.h;
  a.l2 = sp->l_diff * sp->l_diff;
  a.n_sub = sp->n_sub <= 1 && sp->n_sub >= 0 ? 1 : sp->n_sub;
  a.advect = sp->advect;
  a.chi_wall = sp->chi_wall;
  return a;
}

size_t cells(const Dims& d) { return static_cast<size_t>(d.nx) * d.ny * d.nz; }

size_t step_scratch(qs_handle* hd) {
  const Dims d = hd->L[0].d;
  const size_t a = (7 * cells(d) + d.elems()) * sizeof(double) + 512;
  const size_t b = 9 * cells(d) * sizeof(double) + 256;
  return a > b ? a : b;
}

}  // namespace

extern "C" {

qs_status qs_stz_step(qs_handle* hd, const qs_stz_params* sp, const double* v, const double* sigma,
                      const double* chi, double* sigma_star, double* chi_next) {
  if (!hd || !valid_stz(sp) || !v || !sigma || !chi || !sigma_star || !chi_next) return QS_ERR_ARG;
  if (sigma_star == sigma || chi_next == chi) return QS_ERR_ARG;
  if ((sp->l_diff > 0.0 || sp->advect) && hd->L[0].d.nz < 2) return QS_ERR_SHAPE;  // ghost layers need two cells
  launch_stz_step(v, sigma, chi, sigma_star, chi_next, stz_dcell(hd), hd->L[0].d, stz_args(hd, sp),
                  hd->stream);
  return launch_check();
}

qs_status qs_rhs(qs_handle* hd, const double* sigma_star, double dt, double* b) {
  if (!hd || !sigma_star || !b || !(dt != 0.0)) return QS_ERR_ARG;
  launch_rhs(sigma_star, b, hd->L[0].d, hd->p.h, dt, hd->stream);
  return launch_check();
}

qs_status qs_stress_update(qs_handle* hd, const double* sigma_star, const double* v, double dt,
                           double* sigma_out) {
  if (!hd || !sigma_star || !v || !sigma_out) return QS_ERR_ARG;
  launch_stress_update(sigma_star, v, sigma_out, hd->L[0].d, hd->p.h, dt, hd->p.lambda, hd->p.mu,
                       hd->stream);
  return launch_check();
}

qs_status qs_step_scratch_bytes(qs_handle* hd, size_t* bytes) {
  if (!hd || !bytes) return QS_ERR_ARG;
  *bytes = step_scratch(hd);
  return QS_OK;
}

namespace {

// One projection step; the new wall planes of v are (-U,0,0) / (+U,0,0) when
// lo is null, else copied from lo and hi.
qs_status projection_step_impl(qs_handle* hd, const qs_stz_params* sp, double U_wall,
                               const double* lo, const double* hi, double* v, double* sigma,
                               double* chi, void* step_buf, double rtol, int max_cycles,
                               qs_solve_info* info) {
  if (!hd || !valid_stz(sp) || !v || !sigma || !chi || !step_buf || max_cycles < 0 ||
      !aligned16(v))
    return QS_ERR_ARG;
  if (reinterpret_cast<uintptr_t>(step_buf) & 255) return QS_ERR_WORKSPACE;
  const Dims d = hd->L[0].d;
  if ((sp->l_diff > 0.0 || sp->advect) && d.nz < 2) return QS_ERR_SHAPE;
  // every piece is written in full before it is read (sigma*, chi' by the STZ
  // step, b with its wall planes by the RHS), so nothing needs clearing
  Carver cv{static_cast<char*>(step_buf)};
  double* sstar = cv.take<double>(6 * cells(d));
  double* chi1 = cv.take<double>(cells(d));
  double* b = cv.take<double>(d.elems());
  const StzArgs a = stz_args(hd, sp);
  launch_stz_step(v, sigma, chi, sstar, chi1, stz_dcell(hd), d, a, hd->stream);
  if (lo)
    launch_copy_walls(v, lo, hi, d, hd->stream);
  else
    launch_set_walls(v, d, U_wall, hd->stream);
  launch_rhs(sstar, b, d, hd->p.h, sp->dt, hd->stream);
  qs_status st = launch_check();
  if (st != QS_OK) return st;
  st = solve_impl(hd, b, v, rtol, max_cycles, info);
  if (st != QS_OK && st != QS_ERR_NOT_CONVERGED) return st;
  launch_stress_update(sstar, v, sigma, d, hd->p.h, sp->dt, hd->p.lambda, hd->p.mu, hd->stream);
  QS_HIP(hipMemcpyAsync(chi, chi1, cells(d) * sizeof(double), hipMemcpyDeviceToDevice, hd->stream));
  const qs_status lc = launch_check();
  return lc != QS_OK ? lc : st;
}

}  // namespace

qs_status qs_projection_step(qs_handle* hd, const qs_stz_params* sp, double U_wall, double* v,
                             double* sigma, double* chi, void* step_buf, double rtol,
                             int max_cycles, qs_solve_info* info) {
  return projection_step_impl(hd, sp, U_wall, nullptr, nullptr, v, sigma, chi, step_buf, rtol,
                              max_cycles, info);
}

qs_status qs_projection_step_noalloc(qs_handle* hd, const qs_stz_params* sp, double U_wall,
                                     double* v, double* sigma, double* chi, double rtol,
                                     int max_cycles, qs_solve_info* info) {
  if (!hd) return QS_ERR_ARG;
  const size_t need = step_scratch(hd);
  if (need > QS_NOALLOC_SCRATCH_BYTES) {
    std::snprintf(g_last_error, sizeof(g_last_error),
                  "qs_projection_step_noalloc: the grid needs %zu bytes of step scratch, the "
                  "static buffer holds %zu",
                  need, static_cast<size_t>(QS_NOALLOC_SCRATCH_BYTES));
    return QS_ERR_SHAPE;
  }
  if (!hd->static_scratch) return QS_ERR_HIP;  // symbol address not resolved at setup
  return projection_step_impl(hd, sp, U_wall, nullptr, nullptr, v, sigma, chi,
                              hd->static_scratch, rtol, max_cycles, info);
}

qs_status qs_projection_step_walls(qs_handle* hd, const qs_stz_params* sp, const double* wall_lo,
                                   const double* wall_hi, double* v, double* sigma, double* chi,
                                   void* step_buf, double rtol, int max_cycles,
                                   qs_solve_info* info) {
  if (!wall_lo || !wall_hi) return QS_ERR_ARG;
  if (hd) {
    // the wall data must not overlap v, whose wall planes are written from it
    const Dims d = hd->L[0].d;
    const char* v0 = reinterpret_cast<const char*>(v);
    const char* v1 = v0 + d.elems() * sizeof(double);
    const size_t wb = 3 * static_cast<size_t>(d.plane()) * sizeof(double);
    for (const double* w : {wall_lo, wall_hi}) {
      const char* w0 = reinterpret_cast<const char*>(w);
      if (v && w0 < v1 && w0 + wb > v0) return QS_ERR_ARG;
    }
  }
  return projection_step_impl(hd, sp, 0.0, wall_lo, wall_hi, v, sigma, chi, step_buf, rtol,
                              max_cycles, info);
}

qs_status qs_explicit_step(qs_handle* hd, const qs_stz_params* sp, double U_wall, double rho,
                           double kappa, double* v, double* sigma, double* chi, void* step_buf) {
  if (!hd || !valid_stz(sp) || !v || !sigma || !chi || !step_buf || !(rho > 0.0) ||
      !std::isfinite(rho) || !(kappa >= 0.0) || !std::isfinite(kappa) || !std::isfinite(U_wall))
    return QS_ERR_ARG;
  if (reinterpret_cast<uintptr_t>(step_buf) & 255) return QS_ERR_WORKSPACE;
  const Dims d = hd->L[0].d;
  if (d.nz < 2) return QS_ERR_SHAPE;
  Carver cv{static_cast<char*>(step_buf)};
  double* sstar = cv.take<double>(6 * cells(d));
  double* chi1 = cv.take<double>(cells(d));
  double* vnew = cv.take<double>(d.elems());
  StzArgs a = stz_args(hd, sp);
  a.advect = 1;  // the stress equation of the explicit method carries the advection
  launch_stz_step(v, sigma, chi, sstar, chi1, stz_dcell(hd), d, a, hd->stream);
  launch_explicit_velocity(v, sigma, vnew, d, hd->p.h, sp->dt, rho, kappa, hd->stream);
  launch_set_walls(vnew, d, U_wall, hd->stream);
  launch_stress_update(sstar, v, sigma, d, hd->p.h, sp->dt, hd->p.lambda, hd->p.mu, hd->stream);
  QS_HIP(hipMemcpyAsync(v, vnew, d.elems() * sizeof(double), hipMemcpyDeviceToDevice, hd->stream));
  QS_HIP(hipMemcpyAsync(chi, chi1, cells(d) * sizeof(double), hipMemcpyDeviceToDevice, hd->stream));
  return launch_check();
}

qs_status qs_stz_step_vjp(qs_handle* hd, const qs_stz_params* sp, const double* v,
                          const double* sigma, const double* chi, const double* g_sstar,
                          const double* g_chi1, double* g_sigma, double* g_chi, double* g_v,
                          void* step_buf) {
  if (!hd || !valid_stz(sp) || !v || !sigma || !chi || !g_sstar || !g_chi1 || !g_sigma || !g_chi ||
      !g_v || !step_buf || sp->l_diff != 0.0 || sp->n_sub > 1 || sp->n_sub < 0 || sp->advect)
    return QS_ERR_ARG;
  const Dims d = hd->L[0].d;
  // the velocity-gradient cotangent is stored as [9][cells] with 32-bit indices
  if (9LL * cells(d) >= (1LL << 31)) return QS_ERR_SHAPE;
  double* gL = static_cast<double*>(step_buf);
  const StzArgs a = stz_args(hd, sp);
  launch_stz_step_vjp(v, sigma, chi, g_sstar, g_chi1, g_sigma, g_chi, gL, d, a, hd->stream);
  launch_grad_transpose_add(gL, g_v, d, hd->p.h, 1.0, hd->stream);
  return launch_check();
}

qs_status qs_rhs_vjp(qs_handle* hd, const double* g_b, double dt, double* g_sstar) {
  if (!hd || !g_b || !g_sstar || !(dt != 0.0)) return QS_ERR_ARG;
  launch_rhs_vjp(g_b, g_sstar, hd->L[0].d, hd->p.h, dt, hd->stream);
  return launch_check();
}

qs_status qs_stress_update_vjp(qs_handle* hd, const double* g_sigma, double dt, double* g_v) {
  if (!hd || !g_sigma || !g_v) return QS_ERR_ARG;
  launch_stress_update_vjp(g_sigma, g_v, hd->L[0].d, hd->p.h, dt, hd->p.lambda, hd->p.mu,
                           hd->stream);
  return launch_check();
}

// ---- test-facing level pieces (FP64 handles) ------------------------------

qs_status qs_level_colour_pass(qs_handle* hd, int level, double* x, const double* b, int colour) {
  if (!hd || hd->p.precision != QS_FP64 || level < 0 || level >= hd->nlev - 1 || !x || !b ||
      colour < 0 || colour > 7)
    return QS_ERR_ARG;
  colour_pass<double>(hd, level, x, b, colour);
  return launch_check();
}

qs_status qs_level_residual(qs_handle* hd, int level, const double* x, const double* b, double* r) {
  if (!hd || hd->p.precision != QS_FP64 || level < 0 || level >= hd->nlev || !x || !b || !r)
    return QS_ERR_ARG;
  residual<double>(hd, level, x, b, r, false);
  return launch_check();
}

qs_status qs_level_restrict(qs_handle* hd, int level, const double* r, double* b_coarse) {
  if (!hd || level < 0 || level >= hd->nlev - 1 || !r || !b_coarse || !aligned16(r))
    return QS_ERR_ARG;
  launch_restrict<double>(r, b_coarse, nullptr, hd->L[level].d, hd->stream);
  return launch_check();
}

qs_status qs_level_prolong_add(qs_handle* hd, int level, double* x, const double* e_coarse) {
  if (!hd || level < 0 || level >= hd->nlev - 1 || !x || !e_coarse || !aligned16(x))
    return QS_ERR_ARG;
  launch_prolong_add<double>(x, e_coarse, hd->L[level].d, hd->stream);
  return launch_check();
}

qs_status qs_coarse_solve(qs_handle* hd, double* x, const double* b) {
  if (!hd || hd->p.precision != QS_FP64 || !x || !b) return QS_ERR_ARG;
  const int l = hd->nlev - 1;
  LevelBufs& lb = hd->L[l];
  residual<double>(hd, l, x, b, lb.r64, true);
  launch_coarse_solve<double>(hd->Ainv, hd->ncoarse, lb.r64, x, lb.d, hd->stream);
  return launch_check();
}

qs_status qs_smooth(qs_handle* hd, int level, void* x, const void* b, int sweeps) {
  if (!hd || level < 0 || level >= hd->nlev - 1 || !x || !b || sweeps < 0 || !aligned16(x) ||
      !aligned16(b))
    return QS_ERR_ARG;
  // x may carry any wall data here; the second buffer takes a copy for this
  // call and gets zero walls back afterwards where the solver relies on them
  // (coarse levels and FP32 corrections).
  LevelBufs& lb = hd->L[level];
  if (hd->p.precision == QS_FP32_IR) {
    float* xf = static_cast<float*>(x);
    if (lb.y32) copy_walls<float>(xf, lb.y32, lb.d, hd->stream);
    smooth<float>(hd, level, xf, static_cast<const float*>(b), sweeps, false);
    if (lb.y32) zero_walls<float>(lb.y32, lb.d, hd->stream);
  } else {
    double* xd = static_cast<double*>(x);
    if (lb.y64) copy_walls<double>(xd, lb.y64, lb.d, hd->stream);
    smooth<double>(hd, level, xd, static_cast<const double*>(b), sweeps, false);
    if (lb.y64 && level > 0) zero_walls<double>(lb.y64, lb.d, hd->stream);
  }
  return launch_check();
}

qs_status qs_level_stencil(qs_handle* hd, int level, double* out_host) {
  if (!hd || level < 0 || level >= hd->nlev || !out_host) return QS_ERR_ARG;
  const LevelBufs& lb = hd->L[level];
  const size_t n = static_cast<size_t>(lb.d.nz + 1) * kStencil;
  QS_HIP(hipMemcpyAsync(out_host, lb.S64, n * sizeof(double), hipMemcpyDeviceToHost, hd->stream));
  QS_HIP(hipStreamSynchronize(hd->stream));
  return QS_OK;
}

}  // extern "C"
