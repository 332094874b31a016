// cs3d.hip - host runtime and C ABI of the compact-stencil direct solver.
//
// A plan owns small device tables only: the row weights of Sections 3.2-3.5,
// the samples of k^2 and (k^2)_z used by the RHS operator, the modal cosines of
// Section 3.6 and the line-transform tables.  Data and workspace belong to the
// caller.  Every solve is four kernel launches (kernels.hpp) on the caller's
// stream, plus a tiny statistics reset.
#include <hip/hip_runtime.h>

#include <cmath>
#include <cstdint>
#include <cstring>
#include <new>
#include <vector>

#include "../../include/cs3d.h"
#include "kernels.hpp"

using namespace cs3d;

namespace {

constexpr int kMaxN = 1023;
constexpr int kRing = 16;       // solves kept for the per-pass timing average
constexpr int kMaxMarks = 64;   // timed intervals per solve
constexpr int kStages = 6;      // stage ids: RHS, x-DST, y fwd, y back, inverse x, residual
// relative FP64 residual a mixed solve must reach after its refinement steps
constexpr double kResidualTarget = 1e-12;

bool is_pow2(int v) { return v > 0 && (v & (v - 1)) == 0; }

// FFT line length for N interior points (0 = dense sine sums)
int fft_len(int n) {
  const int m = n + 1;
  return (is_pow2(m) && m >= 64 && m <= 1024) ? m : 0;
}

template <typename P>
hipError_t dalloc(P** p, size_t count) {
  return hipMalloc(reinterpret_cast<void**>(p), count * sizeof(P));
}

}  // namespace

struct cs3d_plan_s {
  cs3d_desc d{};
  int Mx = 0, My = 0, fx = 0, fy = 0, ldy = 0;
  double* dW = nullptr;
  double* dLC = nullptr;
  double* dk2 = nullptr;
  double* dk2z = nullptr;
  double* dctx = nullptr;
  double* dcty = nullptr;
  double2* dtwx = nullptr;
  double2* dtwy = nullptr;
  double* dsinx = nullptr;
  double* dsiny = nullptr;
  unsigned long long* dstats = nullptr;
  void* ws = nullptr;
  size_t ws_bytes = 0;
  hipStream_t last_stream = nullptr;
  hipEvent_t ev0 = nullptr, ev1 = nullptr;
  bool timed = false;
  // per-pass timing ring: kRing solves x (kMaxMarks + 1) events; interval k of a solve
  // belongs to stage ring_sid[...]
  std::vector<hipEvent_t> ring;
  std::vector<signed char> ring_sid;
  std::vector<int> ring_n;
  long long solves = 0;   // solves recorded since the last reset
  int cur_marks = 0;
  int refine_done = 0;
  std::vector<double> hW;  // host copy of the weights
};

// ---------------------------------------------------------------------------
// Row weights, Sections 3.2 - 3.5.  W[l][o][(a,b,c,d)], o = 0,1,2 for offsets -1,0,+1.
// ---------------------------------------------------------------------------
static cs3d_status build_weights(const cs3d_desc& d, std::vector<double>& W) {
  const int nz = d.nz;
  W.assign((size_t)nz * 12, 0.0);
  const double rzx = d.hz * d.hz / (d.hx * d.hx), rzy = d.hz * d.hz / (d.hy * d.hy);
  const double hz2 = d.hz * d.hz;
  auto at = [&](int l, int o, int q) -> double& { return W[(size_t)l * 12 + o * 4 + q]; };
  for (int l = 0; l < nz; ++l) {
    const int zl = l + 1;  // sample index of plane z_l
    switch (d.scheme) {
      case CS3D_HELM2: {
        const double k0 = d.k2[zl];
        at(l, 0, 3) = 1.0;
        at(l, 2, 3) = 1.0;
        at(l, 1, 1) = rzx;
        at(l, 1, 2) = rzy;
        at(l, 1, 3) = -2.0 * (rzx + rzy + 1.0) + hz2 * k0;
        break;
      }
      case CS3D_HELM4: {
        const double km = d.k2[zl - 1], k0 = d.k2[zl], kp = d.k2[zl + 1];
        for (int o = 0; o <= 2; o += 2) {
          const double kk = o == 0 ? km : kp;
          at(l, o, 1) = (1.0 + rzx) / 12.0;
          at(l, o, 2) = (1.0 + rzy) / 12.0;
          at(l, o, 3) = 2.0 / 3.0 - (rzx + rzy) / 6.0 + hz2 * kk / 12.0;
        }
        at(l, 1, 0) = (rzx + rzy) / 12.0;
        at(l, 1, 1) = (4.0 * rzx - rzy - 1.0 + hz2 * k0 / 2.0) / 6.0;
        at(l, 1, 2) = (4.0 * rzy - rzx - 1.0 + hz2 * k0 / 2.0) / 6.0;
        at(l, 1, 3) = -4.0 * (1.0 + rzx + rzy) / 3.0 + hz2 * k0 / 2.0;
        break;
      }
      case CS3D_HELM6: {
        const double h = d.hz, h2 = h * h, h3 = h2 * h, h4 = h2 * h2;
        const double km = d.k2[zl - 1], k0 = d.k2[zl], kp = d.k2[zl + 1];
        const double kz = d.k2_z[zl], kzz = d.k2_zz[zl];
        for (int o = 0; o <= 2; o += 2) {
          const double sg = o == 0 ? -1.0 : 1.0, kk = o == 0 ? km : kp;
          at(l, o, 0) = 1.0 / 30.0;
          const double bc = 0.1 + h2 * kk / 90.0 + sg * h3 * kz / 120.0;
          at(l, o, 1) = bc;
          at(l, o, 2) = bc;
          at(l, o, 3) = 7.0 / 15.0 - h2 * kk / 90.0 + sg * (h3 * kz / 20.0) * (1.0 / 3.0 + h2 * kk / 6.0);
        }
        at(l, 1, 0) = 0.1 + h2 * k0 / 90.0;
        at(l, 1, 1) = 7.0 / 15.0 - h2 * k0 / 90.0;
        at(l, 1, 2) = 7.0 / 15.0 - h2 * k0 / 90.0;
        at(l, 1, 3) = -64.0 / 15.0 + 14.0 * h2 * k0 / 15.0 - h4 * k0 * k0 / 20.0 + h4 * kzz / 20.0;
        break;
      }
      case CS3D_CD4: {
        const double t = d.hz * d.gamma;
        for (int o = 0; o <= 2; o += 2) {
          const double sg = o == 0 ? -1.0 : 1.0;
          at(l, o, 1) = (1.0 + rzx) * (2.0 + sg * t) / 24.0;
          at(l, o, 2) = (1.0 + rzy) * (2.0 + sg * t) / 24.0;
          at(l, o, 3) = 2.0 / 3.0 - (rzx + rzy) / 6.0 + sg * (t / 12.0) * (4.0 - rzx - rzy + sg * t);
        }
        at(l, 1, 0) = (rzx + rzy) / 12.0;
        at(l, 1, 1) = (4.0 * rzx - rzy - 1.0) / 6.0;
        at(l, 1, 2) = (4.0 * rzy - rzx - 1.0) / 6.0;
        at(l, 1, 3) = -4.0 * (1.0 + rzx + rzy) / 3.0 - t * t / 6.0;
        break;
      }
      case CS3D_WEIGHTS:
        for (int q = 0; q < 12; ++q) W[(size_t)l * 12 + q] = d.weights[(size_t)l * 12 + q];
        break;
      default:
        return CS3D_E_INVAL;
    }
  }
  return CS3D_OK;
}

// exp(-i pi k/M), k < 2M; angles reduced exactly (k is an integer < 2M)
static void twiddles(int M, std::vector<double2>& tw) {
  tw.resize(2 * (size_t)M);
  for (int k = 0; k < 2 * M; ++k) {
    const long double a = 3.14159265358979323846264338327950288L * (long double)k / (long double)M;
    tw[k] = make_double2((double)cosl(a), (double)-sinl(a));
  }
}

static void sines(int M, std::vector<double>& s) {
  s.resize(2 * (size_t)M);
  for (int k = 0; k < 2 * M; ++k)
    s[k] = (double)sinl(3.14159265358979323846264338327950288L * (long double)k / (long double)M);
}

// s_k = 1 - cos(pi k/(n+1)) = 2 sin^2(pi k/(2(n+1))), k = 1..n, without cancellation
static void one_minus_cosines(int n, std::vector<double>& c) {
  c.resize(n);
  for (int k = 1; k <= n; ++k) {
    const long double sn = sinl(3.14159265358979323846264338327950288L * (long double)k / (2.0L * (n + 1)));
    c[k - 1] = (double)(2.0L * sn * sn);
  }
}

// Modal coefficients of Section 3.6 rewritten with s = 1 - cos:
//   4a cos_n cos_m + 2b cos_n + 2c cos_m + d
//     = (4a + 2b + 2c + d) - s_n (4a + 2b) + s_m (-(4a + 2c) + 4a s_n).
// Z = 4a + 2b + 2c + d is the row sum, small for a consistent Helmholtz row, so it is
// formed in extended precision from the FP64 weights; for low modes every term is then
// small and the FP64 evaluation keeps its relative accuracy even on strongly
// anisotropic grids, where the plain form cancels terms of size h_z^2/h_x^2.
static void modal_coefficients(const std::vector<double>& W, std::vector<double>& LC) {
  LC.resize(W.size());
  for (size_t r = 0; r < W.size() / 4; ++r) {
    const long double a = W[4 * r], b = W[4 * r + 1], c = W[4 * r + 2], d = W[4 * r + 3];
    LC[4 * r + 0] = (double)(4.0L * a + 2.0L * b + 2.0L * c + d);
    LC[4 * r + 1] = (double)(-(4.0L * a + 2.0L * b));
    LC[4 * r + 2] = (double)(-(4.0L * a + 2.0L * c));
    LC[4 * r + 3] = (double)(4.0L * a);
  }
}

static cs3d_status validate(const cs3d_desc* d) {
  if (!d) return CS3D_E_INVAL;
  if (d->nx < 1 || d->ny < 1 || d->nz < 1 || d->nx > kMaxN || d->ny > kMaxN) return CS3D_E_INVAL;
  if (!(d->hx > 0.0) || !(d->hy > 0.0) || !(d->hz > 0.0)) return CS3D_E_INVAL;
  if (!std::isfinite(d->hx) || !std::isfinite(d->hy) || !std::isfinite(d->hz)) return CS3D_E_INVAL;
  if (d->max_rhs < 1) return CS3D_E_INVAL;
  if (d->precision != CS3D_FP64 && d->precision != CS3D_MIXED_FP32) return CS3D_E_INVAL;
  if (d->refine_steps < 0 || d->refine_steps > 7) return CS3D_E_INVAL;
  switch (d->scheme) {
    case CS3D_HELM2:
    case CS3D_HELM4:
      if (!d->k2) return CS3D_E_INVAL;
      break;
    case CS3D_HELM6: {
      if (!d->k2 || !d->k2_z || !d->k2_zz) return CS3D_E_INVAL;
      const double tol = 1e-13 * d->hz;
      if (std::fabs(d->hx - d->hz) > tol || std::fabs(d->hy - d->hz) > tol) return CS3D_E_INVAL;
      if (d->nx < 4 || d->ny < 4 || d->nz < 4) return CS3D_E_INVAL;
      break;
    }
    case CS3D_CD4:
      if (!std::isfinite(d->gamma)) return CS3D_E_INVAL;
      break;
    case CS3D_WEIGHTS:
      if (!d->weights) return CS3D_E_INVAL;
      break;
    default:
      return CS3D_E_INVAL;
  }
  return CS3D_OK;
}

static void plan_free(cs3d_plan p) {
  if (!p) return;
  void* ptrs[] = {p->dW, p->dLC, p->dk2, p->dk2z, p->dctx, p->dcty, p->dtwx, p->dtwy, p->dsinx, p->dsiny, p->dstats};
  for (void* q : ptrs)
    if (q) (void)hipFree(q);
  for (hipEvent_t e : p->ring)
    if (e) (void)hipEventDestroy(e);
  if (p->ev0) (void)hipEventDestroy(p->ev0);
  if (p->ev1) (void)hipEventDestroy(p->ev1);
  delete p;
}

#define CS3D_TRY(expr)                   \
  do {                                   \
    if ((expr) != hipSuccess) {          \
      (void)hipGetLastError();           \
      plan_free(p);                      \
      return CS3D_E_DEVICE;              \
    }                                    \
  } while (0)

extern "C" cs3d_status cs3d_plan_create(const cs3d_desc* desc, void* hip_stream, cs3d_plan* out_plan) {
  if (!out_plan) return CS3D_E_INVAL;
  *out_plan = nullptr;
  cs3d_status st = validate(desc);
  if (st != CS3D_OK) return st;
  cs3d_plan p = new (std::nothrow) cs3d_plan_s();
  if (!p) return CS3D_E_NOMEM;
  p->d = *desc;
  p->d.k2 = p->d.k2_z = p->d.k2_zz = p->d.weights = nullptr;  // host arrays are not kept
  p->Mx = desc->nx + 1;
  p->My = desc->ny + 1;
  p->fx = fft_len(desc->nx);
  p->fy = fft_len(desc->ny);
  p->ldy = ((desc->ny + 1 + 15) / 16) * 16;
  st = build_weights(*desc, p->hW);
  if (st != CS3D_OK) {
    plan_free(p);
    return st;
  }
  hipStream_t s = (hipStream_t)hip_stream;
  const int nzp = desc->nz + 2;
  std::vector<double> k2(nzp, 0.0), k2z(nzp, 0.0);
  if (desc->k2)
    for (int i = 0; i < nzp; ++i) k2[i] = desc->k2[i];
  if (desc->k2_z)
    for (int i = 0; i < nzp; ++i) k2z[i] = desc->k2_z[i];
  std::vector<double> ctx, cty, sx, sy, lc;
  std::vector<double2> twx, twy;
  one_minus_cosines(desc->nx, ctx);
  one_minus_cosines(desc->ny, cty);
  modal_coefficients(p->hW, lc);
  twiddles(p->Mx, twx);
  twiddles(p->My, twy);
  sines(p->Mx, sx);
  sines(p->My, sy);
  CS3D_TRY(dalloc(&p->dW, p->hW.size()));
  CS3D_TRY(dalloc(&p->dLC, lc.size()));
  CS3D_TRY(dalloc(&p->dk2, k2.size()));
  CS3D_TRY(dalloc(&p->dk2z, k2z.size()));
  CS3D_TRY(dalloc(&p->dctx, ctx.size()));
  CS3D_TRY(dalloc(&p->dcty, cty.size()));
  CS3D_TRY(dalloc(&p->dtwx, twx.size()));
  CS3D_TRY(dalloc(&p->dtwy, twy.size()));
  CS3D_TRY(dalloc(&p->dsinx, sx.size()));
  CS3D_TRY(dalloc(&p->dsiny, sy.size()));
  CS3D_TRY(dalloc(&p->dstats, kStatsWords));
  CS3D_TRY(hipMemcpyAsync(p->dW, p->hW.data(), p->hW.size() * 8, hipMemcpyHostToDevice, s));
  CS3D_TRY(hipMemcpyAsync(p->dLC, lc.data(), lc.size() * 8, hipMemcpyHostToDevice, s));
  CS3D_TRY(hipMemcpyAsync(p->dk2, k2.data(), k2.size() * 8, hipMemcpyHostToDevice, s));
  CS3D_TRY(hipMemcpyAsync(p->dk2z, k2z.data(), k2z.size() * 8, hipMemcpyHostToDevice, s));
  CS3D_TRY(hipMemcpyAsync(p->dctx, ctx.data(), ctx.size() * 8, hipMemcpyHostToDevice, s));
  CS3D_TRY(hipMemcpyAsync(p->dcty, cty.data(), cty.size() * 8, hipMemcpyHostToDevice, s));
  CS3D_TRY(hipMemcpyAsync(p->dtwx, twx.data(), twx.size() * 16, hipMemcpyHostToDevice, s));
  CS3D_TRY(hipMemcpyAsync(p->dtwy, twy.data(), twy.size() * 16, hipMemcpyHostToDevice, s));
  CS3D_TRY(hipMemcpyAsync(p->dsinx, sx.data(), sx.size() * 8, hipMemcpyHostToDevice, s));
  CS3D_TRY(hipMemcpyAsync(p->dsiny, sy.data(), sy.size() * 8, hipMemcpyHostToDevice, s));
  CS3D_TRY(hipEventCreate(&p->ev0));
  CS3D_TRY(hipEventCreate(&p->ev1));
  p->ring.assign((size_t)kRing * (kMaxMarks + 1), nullptr);
  p->ring_sid.assign((size_t)kRing * kMaxMarks, 0);
  p->ring_n.assign(kRing, 0);
  for (hipEvent_t& e : p->ring) CS3D_TRY(hipEventCreate(&e));
  k_stats_reset<<<1, 64, 0, s>>>(p->dstats);
  CS3D_TRY(hipGetLastError());
  // the host vectors above go out of scope: wait for the copies
  CS3D_TRY(hipStreamSynchronize(s));
  *out_plan = p;
  return CS3D_OK;
}

#undef CS3D_TRY

extern "C" cs3d_status cs3d_plan_destroy(cs3d_plan plan) {
  if (!plan) return CS3D_OK;
  if (plan->last_stream) (void)hipStreamSynchronize(plan->last_stream);
  plan_free(plan);
  return CS3D_OK;
}

static size_t elem_bytes(const cs3d_plan p) { return p->d.precision == CS3D_FP64 ? 8 : 4; }

static size_t g_elems(const cs3d_plan p) { return (size_t)p->d.nz * p->d.nx * p->ldy; }

static size_t round256(size_t b) { return (b + 255) & ~(size_t)255; }

static size_t n3(const cs3d_plan p) { return (size_t)p->d.nx * p->d.ny * p->d.nz; }

// workspace layout: G (transform intermediate, per rhs) | C (c' of the LU, shared by the
// right-hand sides) | mixed path only: F (FP64 right-hand side, per rhs) | R (FP64 residual)
static size_t off_C(const cs3d_plan p, int nrhs) { return round256(g_elems(p) * elem_bytes(p) * (size_t)nrhs); }
static size_t off_F(const cs3d_plan p, int nrhs) { return off_C(p, nrhs) + round256(g_elems(p) * 8); }
static size_t off_R(const cs3d_plan p, int nrhs) { return off_F(p, nrhs) + round256(n3(p) * 8 * (size_t)nrhs); }

extern "C" size_t cs3d_workspace_bytes(cs3d_plan p, int nrhs) {
  if (!p || nrhs < 1 || nrhs > p->d.max_rhs) return 0;
  if (p->d.precision == CS3D_FP64) return off_F(p, nrhs);
  return off_R(p, nrhs) + round256(n3(p) * 8 * (size_t)nrhs);
}

extern "C" cs3d_status cs3d_set_workspace(cs3d_plan p, void* dev, size_t bytes) {
  if (!p || !dev) return CS3D_E_INVAL;
  if (((uintptr_t)dev & 255) != 0) return CS3D_E_INVAL;
  p->ws = dev;
  p->ws_bytes = bytes;
  return CS3D_OK;
}

// ---------------------------------------------------------------------------
// Launch helpers
// ---------------------------------------------------------------------------
template <typename T, int MX>
static size_t lds_bytes_x_t(const cs3d_plan p) {
  const size_t a = (size_t)kTileJ * line_buf_elems<T, MX>(p->d.nx) * sizeof(T);
  const size_t b = (size_t)kTileJ * tile_stride(p->d.nx) * sizeof(T);
  return (a > b ? a : b) + tw_bytes<T, MX>();
}

template <typename T, int MY>
static size_t lds_bytes_y_t(const cs3d_plan p) {
  return (size_t)YCfg<MY>::LPB * line_buf_elems<T, MY>(p->d.ny) * sizeof(T) + tw_bytes<T, MY>();
}

template <typename KernelT, typename... Args>
static hipError_t launch(KernelT kern, dim3 grid, dim3 block, size_t lds, hipStream_t s, Args... args) {
  if (lds > 160 * 1024) return hipErrorInvalidValue;
  if (lds > 64 * 1024) {
    hipError_t e = hipFuncSetAttribute(reinterpret_cast<const void*>(kern),
                                       hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds);
    if (e != hipSuccess) return e;
  }
  hipLaunchKernelGGL(kern, grid, block, lds, s, args...);
  return hipGetLastError();
}

// persistent x-pass grid: as many workgroups as fit on the device at once
template <typename KernelT>
static int resident_blocks(KernelT kern, int threads, size_t lds, int ntiles) {
  int dev = 0, per_cu = 0, cus = 256;
  if (hipGetDevice(&dev) == hipSuccess) {
    hipDeviceProp_t prop;
    if (hipGetDeviceProperties(&prop, dev) == hipSuccess) cus = prop.multiProcessorCount;
  }
  if (hipOccupancyMaxActiveBlocksPerMultiprocessor(&per_cu, reinterpret_cast<const void*>(kern), threads, lds) !=
          hipSuccess ||
      per_cu < 1)
    per_cu = 1;
  const long long b = (long long)per_cu * cus;
  return (int)(b < ntiles ? b : ntiles);
}

template <typename T, int MX>
static hipError_t run_x_fwd_t(const cs3d_plan p, const ProbDev& pd, int nrhs, hipStream_t s) {
  const int ntiles = (p->ldy / kTileJ) * p->d.nz * nrhs;
  const size_t lds = lds_bytes_x_t<T, MX>(p);
  if (lds > 64 * 1024)
    (void)hipFuncSetAttribute(reinterpret_cast<const void*>(k_fwd_x<T, MX>),
                              hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds);
  const int nb = resident_blocks(k_fwd_x<T, MX>, 64 * kTileJ, lds, ntiles);
  return launch(k_fwd_x<T, MX>, dim3(nb), dim3(64 * kTileJ), lds, s, pd, ntiles);
}

template <typename T, int MX>
static hipError_t run_x_inv_t(const cs3d_plan p, const ProbDev& pd, int nrhs, hipStream_t s) {
  const int ntiles = (p->ldy / kTileJ) * p->d.nz * nrhs;
  const size_t lds = lds_bytes_x_t<T, MX>(p);
  if (lds > 64 * 1024)
    (void)hipFuncSetAttribute(reinterpret_cast<const void*>(k_inv_x<T, MX>),
                              hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds);
  const int nb = resident_blocks(k_inv_x<T, MX>, 64 * kTileJ, lds, ntiles);
  return launch(k_inv_x<T, MX>, dim3(nb), dim3(64 * kTileJ), lds, s, pd, ntiles);
}

template <typename T, int MY>
static hipError_t run_y_fwd_t(const cs3d_plan p, const ProbDev& pd, int nrhs, hipStream_t s) {
  dim3 grid((p->d.nx + YCfg<MY>::LPB - 1) / YCfg<MY>::LPB, nrhs), block(kBlockY);
  return launch(k_fwd_y<T, MY>, grid, block, lds_bytes_y_t<T, MY>(p), s, pd);
}

template <typename T, int MY>
static hipError_t run_y_back_t(const cs3d_plan p, const ProbDev& pd, int nrhs, hipStream_t s) {
  dim3 grid((p->d.nx + YCfg<MY>::LPB - 1) / YCfg<MY>::LPB, nrhs), block(kBlockY);
  return launch(k_back_y<T, MY>, grid, block, lds_bytes_y_t<T, MY>(p), s, pd);
}

#define CS3D_DISPATCH(fn, M, ...)                 \
  switch (M) {                                    \
    case 64: return fn<T, 64>(__VA_ARGS__);       \
    case 128: return fn<T, 128>(__VA_ARGS__);     \
    case 256: return fn<T, 256>(__VA_ARGS__);     \
    case 512: return fn<T, 512>(__VA_ARGS__);     \
    case 1024: return fn<T, 1024>(__VA_ARGS__);   \
    default: return fn<T, 0>(__VA_ARGS__);        \
  }

template <typename T>
static hipError_t run_x_fwd(const cs3d_plan p, const ProbDev& pd, int nrhs, hipStream_t s) {
  CS3D_DISPATCH(run_x_fwd_t, p->fx, p, pd, nrhs, s)
}
template <typename T>
static hipError_t run_x_inv(const cs3d_plan p, const ProbDev& pd, int nrhs, hipStream_t s) {
  CS3D_DISPATCH(run_x_inv_t, p->fx, p, pd, nrhs, s)
}
template <typename T>
static hipError_t run_y_fwd(const cs3d_plan p, const ProbDev& pd, int nrhs, hipStream_t s) {
  CS3D_DISPATCH(run_y_fwd_t, p->fy, p, pd, nrhs, s)
}
template <typename T>
static hipError_t run_y_back(const cs3d_plan p, const ProbDev& pd, int nrhs, hipStream_t s) {
  CS3D_DISPATCH(run_y_back_t, p->fy, p, pd, nrhs, s)
}
#undef CS3D_DISPATCH

static hipError_t run_rhs(const cs3d_plan p, const ProbDev& pd, int nrhs, hipStream_t s) {
  const int nzc = (p->d.nz + kZChunk - 1) / kZChunk;
  dim3 grid((p->d.nx + kRX - 1) / kRX, (p->d.ny + kRY - 1) / kRY, nzc * nrhs);
  if (grid.y > 65535u || grid.z > 65535u) return hipErrorInvalidValue;
  hipLaunchKernelGGL(k_rhs, grid, dim3(kRThreads), 0, s, pd);
  return hipGetLastError();
}

static ProbDev make_pd(const cs3d_plan p, const double* f, const double* glo, const double* ghi,
                       const double* F, double* u, int nrhs) {
  ProbDev pd{};
  pd.nx = p->d.nx;
  pd.ny = p->d.ny;
  pd.nz = p->d.nz;
  pd.Mx = p->Mx;
  pd.My = p->My;
  pd.ldy = p->ldy;
  pd.scheme = p->d.scheme;
  pd.hx = p->d.hx;
  pd.hy = p->d.hy;
  pd.hz = p->d.hz;
  pd.gamma = p->d.gamma;
  pd.scale = 4.0 / ((double)p->Mx * (double)p->My);
  pd.W = p->dW;
  pd.LC = p->dLC;
  pd.k2 = p->dk2;
  pd.k2z = p->dk2z;
  pd.ctx = p->dctx;
  pd.cty = p->dcty;
  pd.twx = p->dtwx;
  pd.twy = p->dtwy;
  pd.sinx = p->dsinx;
  pd.siny = p->dsiny;
  pd.f = f;
  pd.f_stride = (long long)(p->d.nx + 2) * (p->d.ny + 2) * (p->d.nz + 2);
  pd.glo = glo;
  pd.ghi = ghi;
  pd.g_stride = (long long)(p->d.nx + 2) * (p->d.ny + 2);
  pd.F = F;
  pd.u = u;
  pd.u_stride = (long long)p->d.nx * p->d.ny * p->d.nz;
  pd.G = p->ws;
  pd.G_stride = (long long)g_elems(p);
  pd.C = p->ws ? reinterpret_cast<double*>(reinterpret_cast<char*>(p->ws) + off_C(p, nrhs)) : nullptr;
  pd.stats = p->dstats;
  return pd;
}

// Interval timing: mark(stage) starts an interval of that stage, end_solve closes the last.
static hipError_t mark(cs3d_plan p, int stage, hipStream_t s) {
  if (p->cur_marks >= kMaxMarks) return hipSuccess;  // further passes are not timed separately
  const size_t q = (size_t)(p->solves % kRing);
  p->ring_sid[q * kMaxMarks + p->cur_marks] = (signed char)stage;
  return hipEventRecord(p->ring[q * (kMaxMarks + 1) + p->cur_marks++], s);
}

static hipError_t end_solve(cs3d_plan p, hipStream_t s) {
  const size_t q = (size_t)(p->solves % kRing);
  const hipError_t e = hipEventRecord(p->ring[q * (kMaxMarks + 1) + p->cur_marks], s);
  p->ring_n[q] = p->cur_marks;
  p->cur_marks = 0;
  ++p->solves;
  return e;
}

// K1 -> K2 -> K3 -> K4 on the right-hand side pd.F (a solve with the transform type T)
template <typename T>
static hipError_t transform_solve(cs3d_plan p, const ProbDev& pd, int nrhs, hipStream_t s) {
  hipError_t e;
  if ((e = mark(p, 1, s)) != hipSuccess) return e;
  if ((e = run_x_fwd<T>(p, pd, nrhs, s)) != hipSuccess) return e;
  if ((e = mark(p, 2, s)) != hipSuccess) return e;
  if ((e = run_y_fwd<T>(p, pd, nrhs, s)) != hipSuccess) return e;
  if ((e = mark(p, 3, s)) != hipSuccess) return e;
  if ((e = run_y_back<T>(p, pd, nrhs, s)) != hipSuccess) return e;
  if ((e = mark(p, 4, s)) != hipSuccess) return e;
  return run_x_inv<T>(p, pd, nrhs, s);
}

static hipError_t norm_pass(const double* x, long long n, double* acc, hipStream_t s);

// r = F - A U and its squared norm into stats word `slot` (slot < 0: no norm)
static hipError_t residual_pass(cs3d_plan p, const ProbDev& pd, const double* F, const double* U, double* R,
                                int nrhs, int slot, hipStream_t s) {
  const int nzc = (p->d.nz + kZChunk - 1) / kZChunk;
  dim3 grid((p->d.nx + kRX - 1) / kRX, (p->d.ny + kRY - 1) / kRY, nzc * nrhs);
  if (grid.z > 65535u || grid.y > 65535u) return hipErrorInvalidValue;
  double* acc = slot >= 0 ? reinterpret_cast<double*>(p->dstats) + slot : nullptr;
  hipLaunchKernelGGL(k_residual, grid, dim3(kRThreads), 0, s, pd, F, U, R, acc);
  return hipGetLastError();
}

static cs3d_status solve_common(cs3d_plan p, int nrhs, const double* f, int assembled, const double* glo,
                                const double* ghi, double* u, void* hip_stream) {
  if (!p || !f || !u) return CS3D_E_INVAL;
  if (nrhs < 1 || nrhs > p->d.max_rhs) return CS3D_E_INVAL;
  if (!assembled && p->d.scheme == CS3D_WEIGHTS) return CS3D_E_INVAL;
  if (!p->ws || p->ws_bytes < cs3d_workspace_bytes(p, nrhs)) return CS3D_E_WORKSPACE;
  if (assembled && f == u) return CS3D_E_INVAL;  // F must stay intact until K1 has read all of it
  hipStream_t s = (hipStream_t)hip_stream;
  p->last_stream = s;
  p->cur_marks = 0;
  const bool mixed = p->d.precision != CS3D_FP64;
  char* ws = reinterpret_cast<char*>(p->ws);
  // where the interior right-hand side lives: the caller's F, or K0's output (u for the
  // FP64 path, whose K4 overwrites it last; a workspace array for the mixed path, which
  // needs F again for every residual)
  double* Fbuf = mixed ? reinterpret_cast<double*>(ws + off_F(p, nrhs)) : u;
  const double* F = assembled ? f : Fbuf;
  ProbDev pd = make_pd(p, assembled ? nullptr : f, glo, ghi, F, Fbuf, nrhs);
  if (hipEventRecord(p->ev0, s) != hipSuccess) return CS3D_E_DEVICE;
  hipLaunchKernelGGL(k_stats_reset, dim3(1), dim3(64), 0, s, p->dstats);
  if (hipGetLastError() != hipSuccess) return CS3D_E_DEVICE;
  if (!assembled) {
    if (mark(p, 0, s) != hipSuccess || run_rhs(p, pd, nrhs, s) != hipSuccess) return CS3D_E_DEVICE;
  }
  pd.u = u;
  pd.accumulate = 0;
  if (!mixed) {
    if (transform_solve<double>(p, pd, nrhs, s) != hipSuccess) return CS3D_E_DEVICE;
    p->refine_done = 0;
  } else {
    // FP32 transforms + FP64 tridiagonal solves, then refine_steps corrections
    // U += A_mixed^{-1} (F - A U) with the FP64 27-point residual (Section 3.1 operator)
    double* R = reinterpret_cast<double*>(ws + off_R(p, nrhs));
    if (mark(p, 5, s) != hipSuccess) return CS3D_E_DEVICE;
    if (norm_pass(F, (long long)n3(p) * nrhs, reinterpret_cast<double*>(p->dstats) + 2, s) != hipSuccess)
      return CS3D_E_DEVICE;
    if (transform_solve<float>(p, pd, nrhs, s) != hipSuccess) return CS3D_E_DEVICE;
    for (int it = 0; it <= p->d.refine_steps; ++it) {
      if (mark(p, 5, s) != hipSuccess) return CS3D_E_DEVICE;
      if (residual_pass(p, pd, F, u, R, nrhs, 3 + it, s) != hipSuccess) return CS3D_E_DEVICE;
      if (it == p->d.refine_steps) break;
      ProbDev pc = pd;
      pc.F = R;
      pc.accumulate = 1;
      if (transform_solve<float>(p, pc, nrhs, s) != hipSuccess) return CS3D_E_DEVICE;
    }
    p->refine_done = p->d.refine_steps;
  }
  if (end_solve(p, s) != hipSuccess) return CS3D_E_DEVICE;
  if (hipEventRecord(p->ev1, s) != hipSuccess) return CS3D_E_DEVICE;
  p->timed = true;
  return CS3D_OK;
}

static hipError_t norm_pass(const double* x, long long n, double* acc, hipStream_t s) {
  long long blocks = (n + 255) / 256;
  if (blocks > 4096) blocks = 4096;
  if (blocks < 1) blocks = 1;
  hipLaunchKernelGGL(k_sumsq, dim3((unsigned)blocks), dim3(256), 0, s, x, n, acc);
  return hipGetLastError();
}

extern "C" cs3d_status cs3d_solve(cs3d_plan p, int nrhs, const double* dev_f, const double* dev_g_lo,
                                  const double* dev_g_hi, double* dev_u, void* hip_stream) {
  return solve_common(p, nrhs, dev_f, 0, dev_g_lo, dev_g_hi, dev_u, hip_stream);
}

extern "C" cs3d_status cs3d_solve_assembled(cs3d_plan p, int nrhs, const double* dev_F, double* dev_u,
                                            void* hip_stream) {
  return solve_common(p, nrhs, dev_F, 1, nullptr, nullptr, dev_u, hip_stream);
}

extern "C" cs3d_status cs3d_residual(cs3d_plan p, int nrhs, const double* dev_f, int assembled,
                                     const double* dev_g_lo, const double* dev_g_hi, const double* dev_u,
                                     double* dev_r, void* hip_stream) {
  if (!p || !dev_f || !dev_u || !dev_r) return CS3D_E_INVAL;
  if (nrhs < 1 || nrhs > p->d.max_rhs) return CS3D_E_INVAL;
  if (!assembled && p->d.scheme == CS3D_WEIGHTS) return CS3D_E_INVAL;
  if (dev_r == dev_u || dev_r == dev_f) return CS3D_E_INVAL;
  hipStream_t s = (hipStream_t)hip_stream;
  // F (with the lift) goes into r, then r = F - A U in place
  const ProbDev pd = make_pd(p, assembled ? nullptr : dev_f, dev_g_lo, dev_g_hi, nullptr, dev_r, nrhs);
  if (!assembled && run_rhs(p, pd, nrhs, s) != hipSuccess) return CS3D_E_DEVICE;
  return residual_pass(p, pd, assembled ? dev_f : (const double*)dev_r, dev_u, dev_r, nrhs, -1, s) == hipSuccess
             ? CS3D_OK
             : CS3D_E_DEVICE;
}

extern "C" cs3d_status cs3d_get_stats(cs3d_plan p, cs3d_stats* out) {
  if (!p || !out) return CS3D_E_INVAL;
  std::memset(out, 0, sizeof(*out));
  for (double& v : out->residual_history) v = NAN;
  if (p->last_stream && hipStreamSynchronize(p->last_stream) != hipSuccess) return CS3D_E_DEVICE;
  if (!p->last_stream && hipDeviceSynchronize() != hipSuccess) return CS3D_E_DEVICE;
  unsigned long long h[kStatsWords];
  if (hipMemcpy(h, p->dstats, sizeof(h), hipMemcpyDeviceToHost) != hipSuccess) return CS3D_E_DEVICE;
  double d[kStatsWords];
  std::memcpy(d, h, sizeof(d));
  out->min_abs_pivot = d[0];
  out->bad_pivots = (int64_t)h[1];
  out->refine_done = p->refine_done;
  cs3d_status st = h[1] ? CS3D_E_SINGULAR : CS3D_OK;
  if (p->d.precision != CS3D_FP64 && p->timed) {
    const double fn = std::sqrt(d[2]);
    for (int k = 0; k <= p->refine_done && k < 8; ++k) out->residual_history[k] = std::sqrt(d[3 + k]) / fn;
    const double last = out->residual_history[p->refine_done < 8 ? p->refine_done : 7];
    if (st == CS3D_OK && !(last <= kResidualTarget)) st = CS3D_E_NOTCONVERGED;
  }
  float ms = 0.f;
  if (p->timed && hipEventElapsedTime(&ms, p->ev0, p->ev1) == hipSuccess) out->last_solve_ms = ms;
  const long long n = p->solves < kRing ? p->solves : kRing;
  out->stage_count = kStages;
  out->timed_solves = (int)n;
  for (long long q = 0; q < n; ++q)
    for (int k = 0; k < p->ring_n[q]; ++k) {
      float t = 0.f;
      if (hipEventElapsedTime(&t, p->ring[q * (kMaxMarks + 1) + k], p->ring[q * (kMaxMarks + 1) + k + 1]) !=
          hipSuccess)
        return CS3D_E_DEVICE;
      out->stage_ms[p->ring_sid[q * kMaxMarks + k]] += (double)t / (double)n;
    }
  return st;
}

extern "C" cs3d_status cs3d_reset_timers(cs3d_plan p) {
  if (!p) return CS3D_E_INVAL;
  if (p->last_stream) (void)hipStreamSynchronize(p->last_stream);
  p->solves = 0;
  return CS3D_OK;
}

extern "C" const char* cs3d_status_str(cs3d_status st) {
  switch (st) {
    case CS3D_OK: return "ok";
    case CS3D_E_INVAL: return "invalid argument";
    case CS3D_E_NOMEM: return "out of memory";
    case CS3D_E_DEVICE: return "HIP device error";
    case CS3D_E_SINGULAR: return "zero or non-finite pivot";
    case CS3D_E_NOTCONVERGED: return "refinement did not converge";
    case CS3D_E_UNSUPPORTED: return "unsupported request";
    case CS3D_E_WORKSPACE: return "workspace missing or too small";
    default: return "unknown status";
  }
}

extern "C" const char* cs3d_version(void) { return "cs3d 0.1 (gfx950)"; }

// ---------------------------------------------------------------------------
// Batches (first version: one plan per member, launched back to back).
// ---------------------------------------------------------------------------
struct cs3d_batch_s {
  std::vector<cs3d_plan> plans;
  std::vector<size_t> offs;
  size_t bytes = 0;
  void* ws = nullptr;
};

extern "C" cs3d_status cs3d_batch_create(int n, const cs3d_desc* descs, void* hip_stream, cs3d_batch* out) {
  if (!out || n < 1 || !descs) return CS3D_E_INVAL;
  *out = nullptr;
  cs3d_batch b = new (std::nothrow) cs3d_batch_s();
  if (!b) return CS3D_E_NOMEM;
  size_t off = 0;
  for (int i = 0; i < n; ++i) {
    cs3d_plan p = nullptr;
    cs3d_status st = cs3d_plan_create(&descs[i], hip_stream, &p);
    if (st != CS3D_OK) {
      for (cs3d_plan q : b->plans) cs3d_plan_destroy(q);
      delete b;
      return st;
    }
    b->plans.push_back(p);
    b->offs.push_back(off);
    off += round256(cs3d_workspace_bytes(p, 1));
  }
  b->bytes = off;
  *out = b;
  return CS3D_OK;
}

extern "C" size_t cs3d_batch_workspace_bytes(cs3d_batch b) { return b ? b->bytes : 0; }

extern "C" cs3d_status cs3d_batch_set_workspace(cs3d_batch b, void* dev, size_t bytes) {
  if (!b || !dev || ((uintptr_t)dev & 255)) return CS3D_E_INVAL;
  if (bytes < b->bytes) return CS3D_E_WORKSPACE;
  b->ws = dev;
  for (size_t i = 0; i < b->plans.size(); ++i)
    cs3d_set_workspace(b->plans[i], (char*)dev + b->offs[i], cs3d_workspace_bytes(b->plans[i], 1));
  return CS3D_OK;
}

extern "C" cs3d_status cs3d_batch_solve(cs3d_batch b, const double* const* f, double* const* u, void* s) {
  if (!b || !f || !u) return CS3D_E_INVAL;
  if (!b->ws) return CS3D_E_WORKSPACE;
  for (size_t i = 0; i < b->plans.size(); ++i) {
    cs3d_status st = cs3d_solve(b->plans[i], 1, f[i], nullptr, nullptr, u[i], s);
    if (st != CS3D_OK) return st;
  }
  return CS3D_OK;
}

extern "C" cs3d_status cs3d_batch_get_stats(cs3d_batch b, cs3d_stats* out) {
  if (!b || !out) return CS3D_E_INVAL;
  cs3d_stats acc{};
  acc.min_abs_pivot = INFINITY;
  cs3d_status worst = CS3D_OK;
  for (cs3d_plan p : b->plans) {
    cs3d_stats st{};
    cs3d_status r = cs3d_get_stats(p, &st);
    if (r == CS3D_E_DEVICE) return r;
    if (r != CS3D_OK) worst = r;
    acc.min_abs_pivot = std::fmin(acc.min_abs_pivot, st.min_abs_pivot);
    acc.bad_pivots += st.bad_pivots;
  }
  for (double& v : acc.residual_history) v = NAN;
  *out = acc;
  return worst;
}

extern "C" cs3d_status cs3d_batch_destroy(cs3d_batch b) {
  if (!b) return CS3D_OK;
  for (cs3d_plan p : b->plans) cs3d_plan_destroy(p);
  delete b;
  return CS3D_OK;
}
