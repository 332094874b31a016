// cs3d.hip - host runtime and C ABI of the compact-stencil direct solver.
//
// A plan owns small device tables only: the row weights of Sections 3.2-3.5,
// the samples of k^2 and (k^2)_z used by the RHS operator, the modal cosines of
// Section 3.6 and the line-transform tables.  Data and workspace belong to the
// caller.  Every solve is four kernel launches (kernels.hpp) on the caller's
// stream, plus a tiny statistics reset.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <complex>
#include <cstdint>
#include <cstring>
#include <mutex>
#include <new>
#include <type_traits>
#include <vector>

#include "../../include/cs3d.h"
#include "batch.hpp"
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

// Launch-shape choices of a plan or batch (defaults, cs3d_autotune or cs3d_set_tuning)
struct Tuning {
  int zchunk = kZChunk;  // planes per workgroup of the z-marching passes
  int xpersist = 1;      // x passes: 1 = one resident workgroup set walking all tiles,
                         // 0 = one workgroup per tile
  int ywpl = 2;          // waves per y-line where the FFT allows two (M >= 512)
  int order = 1;         // batches: members by decreasing cost per item
  int graph = 1;         // batches: captured graph replay
  int yrhs = 1;          // right-hand sides per y-pass workgroup (1, 2 or 4)
  int xwpl = 1;          // waves per x-line where the FFT allows two (M >= 512)
  int pack = 0;          // batches: lines of 64- and 128-point transforms packed to a wave
};

struct cs3d_plan_s {
  cs3d_desc d{};
  Tuning tune;
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
  bool notime = false;  // a cs3d_solve_static call: no per-pass timing (its ring would need events)
  // Robin z faces: d.nz counts the system's planes (nz + 2), nz_phys the interior ones
  bool robin = false;
  int nz_phys = 0;
  double rb[4] = {0.0, 0.0, 0.0, 0.0};
  // per-pass timing ring: kRing solves x (kMaxMarks + 1) events; interval k of a solve
  // belongs to stage ring_sid[...]
  std::vector<hipEvent_t> ring;
  std::vector<signed char> ring_sid;
  std::vector<int> ring_n;
  long long solves = 0;   // solves recorded since the last reset
  int cur_marks = 0;
  int refine_done = 0;
  std::vector<double> hW;  // host copy of the weights
  // complex k: imaginary parts of the weights, modal coefficients and k^2 samples
  bool cplx = false;
  double* dWi = nullptr;
  double* dLCi = nullptr;
  double* dk2i = nullptr;
  double* dk2zi = nullptr;
  // Neumann sides: d.nx, d.ny count the nodes of a plane (interior + 2 side nodes) and
  // the line transforms are DCT-I
  bool neu = false;
};

// ---------------------------------------------------------------------------
// Row weights, Sections 3.2 - 3.5.  W[l][o][(a,b,c,d)], o = 0,1,2 for offsets -1,0,+1.
// ---------------------------------------------------------------------------
// S = double, or std::complex<double> for complex k (absorbing media): the same formulas
// with complex k^2 samples k2s, k2zs, k2zzs (nz+2 each)
template <typename S>
static cs3d_status build_weights_t(const cs3d_desc& d, const S* k2s, const S* k2zs, const S* k2zzs,
                                   std::vector<S>& W) {
  const int nz = d.nz;
  W.assign((size_t)nz * 12, S(0.0));
  const double rzx = d.hz * d.hz / (d.hx * d.hx), rzy = d.hz * d.hz / (d.hy * d.hy);
  const double hz2 = d.hz * d.hz;
  auto at = [&](int l, int o, int q) -> S& { return W[(size_t)l * 12 + o * 4 + q]; };
  for (int l = 0; l < nz; ++l) {
    const int zl = l + 1;  // sample index of plane z_l
    switch (d.scheme) {
      case CS3D_HELM2: {
        const S k0 = k2s[zl];
        at(l, 0, 3) = 1.0;
        at(l, 2, 3) = 1.0;
        at(l, 1, 1) = rzx;
        at(l, 1, 2) = rzy;
        at(l, 1, 3) = -2.0 * (rzx + rzy + 1.0) + hz2 * k0;
        break;
      }
      case CS3D_HELM4: {
        const S km = k2s[zl - 1], k0 = k2s[zl], kp = k2s[zl + 1];
        for (int o = 0; o <= 2; o += 2) {
          const S kk = o == 0 ? km : kp;
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
        const S km = k2s[zl - 1], k0 = k2s[zl], kp = k2s[zl + 1];
        const S kz = k2zs[zl], kzz = k2zzs[zl];
        for (int o = 0; o <= 2; o += 2) {
          const double sg = o == 0 ? -1.0 : 1.0;
          const S kk = o == 0 ? km : kp;
          at(l, o, 0) = 1.0 / 30.0;
          const S bc = 0.1 + h2 * kk / 90.0 + sg * h3 * kz / 120.0;
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
        for (int q = 0; q < 12; ++q) W[(size_t)l * 12 + q] = S(d.weights[(size_t)l * 12 + q]);
        break;
      default:
        return CS3D_E_INVAL;
    }
  }
  return CS3D_OK;
}

static cs3d_status build_weights(const cs3d_desc& d, std::vector<double>& W) {
  return build_weights_t<double>(d, d.k2, d.k2_z, d.k2_zz, W);
}

// complex k: weights of (Re k^2 + i Im k^2), split into real and imaginary tables
static cs3d_status build_weights_c(const cs3d_desc& d, std::vector<double>& Wr, std::vector<double>& Wi) {
  const int nzp = d.nz + 2;
  std::vector<std::complex<double>> k2(nzp), k2z(nzp, 0.0), k2zz(nzp, 0.0), W;
  for (int i = 0; i < nzp; ++i) {
    k2[i] = {d.k2[i], d.k2_im[i]};
    if (d.k2_z) k2z[i] = {d.k2_z[i], d.k2_z_im ? d.k2_z_im[i] : 0.0};
    if (d.k2_zz) k2zz[i] = {d.k2_zz[i], d.k2_zz_im ? d.k2_zz_im[i] : 0.0};
  }
  const cs3d_status st = build_weights_t<std::complex<double>>(d, k2.data(), k2z.data(), k2zz.data(), W);
  Wr.resize(W.size());
  Wi.resize(W.size());
  for (size_t q = 0; q < W.size(); ++q) {
    Wr[q] = W[q].real();
    Wi[q] = W[q].imag();
  }
  return st;
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

// cos(pi k/M), k < 2M: the direct sums of the cosine transform
static void cosines(int M, std::vector<double>& c) {
  c.resize(2 * (size_t)M);
  for (int k = 0; k < 2 * M; ++k)
    c[k] = (double)cosl(3.14159265358979323846264338327950288L * (long double)k / (long double)M);
}

// Neumann sides: s_k = 1 - cos(pi k/M) = 2 sin^2(pi k/(2M)) for the modes k = 0..M of a
// line of M + 1 nodes (entry k = position k + 1 - 1)
static void one_minus_cosines_dct(int M, std::vector<double>& c) {
  c.resize((size_t)M + 1);
  for (int k = 0; k <= M; ++k) {
    const long double sn = sinl(3.14159265358979323846264338327950288L * (long double)k / (2.0L * M));
    c[k] = (double)(2.0L * sn * sn);
  }
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

// the same coefficients for complex weights (Wr + i Wi), real and imaginary parts
static void modal_coefficients_c(const std::vector<double>& Wr, const std::vector<double>& Wi,
                                 std::vector<double>& LCr, std::vector<double>& LCi) {
  LCr.resize(Wr.size());
  LCi.resize(Wr.size());
  for (size_t r = 0; r < Wr.size() / 4; ++r) {
    using C = std::complex<long double>;
    const C a(Wr[4 * r], Wi[4 * r]), b(Wr[4 * r + 1], Wi[4 * r + 1]), c(Wr[4 * r + 2], Wi[4 * r + 2]),
        d(Wr[4 * r + 3], Wi[4 * r + 3]);
    const C v[4] = {4.0L * a + 2.0L * b + 2.0L * c + d, -(4.0L * a + 2.0L * b), -(4.0L * a + 2.0L * c), 4.0L * a};
    for (int q = 0; q < 4; ++q) {
      LCr[4 * r + q] = (double)v[q].real();
      LCi[4 * r + q] = (double)v[q].imag();
    }
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
  if (d->sides != CS3D_SIDES_DIRICHLET && d->sides != CS3D_SIDES_NEUMANN) return CS3D_E_INVAL;
  if (d->sides == CS3D_SIDES_NEUMANN) {
    // lines of nx + 2 (ny + 2) nodes within the 1023-value line layout of the passes
    if (d->nx + 2 > kMaxN || d->ny + 2 > kMaxN) return CS3D_E_INVAL;
    if (d->precision != CS3D_FP64 || d->k2_im) return CS3D_E_UNSUPPORTED;
  }
  if (d->zfaces != CS3D_ZFACES_DIRICHLET && d->zfaces != CS3D_ZFACES_ROBIN) return CS3D_E_INVAL;
  if (d->zfaces == CS3D_ZFACES_ROBIN) {
    if (d->scheme != CS3D_HELM2 && d->scheme != CS3D_HELM4 && d->scheme != CS3D_HELM6) return CS3D_E_UNSUPPORTED;
    if (d->precision != CS3D_FP64 || d->k2_im || d->sides != CS3D_SIDES_DIRICHLET) return CS3D_E_UNSUPPORTED;
    if (!d->k2_z || d->nz < 4) return CS3D_E_INVAL;
    for (int q = 0; q < 2; ++q)
      if (!std::isfinite(d->robin_alpha[q]) || d->robin_alpha[q] == 0.0 || !std::isfinite(d->robin_beta[q]))
        return CS3D_E_INVAL;
  }
  if (d->k2_im) {  // complex k: Helmholtz schemes, FP64
    if (d->scheme == CS3D_HELM6 && (!d->k2_z_im || !d->k2_zz_im)) return CS3D_E_INVAL;
    if (d->scheme != CS3D_HELM2 && d->scheme != CS3D_HELM4 && d->scheme != CS3D_HELM6) return CS3D_E_UNSUPPORTED;
    if (d->precision != CS3D_FP64) return CS3D_E_UNSUPPORTED;
  }
  return CS3D_OK;
}

static void plan_free(cs3d_plan p) {
  if (!p) return;
  void* ptrs[] = {p->dW,   p->dLC,  p->dk2,    p->dk2z, p->dctx, p->dcty, p->dtwx, p->dtwy,
                  p->dsinx, p->dsiny, p->dstats, p->dWi,  p->dLCi, p->dk2i, p->dk2zi};
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
  p->d.k2_im = p->d.k2_z_im = p->d.k2_zz_im = nullptr;
  p->cplx = desc->k2_im != nullptr;
  p->neu = desc->sides == CS3D_SIDES_NEUMANN;
  // both kinds: the transform of a line spans M = N_interior + 1 intervals
  p->Mx = desc->nx + 1;
  p->My = desc->ny + 1;
  p->fx = fft_len(desc->nx);
  p->fy = fft_len(desc->ny);
  if (p->neu) {
    p->d.nx = desc->nx + 2;  // the side nodes are unknowns
    p->d.ny = desc->ny + 2;
  }
  p->robin = desc->zfaces == CS3D_ZFACES_ROBIN;
  p->nz_phys = desc->nz;
  // the system's z planes: with Robin faces the face nodes z_0, z_{nz+1} are unknowns, and
  // the rows and samples of the desc cover them (the samples z_{-1} .. z_{nz+2})
  cs3d_desc wd = *desc;
  if (p->robin) {
    p->d.nz = desc->nz + 2;
    wd.nz = desc->nz + 2;
  }
  p->ldy = ((p->d.ny + 1 + 15) / 16) * 16;
  p->tune.ywpl = (p->fy == 1024) ? 2 : 1;
  // long z-columns: fewer halo planes per workgroup; FP32 transforms leave registers for
  // two right-hand sides per y-pass workgroup (the autotuner's choices at 1023^3)
  const bool mixed = desc->precision != CS3D_FP64;
  p->tune.zchunk = desc->nz >= 512 ? (mixed ? 128 : 64) : kZChunk;
  p->tune.yrhs = mixed ? 2 : 1;
  std::vector<double> hWi;
  st = p->cplx ? build_weights_c(wd, p->hW, hWi) : build_weights(wd, p->hW);
  if (st != CS3D_OK) {
    plan_free(p);
    return st;
  }
  hipStream_t s = (hipStream_t)hip_stream;
  const int nzp = p->d.nz + 2;
  std::vector<double> k2(nzp, 0.0), k2z(nzp, 0.0);
  if (p->robin) {
    // ghost-plane elimination of the two faces, as c0 + c1 D (D: in-plane 5-point Laplacian)
    const double h = desc->hz, h3 = h * h * h / 3.0;
    const double kl = desc->k2[1], kzl = desc->k2_z[1];              // z_0
    const double kh = desc->k2[nzp - 2], kzh = desc->k2_z[nzp - 2];  // z_{nz+1}
    const double ql = desc->robin_beta[0] / desc->robin_alpha[0];
    const double qh = desc->robin_beta[1] / desc->robin_alpha[1];
    p->rb[0] = h3 * kzl - ql * (-2.0 * h + h3 * kl);
    p->rb[1] = -ql * h3;
    p->rb[2] = -h3 * kzh - qh * (2.0 * h - h3 * kh);
    p->rb[3] = qh * h3;
  }
  if (desc->k2)
    for (int i = 0; i < nzp; ++i) k2[i] = desc->k2[i];
  if (desc->k2_z)
    for (int i = 0; i < nzp; ++i) k2z[i] = desc->k2_z[i];
  std::vector<double> ctx, cty, sx, sy, lc, lci, k2i(nzp, 0.0), k2zi(nzp, 0.0);
  if (p->cplx) {
    for (int i = 0; i < nzp; ++i) k2i[i] = desc->k2_im[i];
    if (desc->k2_z_im)
      for (int i = 0; i < nzp; ++i) k2zi[i] = desc->k2_z_im[i];
  }
  std::vector<double2> twx, twy;
  if (p->neu) {
    one_minus_cosines_dct(p->Mx, ctx);
    one_minus_cosines_dct(p->My, cty);
  } else {
    one_minus_cosines(desc->nx, ctx);
    one_minus_cosines(desc->ny, cty);
  }
  if (p->cplx) modal_coefficients_c(p->hW, hWi, lc, lci);
  else modal_coefficients(p->hW, lc);
  twiddles(p->Mx, twx);
  twiddles(p->My, twy);
  if (p->neu) {
    cosines(p->Mx, sx);
    cosines(p->My, sy);
  } else {
    sines(p->Mx, sx);
    sines(p->My, sy);
  }
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
  if (p->cplx) {
    CS3D_TRY(dalloc(&p->dWi, hWi.size()));
    CS3D_TRY(dalloc(&p->dLCi, lci.size()));
    CS3D_TRY(dalloc(&p->dk2i, k2i.size()));
    CS3D_TRY(dalloc(&p->dk2zi, k2zi.size()));
    CS3D_TRY(hipMemcpyAsync(p->dWi, hWi.data(), hWi.size() * 8, hipMemcpyHostToDevice, s));
    CS3D_TRY(hipMemcpyAsync(p->dLCi, lci.data(), lci.size() * 8, hipMemcpyHostToDevice, s));
    CS3D_TRY(hipMemcpyAsync(p->dk2i, k2i.data(), k2i.size() * 8, hipMemcpyHostToDevice, s));
    CS3D_TRY(hipMemcpyAsync(p->dk2zi, k2zi.data(), k2zi.size() * 8, hipMemcpyHostToDevice, s));
  }
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

// real slots of nrhs right-hand sides (two per complex right-hand side)
static int slots(const cs3d_plan p, int nrhs) { return p->cplx ? 2 * nrhs : nrhs; }

// workspace layout: G (transform intermediate, per real slot) | C (c' of the LU, shared by
// the right-hand sides; real and imaginary parts for complex k) | mixed path only:
// F (FP64 right-hand side, per rhs) | R (FP64 residual)
static size_t off_C(const cs3d_plan p, int nrhs) {
  return round256(g_elems(p) * elem_bytes(p) * (size_t)slots(p, nrhs));
}
static size_t off_F(const cs3d_plan p, int nrhs) {
  return off_C(p, nrhs) + round256(g_elems(p) * 8 * (p->cplx ? 2 : 1));
}
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
  const size_t a = (size_t)kTileJ * line_buf_elems<T, MX, 1>(p->d.nx) * sizeof(T);
  const size_t b = (size_t)kTileJ * tile_stride(p->d.nx) * sizeof(T);
  return (a > b ? a : b) + tw_bytes<T, MX>();
}

// the x passes with two waves per line
template <typename T, int MX>
static size_t lds_bytes_x2_t(const cs3d_plan p) {
  const size_t a = (size_t)kTileJ * line_buf_elems<T, MX, 2>(p->d.nx) * sizeof(T);
  const size_t b = (size_t)kTileJ * tile_stride(p->d.nx) * sizeof(T);
  return (a > b ? a : b) + tw_bytes<T, MX>();
}

template <typename T, int MY, int WPL = default_wpl<MY>(), bool PAIR = false>
static size_t lds_bytes_y_t(const cs3d_plan p) {
  return (size_t)YCfg<MY, WPL>::LPB * line_buf_elems<T, MY, WPL, PAIR>(p->d.ny) * sizeof(T) + tw_bytes<T, MY>();
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

// resident_blocks after raising the kernel's dynamic LDS limit (the occupancy query needs it)
template <typename KernelT>
static int resident_blocks_at(KernelT kern, int threads, size_t lds, int ntiles) {
  if (lds > 64 * 1024)
    (void)hipFuncSetAttribute(reinterpret_cast<const void*>(kern), hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds);
  return resident_blocks(kern, threads, lds, ntiles);
}

template <typename T, int MX, int KIND, typename TI>
static hipError_t run_x_fwd_i(const cs3d_plan p, const ProbDev& pd, int nrhs, hipStream_t s) {
  const int ntiles = (p->ldy / kTileJ) * p->d.nz * nrhs;
  if constexpr (MX >= 512) {
    if (p->tune.xwpl == 2) {  // two waves per line
      const size_t lds = lds_bytes_x2_t<T, MX>(p);
      const int nb = p->tune.xpersist ? resident_blocks_at(k_fwd_x2<T, MX, KIND, TI>, 128 * kTileJ, lds, ntiles) : ntiles;
      return launch(k_fwd_x2<T, MX, KIND, TI>, dim3(nb), dim3(128 * kTileJ), lds, s, pd, ntiles);
    }
  }
  const size_t lds = lds_bytes_x_t<T, MX>(p);
  if (lds > 64 * 1024)
    (void)hipFuncSetAttribute(reinterpret_cast<const void*>(k_fwd_x<T, MX, KIND, TI>),
                              hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds);
  // workgroups that take the tiles in pairs (the two halves of the lines of G; ldy is a
  // multiple of 2 kTileJ, so a plane's tiles pair up)
  static_assert(kTileJ == 8, "tile pairs fill the 16-value rows of the 128-byte lines of G");
  const int nwork = x_tile_pairs<T, MX>() ? ntiles / 2 : ntiles;
  const int nb = p->tune.xpersist ? resident_blocks(k_fwd_x<T, MX, KIND, TI>, 64 * kTileJ, lds, nwork) : nwork;
  return launch(k_fwd_x<T, MX, KIND, TI>, dim3(nb), dim3(64 * kTileJ), lds, s, pd, ntiles);
}

// the input F is FP64, or FP32 for the residuals of the mixed path (pd.f32_input)
template <typename T, int MX, int KIND = kDst>
static hipError_t run_x_fwd_t(const cs3d_plan p, const ProbDev& pd, int nrhs, hipStream_t s) {
  if constexpr (std::is_same<T, float>::value) {
    if (pd.f32_input) return run_x_fwd_i<T, MX, KIND, float>(p, pd, nrhs, s);
  }
  return run_x_fwd_i<T, MX, KIND, double>(p, pd, nrhs, s);
}

template <typename T, int MX, int KIND, bool ACC>
static hipError_t run_x_inv_a(const cs3d_plan p, const ProbDev& pd, int nrhs, hipStream_t s) {
  if constexpr (MX >= 512) {
    if (p->tune.xwpl == 2) {  // two waves per line
      const int ntiles = (p->ldy / kTileJ) * p->d.nz * nrhs;
      const size_t lds = lds_bytes_x2_t<T, MX>(p);
      const int nb = p->tune.xpersist ? resident_blocks_at(k_inv_x2<T, MX, KIND, ACC>, 128 * kTileJ, lds, ntiles) : ntiles;
      return launch(k_inv_x2<T, MX, KIND, ACC>, dim3(nb), dim3(128 * kTileJ), lds, s, pd, ntiles);
    }
  }
  const int ntiles = (p->ldy / kTileJ) * p->d.nz * nrhs;
  const size_t lds = lds_bytes_x_t<T, MX>(p);
  if (lds > 64 * 1024)
    (void)hipFuncSetAttribute(reinterpret_cast<const void*>(k_inv_x<T, MX, KIND, ACC>),
                              hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds);
  const int nb = p->tune.xpersist ? resident_blocks(k_inv_x<T, MX, KIND, ACC>, 64 * kTileJ, lds, ntiles) : ntiles;
  return launch(k_inv_x<T, MX, KIND, ACC>, dim3(nb), dim3(64 * kTileJ), lds, s, pd, ntiles);
}

// u = the result, or u += it for the corrections of the mixed path
template <typename T, int MX, int KIND = kDst>
static hipError_t run_x_inv_t(const cs3d_plan p, const ProbDev& pd, int nrhs, hipStream_t s) {
  return pd.accumulate ? run_x_inv_a<T, MX, KIND, true>(p, pd, nrhs, s) : run_x_inv_a<T, MX, KIND, false>(p, pd, nrhs, s);
}

// grid: (line groups, groups of NR right-hand sides)
template <int MY, int WPL, int NR>
static dim3 y_grid(const cs3d_plan p, int nrhs) {
  using C = YCfg<MY, WPL>;
  return dim3((p->d.nx + C::LPB - 1) / C::LPB, (nrhs + NR - 1) / NR);
}

// right-hand sides per y-pass workgroup: the tuned choice (1, 2 or 4), at most what the
// register budget of the transform size allows
template <typename T, int MY, int WPL, int NR, int KIND = kDst, bool ROBIN = false>
static hipError_t run_y_fwd_n(const cs3d_plan p, const ProbDev& pd, int nrhs, hipStream_t s) {
  return launch(k_fwd_y<T, MY, WPL, NR, KIND, ROBIN>, y_grid<MY, WPL, NR>(p, nrhs), dim3(kBlockY),
                lds_bytes_y_t<T, MY, WPL, ypair<T, MY, WPL, true>()>(p), s, pd, nrhs);
}

template <typename T, int MY, int WPL, int NR, int KIND = kDst>
static hipError_t run_y_back_n(const cs3d_plan p, const ProbDev& pd, int nrhs, hipStream_t s) {
  return launch(k_back_y<T, MY, WPL, NR, KIND>, y_grid<MY, WPL, NR>(p, nrhs), dim3(kBlockY),
                lds_bytes_y_t<T, MY, WPL, ypair<T, MY, WPL, false>()>(p), s, pd, nrhs);
}

static int y_rhs(const cs3d_plan p, int nrhs, int nrmax) {
  int nr = p->tune.yrhs < nrmax ? p->tune.yrhs : nrmax;
  while (nr > 1 && nr / 2 >= nrhs) nr /= 2;  // no wider than the solve
  return nr;
}

template <typename T, int MY, int WPL, int KIND = kDst, bool ROBIN = false>
static hipError_t run_y_fwd_w(const cs3d_plan p, const ProbDev& pd, int nrhs, hipStream_t s) {
  if constexpr (ROBIN) return run_y_fwd_n<T, MY, WPL, 1, KIND, true>(p, pd, nrhs, s);  // one RHS per group
  if constexpr (YCfg<MY, WPL, KIND>::NRMAX >= 4) {
    const int nr = y_rhs(p, nrhs, 4);
    if (nr == 4) return run_y_fwd_n<T, MY, WPL, 4, KIND>(p, pd, nrhs, s);
    if (nr == 2) return run_y_fwd_n<T, MY, WPL, 2, KIND>(p, pd, nrhs, s);
  }
  return run_y_fwd_n<T, MY, WPL, 1, KIND>(p, pd, nrhs, s);
}

template <typename T, int MY, int WPL, int KIND = kDst>
static hipError_t run_y_back_w(const cs3d_plan p, const ProbDev& pd, int nrhs, hipStream_t s) {
  if constexpr (YCfg<MY, WPL, KIND>::NRMAX >= 4) {
    const int nr = y_rhs(p, nrhs, 4);
    if (nr == 4) return run_y_back_n<T, MY, WPL, 4, KIND>(p, pd, nrhs, s);
    if (nr == 2) return run_y_back_n<T, MY, WPL, 2, KIND>(p, pd, nrhs, s);
  }
  return run_y_back_n<T, MY, WPL, 1, KIND>(p, pd, nrhs, s);
}

// waves per y-line: the tuned choice where two are possible (M >= 512), else one
template <typename T, int MY, int KIND = kDst, bool ROBIN = false>
static hipError_t run_y_fwd_t(const cs3d_plan p, const ProbDev& pd, int nrhs, hipStream_t s) {
  if constexpr (MY >= 512) {
    if (p->tune.ywpl == 2) return run_y_fwd_w<T, MY, 2, KIND, ROBIN>(p, pd, nrhs, s);
  }
  return run_y_fwd_w<T, MY, 1, KIND, ROBIN>(p, pd, nrhs, s);
}
// Robin z faces (FP64 sine transforms)
template <typename T, int MY>
static hipError_t run_y_fwd_robin(const cs3d_plan p, const ProbDev& pd, int nrhs, hipStream_t s) {
  return run_y_fwd_t<T, MY, kDst, true>(p, pd, nrhs, s);
}

template <typename T, int MY, int KIND = kDst>
static hipError_t run_y_back_t(const cs3d_plan p, const ProbDev& pd, int nrhs, hipStream_t s) {
  if constexpr (MY >= 512) {
    if (p->tune.ywpl == 2) return run_y_back_w<T, MY, 2, KIND>(p, pd, nrhs, s);
  }
  return run_y_back_w<T, MY, 1, KIND>(p, pd, nrhs, s);
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

// the cosine transforms of Neumann sides (FP64; lines of at most 1023 nodes, so M <= 512)
#define CS3D_DISPATCH_DCT(fn, M, ...)                  \
  switch (M) {                                         \
    case 64: return fn<double, 64, kDct>(__VA_ARGS__);   \
    case 128: return fn<double, 128, kDct>(__VA_ARGS__); \
    case 256: return fn<double, 256, kDct>(__VA_ARGS__); \
    case 512: return fn<double, 512, kDct>(__VA_ARGS__); \
    case 0: return fn<double, 0, kDct>(__VA_ARGS__);     \
    default: return hipErrorInvalidValue;              \
  }

template <typename T>
static hipError_t run_x_fwd(const cs3d_plan p, const ProbDev& pd, int nrhs, hipStream_t s) {
  if constexpr (std::is_same<T, double>::value) {
    if (p->neu) { CS3D_DISPATCH_DCT(run_x_fwd_t, p->fx, p, pd, nrhs, s) }
  }
  CS3D_DISPATCH(run_x_fwd_t, p->fx, p, pd, nrhs, s)
}
template <typename T>
static hipError_t run_x_inv(const cs3d_plan p, const ProbDev& pd, int nrhs, hipStream_t s) {
  if constexpr (std::is_same<T, double>::value) {
    if (p->neu) { CS3D_DISPATCH_DCT(run_x_inv_t, p->fx, p, pd, nrhs, s) }
  }
  CS3D_DISPATCH(run_x_inv_t, p->fx, p, pd, nrhs, s)
}
template <typename T>
static hipError_t run_y_fwd(const cs3d_plan p, const ProbDev& pd, int nrhs, hipStream_t s) {
  if constexpr (std::is_same<T, double>::value) {
    if (p->neu) { CS3D_DISPATCH_DCT(run_y_fwd_t, p->fy, p, pd, nrhs, s) }
    if (p->robin) { CS3D_DISPATCH(run_y_fwd_robin, p->fy, p, pd, nrhs, s) }
  }
  CS3D_DISPATCH(run_y_fwd_t, p->fy, p, pd, nrhs, s)
}
template <typename T>
static hipError_t run_y_back(const cs3d_plan p, const ProbDev& pd, int nrhs, hipStream_t s) {
  if constexpr (std::is_same<T, double>::value) {
    if (p->neu) { CS3D_DISPATCH_DCT(run_y_back_t, p->fy, p, pd, nrhs, s) }
  }
  CS3D_DISPATCH(run_y_back_t, p->fy, p, pd, nrhs, s)
}
#undef CS3D_DISPATCH
#undef CS3D_DISPATCH_DCT

static hipError_t run_rhs(const cs3d_plan p, const ProbDev& pd, int nrhs, hipStream_t s) {
  if (p->neu) {
    const dim3 grid((p->d.nx * p->d.ny + 255) / 256, (p->d.nz + kSidesChunk - 1) / kSidesChunk, nrhs);
    if (grid.y > 65535u || grid.z > 65535u) return hipErrorInvalidValue;
    hipLaunchKernelGGL(k_rhs_sides, grid, dim3(256), 0, s, pd);
    return hipGetLastError();
  }
  const int nzc = (pd.nz + pd.zchunk - 1) / pd.zchunk;
  dim3 grid((p->d.nx + kRX - 1) / kRX, (p->d.ny + kRYPlan - 1) / kRYPlan, nzc * nrhs);
  if (grid.y > 65535u || grid.z > 65535u) return hipErrorInvalidValue;
  hipLaunchKernelGGL(k_rhs, grid, dim3(kRThreadsPlan), 0, s, pd);
  hipError_t e = hipGetLastError();
  // face corrections: x and y faces (6th order), z faces (6th order and the lift)
  const bool h6 = p->d.scheme == CS3D_HELM6;
  const int nx = p->d.nx, ny = p->d.ny, nz = pd.nz;
  for (int axis = 0; axis < 3 && e == hipSuccess; ++axis) {
    if (axis < 2 && !h6) continue;
    if (axis == 2 && !h6 && !pd.glo && !pd.ghi) continue;
    const int npts = axis == 0 ? ny * nz : (axis == 1 ? nx * nz : nx * ny);
    hipLaunchKernelGGL(k_rhs_faces, dim3((npts + 255) / 256, 2, nrhs), dim3(256), 0, s, pd, axis);
    e = hipGetLastError();
  }
  return e;
}

// Robin z faces: the interior planes z_1..z_N through the RHS pass of the physical grid (no
// lift: the face data are not Dirichlet values), written from the second plane of u on, then
// the rows of the two face planes (k_robin_faces)
static hipError_t run_rhs_robin(const cs3d_plan p, const ProbDev& pd, int nrhs, hipStream_t s) {
  ProbDev pi = pd;
  pi.nz = p->nz_phys;
  pi.u = pd.u + (long long)p->d.nx * p->d.ny;
  pi.k2 = pd.k2 + 1;  // samples from z_0 on
  pi.k2z = pd.k2z + 1;
  pi.glo = pi.ghi = nullptr;
  pi.robin = 0;
  hipError_t e = run_rhs(p, pi, nrhs, s);
  if (e != hipSuccess) return e;
  const dim3 grid((p->d.nx * p->d.ny + 255) / 256, 2, nrhs);
  if (grid.z > 65535u) return hipErrorInvalidValue;
  hipLaunchKernelGGL(k_robin_faces, grid, dim3(256), 0, s, pd);
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
  pd.fx = p->fx;
  pd.fy = p->fy;
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
  const int cx = p->neu ? p->d.nx : p->d.nx + 2, cy = p->neu ? p->d.ny : p->d.ny + 2;  // closed grid
  pd.f_stride = (long long)cx * cy * (p->robin ? p->d.nz : p->d.nz + 2);  // f: physical closed grid
  pd.glo = glo;
  pd.ghi = ghi;
  pd.g_stride = (long long)cx * cy;
  pd.F = F;
  pd.u = u;
  pd.u_stride = (long long)p->d.nx * p->d.ny * p->d.nz;
  pd.G = p->ws;
  pd.G_stride = (long long)g_elems(p);
  pd.C = p->ws ? reinterpret_cast<double*>(reinterpret_cast<char*>(p->ws) + off_C(p, nrhs)) : nullptr;
  pd.stats = p->dstats;
  pd.zchunk = p->tune.zchunk;
  if (p->robin) {
    pd.robin = 1;
    for (int q = 0; q < 4; ++q) pd.rb[q] = p->rb[q];
    for (int q = 0; q < 2; ++q) {
      pd.ralpha[q] = p->d.robin_alpha[q];
      pd.rbeta[q] = p->d.robin_beta[q];
    }
  }
  if (p->cplx) {
    pd.Wi = p->dWi;
    pd.LCi = p->dLCi;
    pd.k2i = p->dk2i;
    pd.k2zi = p->dk2zi;
    pd.Ci = pd.C ? pd.C + g_elems(p) : nullptr;
  }
  return pd;
}

// The timing ring is created by the first solve of a plan (plans made for batch members
// never solve on their own and hold no ring).
static hipError_t ensure_ring(cs3d_plan p) {
  if (!p->ring.empty()) return hipSuccess;
  p->ring.assign((size_t)kRing * (kMaxMarks + 1), nullptr);
  p->ring_sid.assign((size_t)kRing * kMaxMarks, 0);
  p->ring_n.assign(kRing, 0);
  for (hipEvent_t& e : p->ring) {
    const hipError_t r = hipEventCreate(&e);
    if (r != hipSuccess) return r;
  }
  return hipSuccess;
}

// Interval timing: mark(stage) starts an interval of that stage, end_solve closes the last.
static hipError_t mark(cs3d_plan p, int stage, hipStream_t s) {
  if (p->notime) return hipSuccess;
  if (p->cur_marks >= kMaxMarks) return hipSuccess;  // further passes are not timed separately
  const size_t q = (size_t)(p->solves % kRing);
  p->ring_sid[q * kMaxMarks + p->cur_marks] = (signed char)stage;
  return hipEventRecord(p->ring[q * (kMaxMarks + 1) + p->cur_marks++], s);
}

static hipError_t end_solve(cs3d_plan p, hipStream_t s) {
  if (p->notime) return hipSuccess;
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

// complex k: the y passes carry both real slots of each complex right-hand side
template <int MY>
static hipError_t run_y_c_t(const cs3d_plan p, const ProbDev& pd, int nrhs, hipStream_t s, bool fwd) {
  constexpr int WPL = default_wpl<MY>();
  const dim3 grid((p->d.nx + YCfg<MY, WPL>::LPB - 1) / YCfg<MY, WPL>::LPB, nrhs);
  const size_t lds = lds_bytes_y_t<double, MY, WPL>(p);
  return fwd ? launch(k_fwd_y_c<MY, WPL>, grid, dim3(kBlockY), lds, s, pd)
             : launch(k_back_y_c<MY, WPL>, grid, dim3(kBlockY), lds, s, pd);
}

static hipError_t run_y_c(const cs3d_plan p, const ProbDev& pd, int nrhs, hipStream_t s, bool fwd) {
  switch (p->fy) {
    case 64: return run_y_c_t<64>(p, pd, nrhs, s, fwd);
    case 128: return run_y_c_t<128>(p, pd, nrhs, s, fwd);
    case 256: return run_y_c_t<256>(p, pd, nrhs, s, fwd);
    case 512: return run_y_c_t<512>(p, pd, nrhs, s, fwd);
    case 1024: return run_y_c_t<1024>(p, pd, nrhs, s, fwd);
    default: return run_y_c_t<0>(p, pd, nrhs, s, fwd);
  }
}

// K1 -> K2 -> K3 -> K4 for nrhs complex right-hand sides (FP64)
static hipError_t transform_solve_c(cs3d_plan p, const ProbDev& pd, int nrhs, hipStream_t s) {
  hipError_t e;
  if ((e = mark(p, 1, s)) != hipSuccess) return e;
  if ((e = run_x_fwd<double>(p, pd, 2 * nrhs, s)) != hipSuccess) return e;
  if ((e = mark(p, 2, s)) != hipSuccess) return e;
  if ((e = run_y_c(p, pd, nrhs, s, true)) != hipSuccess) return e;
  if ((e = mark(p, 3, s)) != hipSuccess) return e;
  if ((e = run_y_c(p, pd, nrhs, s, false)) != hipSuccess) return e;
  if ((e = mark(p, 4, s)) != hipSuccess) return e;
  return run_x_inv<double>(p, pd, 2 * nrhs, s);
}

// complex k: the terms of the RHS operator and the lift that couple the two parts
static hipError_t run_rhs_cx(const cs3d_plan p, const ProbDev& pd, int nrhs, hipStream_t s) {
  const bool h6 = p->d.scheme == CS3D_HELM6;
  if (!h6 && !pd.glo && !pd.ghi) return hipSuccess;
  const dim3 grid((p->d.nx * p->d.ny + 255) / 256,
                  h6 ? (p->d.nz + kSidesChunk - 1) / kSidesChunk : (p->d.nz == 1 ? 1 : 2), nrhs);
  hipLaunchKernelGGL(k_rhs_cx, grid, dim3(256), 0, s, pd);
  return hipGetLastError();
}


// r = F - A U (FP64 arithmetic) and its squared norm into stats word `slot` (slot < 0: no
// norm); r is stored as TR, or not at all when R is null; slotF >= 0 also sums ||F||^2 there
template <typename TR>
static hipError_t residual_pass(cs3d_plan p, const ProbDev& pd, const double* F, const double* U, TR* R,
                                int nrhs, int slot, hipStream_t s, int slotF = -1) {
  const int nzc = (p->d.nz + pd.zchunk - 1) / pd.zchunk;
  dim3 grid((p->d.nx + kQTX - 1) / kQTX, (p->d.ny + kQTY - 1) / kQTY, nzc * nrhs);
  if (grid.z > 65535u || grid.y > 65535u) return hipErrorInvalidValue;
  double* acc = slot >= 0 ? reinterpret_cast<double*>(p->dstats) + slot : nullptr;
  double* accF = (slot >= 0 && slotF >= 0) ? reinterpret_cast<double*>(p->dstats) + slotF : nullptr;
  if (R) {
    hipLaunchKernelGGL((k_residual<TR, true>), grid, dim3(kQThreads), 0, s, pd, F, U, R, acc, accF);
  } else {
    hipLaunchKernelGGL((k_residual<TR, false>), grid, dim3(kQThreads), 0, s, pd, F, U, R, acc, accF);
  }
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
  if (!p->notime && ensure_ring(p) != hipSuccess) return CS3D_E_DEVICE;
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
    if (mark(p, 0, s) != hipSuccess) return CS3D_E_DEVICE;
    if ((p->robin ? run_rhs_robin(p, pd, nrhs, s) : run_rhs(p, pd, slots(p, nrhs), s)) != hipSuccess)
      return CS3D_E_DEVICE;
    if (p->cplx && run_rhs_cx(p, pd, nrhs, s) != hipSuccess) return CS3D_E_DEVICE;
  }
  pd.u = u;
  pd.accumulate = 0;
  if (p->cplx) {
    if (transform_solve_c(p, pd, nrhs, s) != hipSuccess) return CS3D_E_DEVICE;
    p->refine_done = 0;
  } else if (!mixed) {
    if (transform_solve<double>(p, pd, nrhs, s) != hipSuccess) return CS3D_E_DEVICE;
    p->refine_done = 0;
  } else {
    // FP32 transforms + FP64 tridiagonal solves, then refine_steps corrections
    // U += A_mixed^{-1} (F - A U) with the FP64 27-point residual (Section 3.1 operator)
    // r is computed in FP64 and stored in FP32: it only feeds an FP32 correction solve,
    // whose own rounding is larger; the last residual (the convergence check) is a norm only
    // ||F||^2 (stats word 2, the scale of the residual history) comes with the first residual
    float* R = reinterpret_cast<float*>(ws + off_R(p, nrhs));
    if (transform_solve<float>(p, pd, nrhs, s) != hipSuccess) return CS3D_E_DEVICE;
    for (int it = 0; it <= p->d.refine_steps; ++it) {
      const bool last = it == p->d.refine_steps;
      if (mark(p, 5, s) != hipSuccess) return CS3D_E_DEVICE;
      if (residual_pass<float>(p, pd, F, u, last ? nullptr : R, nrhs, 3 + it, s, it == 0 ? 2 : -1) != hipSuccess)
        return CS3D_E_DEVICE;
      if (last) break;
      ProbDev pc = pd;
      pc.F = reinterpret_cast<const double*>(R);
      pc.f32_input = 1;
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

extern "C" cs3d_status cs3d_solve(cs3d_plan p, int nrhs, const double* dev_f, const double* dev_g_lo,
                                  const double* dev_g_hi, double* dev_u, void* hip_stream) {
  return solve_common(p, nrhs, dev_f, 0, dev_g_lo, dev_g_hi, dev_u, hip_stream);
}

// ---------------------------------------------------------------------------
// Static scratch for callers that cannot allocate (cs3d_solve_static).  Every device the
// library runs on holds its own copy of the array until the process ends.  In host code
// the array's name is only a stand-in: its address on a device comes from
// hipGetSymbolAddress with that device current, taken once per device and kept.
// ---------------------------------------------------------------------------
static __device__ __align__(256) unsigned char cs3d_scratch[CS3D_STATIC_SCRATCH_BYTES];

namespace {
constexpr int kMaxDevices = 64;
std::mutex g_scratch_mu;
void* g_scratch_ptr[kMaxDevices] = {};

cs3d_status static_scratch(void** out) {
  int dev = -1;
  if (hipGetDevice(&dev) != hipSuccess || dev < 0 || dev >= kMaxDevices) {
    (void)hipGetLastError();
    return CS3D_E_DEVICE;
  }
  std::lock_guard<std::mutex> lock(g_scratch_mu);
  if (!g_scratch_ptr[dev]) {
    void* ptr = nullptr;
    if (hipGetSymbolAddress(&ptr, HIP_SYMBOL(cs3d_scratch)) != hipSuccess || !ptr) {
      (void)hipGetLastError();
      return CS3D_E_DEVICE;
    }
    g_scratch_ptr[dev] = ptr;
  }
  *out = g_scratch_ptr[dev];
  return CS3D_OK;
}
}  // namespace

extern "C" cs3d_status cs3d_solve_static(cs3d_plan p, int nrhs, const double* dev_f, const double* dev_g_lo,
                                         const double* dev_g_hi, double* dev_u, void* hip_stream) {
  if (!p) return CS3D_E_INVAL;
  if (nrhs < 1 || nrhs > p->d.max_rhs) return CS3D_E_INVAL;
  if (cs3d_workspace_bytes(p, nrhs) > (size_t)CS3D_STATIC_SCRATCH_BYTES) return CS3D_E_TOO_LARGE;
  void* scratch = nullptr;
  const cs3d_status got = static_scratch(&scratch);
  if (got != CS3D_OK) return got;
  // the plan's own workspace (if any) is left alone; the kernels take the scratch address
  void* const ws = p->ws;
  const size_t ws_bytes = p->ws_bytes;
  p->ws = scratch;
  p->ws_bytes = (size_t)CS3D_STATIC_SCRATCH_BYTES;
  p->notime = true;
  const cs3d_status st = solve_common(p, nrhs, dev_f, 0, dev_g_lo, dev_g_hi, dev_u, hip_stream);
  p->ws = ws;
  p->ws_bytes = ws_bytes;
  p->notime = false;
  return st;
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
  if (p->cplx || p->neu || p->robin) return CS3D_E_UNSUPPORTED;
  hipStream_t s = (hipStream_t)hip_stream;
  // F (with the lift) goes into r, then r = F - A U in place
  const ProbDev pd = make_pd(p, assembled ? nullptr : dev_f, dev_g_lo, dev_g_hi, nullptr, dev_r, nrhs);
  if (!assembled && run_rhs(p, pd, nrhs, s) != hipSuccess) return CS3D_E_DEVICE;
  return residual_pass<double>(p, pd, assembled ? dev_f : (const double*)dev_r, dev_u, dev_r, nrhs, -1, s) == hipSuccess
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
    case CS3D_E_TOO_LARGE: return "problem needs more scratch than cs3d_solve_static holds";
    default: return "unknown status";
  }
}

extern "C" const char* cs3d_version(void) { return "cs3d 0.1 (gfx950)"; }


// ---------------------------------------------------------------------------
// Launch-shape choices and the autotuner
// ---------------------------------------------------------------------------
static bool tuning_ok(const cs3d_tuning* t) {
  return t && t->zchunk >= 8 && t->zchunk <= 512 && (t->xpersist == 0 || t->xpersist == 1) &&
         (t->ywpl == 1 || t->ywpl == 2) && (t->order == 0 || t->order == 1) && (t->graph == 0 || t->graph == 1) &&
         (t->yrhs == 1 || t->yrhs == 2 || t->yrhs == 4) && (t->xwpl == 1 || t->xwpl == 2) &&
         (t->pack == 0 || t->pack == 1);
}

static void tuning_out(const Tuning& t, cs3d_tuning* o) {
  o->zchunk = t.zchunk;
  o->xpersist = t.xpersist;
  o->ywpl = t.ywpl;
  o->order = t.order;
  o->graph = t.graph;
  o->yrhs = t.yrhs;
  o->xwpl = t.xwpl;
  o->pack = t.pack;
}

extern "C" cs3d_status cs3d_get_tuning(cs3d_plan p, cs3d_tuning* out) {
  if (!p || !out) return CS3D_E_INVAL;
  tuning_out(p->tune, out);
  return CS3D_OK;
}

extern "C" cs3d_status cs3d_set_tuning(cs3d_plan p, const cs3d_tuning* t) {
  if (!p || !tuning_ok(t)) return CS3D_E_INVAL;
  p->tune.zchunk = t->zchunk;
  p->tune.xpersist = t->xpersist;
  p->tune.ywpl = t->ywpl;
  p->tune.yrhs = t->yrhs;
  p->tune.xwpl = t->xwpl;
  return CS3D_OK;
}

// Mean per-pass device times of `reps` solves with tuning t (after one untimed solve).
static cs3d_status timed_solves(cs3d_plan p, const Tuning& t, int nrhs, const double* f, const double* glo,
                                const double* ghi, double* u, void* s, int reps, double (&stage)[8]) {
  p->tune = t;
  cs3d_status st = cs3d_solve(p, nrhs, f, glo, ghi, u, s);
  if (st != CS3D_OK) return st;
  if ((st = cs3d_reset_timers(p)) != CS3D_OK) return st;
  for (int k = 0; k < reps; ++k)
    if ((st = cs3d_solve(p, nrhs, f, glo, ghi, u, s)) != CS3D_OK) return st;
  cs3d_stats S;
  st = cs3d_get_stats(p, &S);
  if (st == CS3D_E_DEVICE || st == CS3D_E_INVAL) return st;
  for (int k = 0; k < 8; ++k) stage[k] = S.stage_ms[k];
  return CS3D_OK;
}

extern "C" cs3d_status cs3d_autotune(cs3d_plan p, int nrhs, const double* f, const double* glo, const double* ghi,
                                     double* u, void* s, int reps, cs3d_tuning* out_best, double* out_ms) {
  if (!p || reps < 1) return CS3D_E_INVAL;
  Tuning best = p->tune;
  double stage[8];
  cs3d_status st;
  // each choice is judged by the passes it shapes; the others keep their current choice
  struct Axis {
    int Tuning::*field;
    std::vector<int> values;
    std::vector<int> stages;
  };
  std::vector<Axis> axes;
  axes.push_back({&Tuning::zchunk, {16, 32, 64, 128}, {0, 5}});
  axes.push_back({&Tuning::xpersist, {0, 1}, {1, 4}});
  if (p->fx >= 512) axes.push_back({&Tuning::xwpl, {1, 2}, {1, 4}});
  if (p->fy >= 512) axes.push_back({&Tuning::ywpl, {1, 2}, {2, 3}});
  if (nrhs > 1) axes.push_back({&Tuning::yrhs, {1, 2, 4}, {2, 3}});
  for (const Axis& a : axes) {
    double best_t = INFINITY;
    int best_v = best.*(a.field);
    for (int v : a.values) {
      Tuning t = best;
      t.*(a.field) = v;
      if ((st = timed_solves(p, t, nrhs, f, glo, ghi, u, s, reps, stage)) != CS3D_OK) {
        p->tune = best;
        return st;
      }
      double tt = 0.0;
      for (int k : a.stages) tt += stage[k];
      if (tt < best_t) {
        best_t = tt;
        best_v = v;
      }
    }
    best.*(a.field) = best_v;
  }
  if ((st = timed_solves(p, best, nrhs, f, glo, ghi, u, s, reps, stage)) != CS3D_OK) return st;
  p->tune = best;
  if (out_best) tuning_out(best, out_best);
  if (out_ms) {
    double tt = 0.0;
    for (int k = 0; k < kStages; ++k) tt += stage[k];
    *out_ms = tt;
  }
  return CS3D_OK;
}

// ---------------------------------------------------------------------------
// Batches: each pass is one launch over the work items of all members (batch.hpp),
// the five launches captured once into a HIP graph.
// ---------------------------------------------------------------------------
namespace {
enum BatchPass { kPassRhs = 0, kPassXf, kPassYf, kPassYb, kPassXi, kPasses };
}

struct cs3d_batch_s {
  int n = 0;
  std::vector<cs3d_plan> plans;  // member tables (weights, cosines, twiddles)
  std::vector<size_t> offs;      // workspace offset of each member
  size_t bytes = 0;
  void* ws = nullptr;
  int general = 0;               // kernel variant: 0 = FFT lengths 64..256 only,
                                 // 1 = every transform (FFT up to 1024 and dense sums)
  Tuning tune;
  std::vector<const double*> cur_f;
  std::vector<double*> cur_u;
  bool have_ptrs = false;        // dP holds the descriptors of cur_f / cur_u
  ProbDev* hP = nullptr;         // pinned staging of the member descriptors
  ProbDev* dP = nullptr;
  int* dlist = nullptr;          // per pass: start[n + 1], perm[n]
  unsigned long long* dstats = nullptr;  // n x kStatsWords
  int total[kPasses] = {};
  int grid[kPasses] = {};
  size_t lds[kPasses] = {};
  bool ready = false;            // work lists and grids match tune
  hipEvent_t up_ev = nullptr;    // the last upload of hP has been read
  bool up_pending = false;
  hipStream_t cap = nullptr;     // capture stream
  hipGraph_t graph = nullptr;
  hipGraphExec_t exec = nullptr;
  hipEvent_t ev[kPasses + 1] = {};
  hipEvent_t tev0 = nullptr, tev1 = nullptr;
  hipStream_t last_stream = nullptr;
  bool timed = false, staged = false;
};

static int list_stride(const cs3d_batch b) { return 2 * b->n + 1; }

// relative cost of one line transform of N points (FFT of length f, or dense sums)
static double line_cost(int f, int N) { return f ? f * std::log2((double)f) : 0.25 * (double)N * N; }


// LDS elements (doubles) of one line buffer of the y passes, as line_buf_elems for T = double
// with the default waves per line; at 1024 points the larger of the forward pass's buffer
// (paired exchanges) and the backward pass's, since both passes share the size
static size_t line_elems(int f, int N) {
  constexpr int W = default_wpl<1024>();
  switch (f) {
    case 64: return line_buf_elems<double, 64, 1>(N);
    case 128: return line_buf_elems<double, 128, 1>(N);
    case 256: return line_buf_elems<double, 256, 1>(N);
    case 512: return line_buf_elems<double, 512, default_wpl<512>()>(N);
    case 1024: return std::max(line_buf_elems<double, 1024, W, ypair<double, 1024, W, true>()>(N),
                               line_buf_elems<double, 1024, W, ypair<double, 1024, W, false>()>(N));
    default: return line_buf_elems<double, 0, 1>(N);
  }
}

// as above for the x passes (one wave per line)
static size_t line_elems_x(int f, int N) {
  switch (f) {
    case 512: return line_buf_elems<double, 512, 1>(N);
    case 1024: return line_buf_elems<double, 1024, 1>(N);
    default: return line_elems(f, N);
  }
}

template <int MAXM, bool DENSE>
static cs3d_status batch_grids_t(cs3d_batch b) {
  size_t lx = 0, ly = 0;
  const int pk = b->tune.pack;
  for (cs3d_plan q : b->plans) {
    const int tj = x_tile_lines(q->fx, pk);
    const size_t ts = (size_t)tile_stride(q->d.nx, tj);
    const size_t bx = line_elems_x(q->fx, q->d.nx);
    lx = std::max(lx, (size_t)tj * std::max(bx, ts) * 8);
    ly = std::max(ly, (size_t)(kBlockY / y_lanes(q->fy, pk)) * line_elems(q->fy, q->d.ny) * 8);
  }
  const size_t tw = (size_t)tw_entries<MAXM>() * sizeof(cx<double>);
  b->lds[kPassRhs] = 0;
  b->lds[kPassXf] = b->lds[kPassXi] = tw + lx;
  b->lds[kPassYf] = b->lds[kPassYb] = tw + ly;
  const void* kern[kPasses] = {
      reinterpret_cast<const void*>(kb_rhs),
      pk ? reinterpret_cast<const void*>(kb_x<double, MAXM, DENSE, true, true>)
         : reinterpret_cast<const void*>(kb_x<double, MAXM, DENSE, true, false>),
      pk ? reinterpret_cast<const void*>(kb_y<double, MAXM, DENSE, true, true>)
         : reinterpret_cast<const void*>(kb_y<double, MAXM, DENSE, true, false>),
      pk ? reinterpret_cast<const void*>(kb_y<double, MAXM, DENSE, false, true>)
         : reinterpret_cast<const void*>(kb_y<double, MAXM, DENSE, false, false>),
      pk ? reinterpret_cast<const void*>(kb_x<double, MAXM, DENSE, false, true>)
         : reinterpret_cast<const void*>(kb_x<double, MAXM, DENSE, false, false>)};
  const int threads[kPasses] = {kRThreadsBatch, 64 * kTileJ, kBlockY, kBlockY, 64 * kTileJ};
  for (int k = 0; k < kPasses; ++k) {
    if (b->lds[k] > 160 * 1024) return CS3D_E_UNSUPPORTED;
    if (b->lds[k] > 64 * 1024 &&
        hipFuncSetAttribute(kern[k], hipFuncAttributeMaxDynamicSharedMemorySize, (int)b->lds[k]) != hipSuccess)
      return CS3D_E_DEVICE;
    b->grid[k] = b->total[k] > 0 ? resident_blocks(kern[k], threads[k], b->lds[k], b->total[k]) : 0;
  }
  return CS3D_OK;
}

// Work lists of every pass (member order and item prefix sums) and the resident grids.
static cs3d_status batch_prepare(cs3d_batch b) {
  const int n = b->n;
  std::vector<int> host((size_t)kPasses * list_stride(b));
  for (int pass = 0; pass < kPasses; ++pass) {
    std::vector<long long> items(n);
    std::vector<double> cost(n);
    for (int i = 0; i < n; ++i) {
      const cs3d_plan q = b->plans[i];
      const int nx = q->d.nx, ny = q->d.ny, nz = q->d.nz;
      switch (pass) {
        case kPassRhs:
          items[i] = rhs_items(nx, ny, nz, b->tune.zchunk);
          cost[i] = std::min(nz, b->tune.zchunk);
          break;
        case kPassXf:
        case kPassXi:
          // (a packed item holds more lines on more lanes, in about the time of an unpacked one)
          items[i] = x_items(q->ldy, nz, x_tile_lines(q->fx, b->tune.pack));
          cost[i] = line_cost(q->fx, nx);
          break;
        default:
          items[i] = y_items(nx, kBlockY / y_lanes(q->fy, b->tune.pack));
          cost[i] = nz * line_cost(q->fy, ny) * 64 / y_lanes(q->fy, 0);
          break;
      }
    }
    std::vector<int> perm(n);
    for (int i = 0; i < n; ++i) perm[i] = i;
    if (b->tune.order)
      std::stable_sort(perm.begin(), perm.end(), [&](int a, int c) { return cost[a] > cost[c]; });
    int* st = host.data() + (size_t)pass * list_stride(b);
    long long acc = 0;
    st[0] = 0;
    for (int k = 0; k < n; ++k) {
      acc += items[perm[k]];
      if (acc > 0x7FFFFFFFLL) return CS3D_E_UNSUPPORTED;
      st[k + 1] = (int)acc;
      st[n + 1 + k] = perm[k];
    }
    b->total[pass] = (int)acc;
  }
  if (hipMemcpy(b->dlist, host.data(), host.size() * sizeof(int), hipMemcpyHostToDevice) != hipSuccess)
    return CS3D_E_DEVICE;
  const cs3d_status st = b->general ? batch_grids_t<1024, true>(b) : batch_grids_t<256, false>(b);
  if (st != CS3D_OK) return st;
  b->ready = true;
  return CS3D_OK;
}

template <int MAXM, bool DENSE, bool PACK>
static hipError_t batch_pass_t(const cs3d_batch b, int pass, hipStream_t s) {
  if (b->total[pass] == 0) return hipSuccess;
  const int* lst = b->dlist + (size_t)pass * list_stride(b);
  const BatchArgs a{b->dP, lst, lst + b->n + 1, b->n, b->total[pass]};
  const dim3 g(b->grid[pass]);
  switch (pass) {
    case kPassRhs: hipLaunchKernelGGL(kb_rhs, g, dim3(kRThreadsBatch), 0, s, a); break;
    case kPassXf:
      hipLaunchKernelGGL((kb_x<double, MAXM, DENSE, true, PACK>), g, dim3(64 * kTileJ), b->lds[pass], s, a);
      break;
    case kPassYf:
      hipLaunchKernelGGL((kb_y<double, MAXM, DENSE, true, PACK>), g, dim3(kBlockY), b->lds[pass], s, a);
      break;
    case kPassYb:
      hipLaunchKernelGGL((kb_y<double, MAXM, DENSE, false, PACK>), g, dim3(kBlockY), b->lds[pass], s, a);
      break;
    default:
      hipLaunchKernelGGL((kb_x<double, MAXM, DENSE, false, PACK>), g, dim3(64 * kTileJ), b->lds[pass], s, a);
      break;
  }
  return hipGetLastError();
}

static hipError_t batch_pass(const cs3d_batch b, int pass, hipStream_t s) {
  if (b->general) return b->tune.pack ? batch_pass_t<1024, true, true>(b, pass, s) : batch_pass_t<1024, true, false>(b, pass, s);
  return b->tune.pack ? batch_pass_t<256, false, true>(b, pass, s) : batch_pass_t<256, false, false>(b, pass, s);
}

// statistics reset + the five passes; with events between the passes when `marks`
static hipError_t batch_launch(const cs3d_batch b, hipStream_t s, bool marks) {
  hipError_t e;
  const int words = b->n * kStatsWords;
  hipLaunchKernelGGL(kb_stats_reset, dim3((words + 255) / 256), dim3(256), 0, s, b->dstats, b->n);
  if ((e = hipGetLastError()) != hipSuccess) return e;
  for (int k = 0; k < kPasses; ++k) {
    if ((e = batch_pass(b, k, s)) != hipSuccess) return e;
    if (marks && (e = hipEventRecord(b->ev[k + 1], s)) != hipSuccess) return e;
  }
  return hipSuccess;
}

static void batch_drop_graph(cs3d_batch b) {
  if (b->exec) (void)hipGraphExecDestroy(b->exec);
  if (b->graph) (void)hipGraphDestroy(b->graph);
  b->exec = nullptr;
  b->graph = nullptr;
}

static cs3d_status batch_capture(cs3d_batch b) {
  if (!b->cap && hipStreamCreateWithFlags(&b->cap, hipStreamNonBlocking) != hipSuccess) return CS3D_E_DEVICE;
  if (hipStreamBeginCapture(b->cap, hipStreamCaptureModeThreadLocal) != hipSuccess) return CS3D_E_DEVICE;
  const hipError_t e = batch_launch(b, b->cap, false);
  hipGraph_t g = nullptr;
  const hipError_t e2 = hipStreamEndCapture(b->cap, &g);
  if (e != hipSuccess || e2 != hipSuccess || !g) {
    if (g) (void)hipGraphDestroy(g);
    (void)hipGetLastError();
    return CS3D_E_DEVICE;
  }
  b->graph = g;
  if (hipGraphInstantiate(&b->exec, g, nullptr, nullptr, 0) != hipSuccess) {
    batch_drop_graph(b);
    return CS3D_E_DEVICE;
  }
  return CS3D_OK;
}

static void batch_free(cs3d_batch b) {
  if (!b) return;
  if (b->last_stream) (void)hipStreamSynchronize(b->last_stream);
  if (b->up_pending) (void)hipEventSynchronize(b->up_ev);
  batch_drop_graph(b);
  if (b->cap) (void)hipStreamDestroy(b->cap);
  for (hipEvent_t e : b->ev)
    if (e) (void)hipEventDestroy(e);
  if (b->tev0) (void)hipEventDestroy(b->tev0);
  if (b->tev1) (void)hipEventDestroy(b->tev1);
  if (b->up_ev) (void)hipEventDestroy(b->up_ev);
  if (b->dP) (void)hipFree(b->dP);
  if (b->dlist) (void)hipFree(b->dlist);
  if (b->dstats) (void)hipFree(b->dstats);
  if (b->hP) (void)hipHostFree(b->hP);
  for (cs3d_plan q : b->plans) cs3d_plan_destroy(q);
  delete b;
}

extern "C" cs3d_status cs3d_batch_create(int n, const cs3d_desc* descs, void* hip_stream, cs3d_batch* out) {
  if (!out || n < 1 || !descs) return CS3D_E_INVAL;
  *out = nullptr;
  for (int i = 0; i < n; ++i) {  // every description is checked before any allocation
    cs3d_desc d = descs[i];
    d.max_rhs = 1;
    const cs3d_status st = validate(&d);
    if (st != CS3D_OK) return st;
    if (d.scheme == CS3D_WEIGHTS) return CS3D_E_INVAL;
    if (d.precision != CS3D_FP64 || d.k2_im || d.sides != CS3D_SIDES_DIRICHLET || d.zfaces != CS3D_ZFACES_DIRICHLET)
      return CS3D_E_UNSUPPORTED;
  }
  cs3d_batch b = new (std::nothrow) cs3d_batch_s();
  if (!b) return CS3D_E_NOMEM;
  b->n = n;
  size_t off = 0;
  bool small = true;  // every transform an FFT of length 64..256
  for (int i = 0; i < n; ++i) {
    cs3d_desc d = descs[i];
    d.max_rhs = 1;
    cs3d_plan p = nullptr;
    const cs3d_status st = cs3d_plan_create(&d, hip_stream, &p);
    if (st != CS3D_OK) {
      batch_free(b);
      return st;
    }
    b->plans.push_back(p);
    b->offs.push_back(off);
    off += round256(cs3d_workspace_bytes(p, 1));
    small = small && p->fx && p->fy && p->fx <= 256 && p->fy <= 256;
  }
  b->bytes = off;
  b->general = small ? 0 : 1;
  b->cur_f.assign(n, nullptr);
  b->cur_u.assign(n, nullptr);
  bool ok = hipHostMalloc(reinterpret_cast<void**>(&b->hP), n * sizeof(ProbDev)) == hipSuccess &&
            dalloc(&b->dP, n) == hipSuccess && dalloc(&b->dlist, (size_t)kPasses * list_stride(b)) == hipSuccess &&
            dalloc(&b->dstats, (size_t)n * kStatsWords) == hipSuccess &&
            hipEventCreateWithFlags(&b->up_ev, hipEventDisableTiming) == hipSuccess &&
            hipEventCreate(&b->tev0) == hipSuccess && hipEventCreate(&b->tev1) == hipSuccess;
  for (hipEvent_t& e : b->ev) ok = ok && hipEventCreate(&e) == hipSuccess;
  if (!ok) {
    (void)hipGetLastError();
    batch_free(b);
    return CS3D_E_DEVICE;
  }
  *out = b;
  return CS3D_OK;
}

extern "C" size_t cs3d_batch_workspace_bytes(cs3d_batch b) { return b ? b->bytes : 0; }

extern "C" cs3d_status cs3d_batch_set_workspace(cs3d_batch b, void* dev, size_t bytes) {
  if (!b || !dev || ((uintptr_t)dev & 255)) return CS3D_E_INVAL;
  if (bytes < b->bytes) return CS3D_E_WORKSPACE;
  if (b->last_stream) (void)hipStreamSynchronize(b->last_stream);
  b->ws = dev;
  for (size_t i = 0; i < b->plans.size(); ++i)
    cs3d_set_workspace(b->plans[i], (char*)dev + b->offs[i], cs3d_workspace_bytes(b->plans[i], 1));
  b->have_ptrs = false;  // the descriptors carry the workspace addresses
  return CS3D_OK;
}

static cs3d_status batch_solve_impl(cs3d_batch b, const double* const* f, double* const* u, hipStream_t s) {
  if (!b || !f || !u) return CS3D_E_INVAL;
  for (int i = 0; i < b->n; ++i)
    if (!f[i] || !u[i]) return CS3D_E_INVAL;
  if (!b->ws) return CS3D_E_WORKSPACE;
  cs3d_status st;
  if (!b->ready && (st = batch_prepare(b)) != CS3D_OK) return st;
  bool changed = !b->have_ptrs;
  for (int i = 0; i < b->n && !changed; ++i) changed = f[i] != b->cur_f[i] || u[i] != b->cur_u[i];
  if (changed) {
    if (b->up_pending && hipEventSynchronize(b->up_ev) != hipSuccess) return CS3D_E_DEVICE;
    for (int i = 0; i < b->n; ++i) {
      // the FP64 path: the RHS pass writes F into u, which the inverse x pass overwrites last
      ProbDev pd = make_pd(b->plans[i], f[i], nullptr, nullptr, u[i], u[i], 1);
      pd.stats = b->dstats + (size_t)i * kStatsWords;
      pd.zchunk = b->tune.zchunk;
      pd.accumulate = 0;
      b->hP[i] = pd;
      b->cur_f[i] = f[i];
      b->cur_u[i] = u[i];
    }
    if (hipMemcpyAsync(b->dP, b->hP, b->n * sizeof(ProbDev), hipMemcpyHostToDevice, s) != hipSuccess ||
        hipEventRecord(b->up_ev, s) != hipSuccess)
      return CS3D_E_DEVICE;
    b->up_pending = true;
    b->have_ptrs = true;
  }
  if (b->tune.graph) {
    if (!b->exec && (st = batch_capture(b)) != CS3D_OK) return st;
    if (hipEventRecord(b->ev[0], s) != hipSuccess || hipGraphLaunch(b->exec, s) != hipSuccess ||
        hipEventRecord(b->ev[kPasses], s) != hipSuccess)
      return CS3D_E_DEVICE;
    b->staged = false;
  } else {
    if (hipEventRecord(b->ev[0], s) != hipSuccess || batch_launch(b, s, true) != hipSuccess) return CS3D_E_DEVICE;
    b->staged = true;
  }
  b->last_stream = s;
  b->timed = true;
  return CS3D_OK;
}

extern "C" cs3d_status cs3d_batch_solve(cs3d_batch b, const double* const* f, double* const* u, void* s) {
  return batch_solve_impl(b, f, u, (hipStream_t)s);
}

static cs3d_status batch_sync(cs3d_batch b) {
  if (b->last_stream && hipStreamSynchronize(b->last_stream) != hipSuccess) return CS3D_E_DEVICE;
  if (!b->last_stream && hipDeviceSynchronize() != hipSuccess) return CS3D_E_DEVICE;
  return CS3D_OK;
}

static cs3d_status batch_timing(cs3d_batch b, cs3d_stats* out) {
  for (double& v : out->residual_history) v = NAN;
  if (!b->timed) return CS3D_OK;
  float ms = 0.f;
  if (hipEventElapsedTime(&ms, b->ev[0], b->ev[kPasses]) != hipSuccess) return CS3D_E_DEVICE;
  out->last_solve_ms = ms;
  if (b->staged) {
    out->stage_count = kPasses;
    out->timed_solves = 1;
    for (int k = 0; k < kPasses; ++k) {
      if (hipEventElapsedTime(&ms, b->ev[k], b->ev[k + 1]) != hipSuccess) return CS3D_E_DEVICE;
      out->stage_ms[k] = ms;
    }
  }
  return CS3D_OK;
}

extern "C" cs3d_status cs3d_batch_get_stats(cs3d_batch b, cs3d_stats* out) {
  if (!b || !out) return CS3D_E_INVAL;
  std::memset(out, 0, sizeof(*out));
  cs3d_status st = batch_sync(b);
  if (st != CS3D_OK) return st;
  std::vector<unsigned long long> h((size_t)b->n * kStatsWords);
  if (hipMemcpy(h.data(), b->dstats, h.size() * 8, hipMemcpyDeviceToHost) != hipSuccess) return CS3D_E_DEVICE;
  double mn = INFINITY;
  long long bad = 0;
  for (int i = 0; i < b->n; ++i) {
    double v;
    std::memcpy(&v, &h[(size_t)i * kStatsWords], 8);
    mn = std::fmin(mn, v);
    bad += (long long)h[(size_t)i * kStatsWords + 1];
  }
  out->min_abs_pivot = mn;
  out->bad_pivots = bad;
  if ((st = batch_timing(b, out)) != CS3D_OK) return st;
  return bad ? CS3D_E_SINGULAR : CS3D_OK;
}

extern "C" cs3d_status cs3d_batch_member_stats(cs3d_batch b, int i, cs3d_stats* out) {
  if (!b || !out || i < 0 || i >= b->n) return CS3D_E_INVAL;
  std::memset(out, 0, sizeof(*out));
  cs3d_status st = batch_sync(b);
  if (st != CS3D_OK) return st;
  unsigned long long h[2];
  if (hipMemcpy(h, b->dstats + (size_t)i * kStatsWords, sizeof(h), hipMemcpyDeviceToHost) != hipSuccess)
    return CS3D_E_DEVICE;
  std::memcpy(&out->min_abs_pivot, &h[0], 8);
  out->bad_pivots = (int64_t)h[1];
  if ((st = batch_timing(b, out)) != CS3D_OK) return st;
  return h[1] ? CS3D_E_SINGULAR : CS3D_OK;
}

extern "C" cs3d_status cs3d_batch_get_tuning(cs3d_batch b, cs3d_tuning* out) {
  if (!b || !out) return CS3D_E_INVAL;
  tuning_out(b->tune, out);
  return CS3D_OK;
}

extern "C" cs3d_status cs3d_batch_set_tuning(cs3d_batch b, const cs3d_tuning* t) {
  if (!b || !tuning_ok(t)) return CS3D_E_INVAL;
  if (b->last_stream && hipStreamSynchronize(b->last_stream) != hipSuccess) return CS3D_E_DEVICE;
  const bool lists = t->zchunk != b->tune.zchunk || t->order != b->tune.order || t->pack != b->tune.pack;
  b->tune.zchunk = t->zchunk;
  b->tune.order = t->order;
  b->tune.graph = t->graph;
  b->tune.pack = t->pack;
  if (lists) {
    b->ready = false;
    b->have_ptrs = false;  // zchunk is in the descriptors
    batch_drop_graph(b);   // grids and totals are baked into the graph
  }
  return CS3D_OK;
}

extern "C" cs3d_status cs3d_batch_autotune(cs3d_batch b, const double* const* f, double* const* u, void* stream,
                                           int reps, cs3d_tuning* out_best, double* out_ms) {
  if (!b || reps < 1) return CS3D_E_INVAL;
  hipStream_t s = (hipStream_t)stream;
  cs3d_tuning best;
  tuning_out(b->tune, &best);
  cs3d_status st;
  // per-pass timings of `reps` solves launched pass by pass
  auto run = [&](const cs3d_tuning& t, double (&stage)[kPasses]) -> cs3d_status {
    cs3d_tuning u0 = t;
    u0.graph = 0;
    cs3d_status r = cs3d_batch_set_tuning(b, &u0);
    if (r != CS3D_OK) return r;
    for (double& v : stage) v = 0.0;
    for (int k = 0; k <= reps; ++k) {
      if ((r = batch_solve_impl(b, f, u, s)) != CS3D_OK) return r;
      cs3d_stats S;
      r = cs3d_batch_get_stats(b, &S);
      if (r == CS3D_E_DEVICE) return r;
      if (k > 0)  // the first solve is a warm-up
        for (int q = 0; q < kPasses; ++q) stage[q] += S.stage_ms[q] / reps;
    }
    return CS3D_OK;
  };
  double stage[kPasses];
  // zchunk shapes the RHS pass only
  double bt = INFINITY;
  int bz = best.zchunk;
  for (int z : {16, 32, 64, 128}) {
    cs3d_tuning t = best;
    t.zchunk = z;
    if ((st = run(t, stage)) != CS3D_OK) return st;
    if (stage[kPassRhs] < bt) {
      bt = stage[kPassRhs];
      bz = z;
    }
  }
  best.zchunk = bz;
  // packed lines shape the transform passes (x and y, both directions)
  bt = INFINITY;
  int bp = best.pack;
  for (int pk : {0, 1}) {
    cs3d_tuning t = best;
    t.pack = pk;
    if ((st = run(t, stage)) != CS3D_OK) return st;
    const double tt = stage[kPassXf] + stage[kPassYf] + stage[kPassYb] + stage[kPassXi];
    if (tt < bt) {
      bt = tt;
      bp = pk;
    }
  }
  best.pack = bp;
  // the member order shapes every pass
  bt = INFINITY;
  int bo = best.order;
  for (int o : {0, 1}) {
    cs3d_tuning t = best;
    t.order = o;
    if ((st = run(t, stage)) != CS3D_OK) return st;
    double tt = 0.0;
    for (double v : stage) tt += v;
    if (tt < bt) {
      bt = tt;
      bo = o;
    }
  }
  best.order = bo;
  best.graph = 1;
  if ((st = cs3d_batch_set_tuning(b, &best)) != CS3D_OK) return st;
  // graph replay timing of the final choice
  if ((st = batch_solve_impl(b, f, u, s)) != CS3D_OK) return st;
  if (hipEventRecord(b->tev0, s) != hipSuccess) return CS3D_E_DEVICE;
  for (int k = 0; k < reps; ++k)
    if ((st = batch_solve_impl(b, f, u, s)) != CS3D_OK) return st;
  if (hipEventRecord(b->tev1, s) != hipSuccess || hipEventSynchronize(b->tev1) != hipSuccess) return CS3D_E_DEVICE;
  float ms = 0.f;
  if (hipEventElapsedTime(&ms, b->tev0, b->tev1) != hipSuccess) return CS3D_E_DEVICE;
  if (out_best) *out_best = best;
  if (out_ms) *out_ms = ms / reps;
  return CS3D_OK;
}

extern "C" cs3d_status cs3d_batch_destroy(cs3d_batch b) {
  batch_free(b);
  return CS3D_OK;
}
