// kernels.hpp - the four streaming passes of the direct solve (Section 3.6) on CDNA4.
//
//  K1 fwd_x   : RHS operator (Sections 3.2-3.5) + z-face lift + DST-I along x of
//               16 x-lines per workgroup; the results are transposed through LDS and
//               stored as y-lines  G[l][n][j]  (j fastest, 128-byte rows).
//  K2 fwd_y   : one wavefront per x-mode n marches l = 1..N_z: DST-I along y of the
//               line G[l][n][:], modal eigenvalues lambda^{-,0,+} from the row weights
//               (built on the fly), forward elimination of the N_y tridiagonal systems
//               (one mode m per lane slot).  d'_l is stored in place, c'_l once per plan
//               column in C.
//  K3 back_y  : the same wavefronts march l = N_z..1: back substitution
//               W_l = d'_l - c'_l W_{l+1}, inverse DST-I along y, stored in place.
//  K4 inv_x   : 16 y-lines per workgroup are transposed back through LDS, inverse
//               DST-I along x, scaled by 4/((N_x+1)(N_y+1)) and stored as u (x fastest).
//
// The DST-I is its own inverse up to the factor (N+1)/2, so the four line
// transforms are the same routine and the orthonormal V of Section 3.6 is
// recovered by the single final scale.
#pragma once
#include "wave_dst.hpp"

namespace cs3d {

enum SchemeId : int { kHelm2 = 2, kHelm4 = 4, kHelm6 = 6, kCd4 = 14, kWeights = 99 };

constexpr int kTileJ = 16;     // y-lines per K1/K4 workgroup (128-byte rows of doubles)
constexpr int kWavesY = 4;     // x-modes (wavefronts) per K2/K3 workgroup

struct ProbDev {
  int nx, ny, nz;
  int Mx, My;          // N+1 per axis
  int ldy;             // row length of a y-line in G / C (multiple of 16, >= ny+1)
  int scheme;
  double hx, hy, hz, gamma;
  double scale;        // 4 / (Mx My)
  const double* W;     // [nz][3][4] row weights
  const double* LC;    // [nz][3][4] modal coefficients (Z, B, C, A) of each row and offset:
                       // lambda = Z + s_n B + s_m (C + A s_n),  s = 1 - cos
  const double* k2;    // [nz+2]
  const double* k2z;   // [nz+2]
  const double* ctx;   // 1 - cos(pi n/Mx), n = 1..nx   [nx]
  const double* cty;   // 1 - cos(pi m/My), m = 1..ny   [ny]
  const double2* twx;  // exp(-i pi k/Mx), k < 2 Mx  (FFT path)
  const double2* twy;
  const double* sinx;  // sin(pi r/Mx), r < 2 Mx      (dense path)
  const double* siny;
  // data (per right-hand side strides in elements)
  const double* f;     // closed grid, or interior F when assembled
  long long f_stride;
  const double* glo;   // closed planes or null
  const double* ghi;
  long long g_stride;
  double* u;           // interior
  long long u_stride;
  void* G;             // [nrhs][nz][nx][ldy] of the transform type
  long long G_stride;
  double* C;           // [nz][nx][ldy]   c' of the tridiagonal LU
  unsigned long long* stats;  // [0] = bits of min |pivot|, [1] = count of bad pivots
  int assembled;
};

template <int M>
struct Tx {
  static constexpr int NS = FftGeom<M>::R;
};
template <>
struct Tx<0> {
  static constexpr int NS = kDenseSlots;
};

template <typename T, int M>
__device__ __forceinline__ void line_dst(T* buf, int N, T (&out)[Tx<M>::NS], int lane,
                                         const double2* tw, const double* sintab) {
  if constexpr (M == 0) {
    dst_dense<T>(buf, N, out, lane, sintab);
  } else {
    dst_fft<T, M>(buf, out, lane, tw);
  }
}

template <int M>
__device__ __forceinline__ int line_mode(int lane, int s, int N) {
  if constexpr (M == 0) {
    return dense_mode(lane, s, N);
  } else {
    return fft_mode<M>(lane, s);
  }
}

// elements of T in one wave's LDS line region
template <typename T, int M>
__host__ __device__ constexpr int region_elems(int N) {
  return M ? (M * 8) / (int)sizeof(T) : ((N + 1 + 63) / 64) * 64;
}

// ---------------------------------------------------------------------------
// RHS operator at interior point (i, j, l) from f on the closed grid.
// ---------------------------------------------------------------------------
__device__ __forceinline__ double d4_axis(const double* c, long long s, int i, int n) {
  // fourth difference along one axis: central inside, one-sided 6-point at the
  // first and last interior layer (needs n >= 4)
  if (i >= 2 && i <= n - 1)
    return c[-2 * s] - 4.0 * c[-s] + 6.0 * c[0] - 4.0 * c[s] + c[2 * s];
  if (i == 1)
    return 2.0 * c[-s] - 9.0 * c[0] + 16.0 * c[s] - 14.0 * c[2 * s] + 6.0 * c[3 * s] - c[4 * s];
  return 2.0 * c[s] - 9.0 * c[0] + 16.0 * c[-s] - 14.0 * c[-2 * s] + 6.0 * c[-3 * s] - c[-4 * s];
}

__device__ __forceinline__ double rhs_point(const ProbDev& p, const double* __restrict__ f, int i,
                                            int j, int l) {
  const long long sy = p.nx + 2, sz = (long long)(p.nx + 2) * (p.ny + 2);
  const double* c = f + i + sy * j + sz * l;
  const double f0 = c[0];
  const double hz2 = p.hz * p.hz;
  if (p.scheme == kHelm2) return hz2 * f0;
  const double d2x = c[-1] + c[1] - 2.0 * f0;
  const double d2y = c[-sy] + c[sy] - 2.0 * f0;
  const double d2z = c[-sz] + c[sz] - 2.0 * f0;
  if (p.scheme == kHelm4) return hz2 * (f0 + (d2x + d2y + d2z) * (1.0 / 12.0));
  if (p.scheme == kCd4) {
    const double dz1 = 0.5 * (c[sz] - c[-sz]);
    return hz2 * (f0 + (d2x + d2y) * (1.0 / 12.0) + (p.hz * p.gamma * dz1 + d2z) * (1.0 / 12.0));
  }
  // kHelm6: f + h^2/12 sum d2 - h^4/240 sum d4 + h^4/90 sum d2d2 - h^2 k^2 f/20
  //         + h^4 (k^2)_z f_z / 60, every difference undivided (h folded in).
  const double d4 = d4_axis(c, 1, i, p.nx) + d4_axis(c, sy, j, p.ny) + d4_axis(c, sz, l, p.nz);
  const double exy = c[-sy - 1] + c[-sy + 1] + c[sy - 1] + c[sy + 1];
  const double exz = c[-sz - 1] + c[-sz + 1] + c[sz - 1] + c[sz + 1];
  const double eyz = c[-sz - sy] + c[-sz + sy] + c[sz - sy] + c[sz + sy];
  const double ax = c[-1] + c[1], ay = c[-sy] + c[sy], az = c[-sz] + c[sz];
  const double dxy = exy - 2.0 * (ax + ay) + 4.0 * f0;
  const double dxz = exz - 2.0 * (ax + az) + 4.0 * f0;
  const double dyz = eyz - 2.0 * (ay + az) + 4.0 * f0;
  const double h = p.hz;
  const double kl = p.k2[l], kzl = p.k2z[l];
  return hz2 * (f0 + (d2x + d2y + d2z) * (1.0 / 12.0) - d4 * (1.0 / 240.0) +
                (dxy + dxz + dyz) * (1.0 / 90.0) - h * h * kl * f0 * (1.0 / 20.0) +
                h * h * h * kzl * (c[sz] - c[-sz]) * (1.0 / 120.0));
}

// in-plane 9-point stencil of weights w = (a, b, c, d) on a closed plane at (i, j)
__device__ __forceinline__ double plane9(const double* __restrict__ w, const double* __restrict__ P,
                                         int nx, int i, int j) {
  const long long sy = nx + 2;
  const double* c = P + i + sy * j;
  return w[0] * (c[-sy - 1] + c[-sy + 1] + c[sy - 1] + c[sy + 1]) + w[1] * (c[-1] + c[1]) +
         w[2] * (c[-sy] + c[sy]) + w[3] * c[0];
}

__device__ __forceinline__ double assembled_rhs(const ProbDev& p, int r, int i, int j, int l) {
  if (p.assembled)
    return p.f[r * p.f_stride + (i - 1) + (long long)p.nx * ((j - 1) + (long long)p.ny * (l - 1))];
  double F = rhs_point(p, p.f + r * p.f_stride, i, j, l);
  if (l == 1 && p.glo) F -= plane9(p.W + 0, p.glo + r * p.g_stride, p.nx, i, j);
  if (l == p.nz && p.ghi) F -= plane9(p.W + (p.nz - 1) * 12 + 8, p.ghi + r * p.g_stride, p.nx, i, j);
  return F;
}

// ---------------------------------------------------------------------------
// K1: RHS + lift + DST along x, transposed store into y-lines.
// ---------------------------------------------------------------------------
template <typename T, int MX>
__global__ void __launch_bounds__(1024) k_fwd_x(ProbDev p) {
  extern __shared__ double smem_raw[];
  T* smem = reinterpret_cast<T*>(smem_raw);
  constexpr int NS = Tx<MX>::NS;
  const int jt = blockIdx.x, l = blockIdx.y + 1, r = blockIdx.z;
  const int w = threadIdx.x >> 6, lane = threadIdx.x & 63;
  const int reg = region_elems<T, MX>(p.nx);
  T* buf = smem + w * reg;
  const int j = jt * kTileJ + w;
  const bool active = (j >= 1 && j <= p.ny);
  T out[NS];
  if (active) {
    if (lane == 0) buf[0] = (T)0;
    for (int i = 1 + lane; i <= p.nx; i += 64) buf[i] = (T)assembled_rhs(p, r, i, j, l);
    wave_sync();
    line_dst<T, MX>(buf, p.nx, out, lane, p.twx, p.sinx);
  }
  __syncthreads();
  // tile[n-1][jj ^ ((n-1) & 15)]
  if (active) {
#pragma unroll
    for (int s = 0; s < NS; ++s) {
      const int n = line_mode<MX>(lane, s, p.nx);
      if (n > 0) smem[(n - 1) * kTileJ + (w ^ ((n - 1) & 15))] = out[s];
    }
  } else {
    for (int n = 1 + lane; n <= p.nx; n += 64) smem[(n - 1) * kTileJ + (w ^ ((n - 1) & 15))] = (T)0;
  }
  __syncthreads();
  T* G = reinterpret_cast<T*>(p.G) + r * p.G_stride + (long long)(l - 1) * p.nx * p.ldy + jt * kTileJ;
  for (int idx = threadIdx.x; idx < p.nx * kTileJ; idx += blockDim.x) {
    const int n0 = idx / kTileJ, jj = idx % kTileJ;
    G[(long long)n0 * p.ldy + jj] = smem[n0 * kTileJ + (jj ^ (n0 & 15))];
  }
}

// ---------------------------------------------------------------------------
// K2: DST along y + modal eigenvalues + forward elimination (one wave per x-mode).
// ---------------------------------------------------------------------------
__device__ __forceinline__ void record_pivot(double piv, double& minpiv, unsigned& bad) {
  const double a = fabs(piv);
  if (!(a > 0.0) || !isfinite(a)) {
    ++bad;
  } else if (a < minpiv) {
    minpiv = a;
  }
}

__device__ __forceinline__ void flush_stats(const ProbDev& p, double minpiv, unsigned bad) {
  // wave reduction, then one atomic per wave (vector memory atomics)
  for (int off = 32; off > 0; off >>= 1) {
    minpiv = fmin(minpiv, __shfl_xor(minpiv, off, 64));
    bad += __shfl_xor(bad, off, 64);
  }
  if ((threadIdx.x & 63) == 0) {
    if (minpiv < 1.0e308) atomicMin(&p.stats[0], (unsigned long long)__double_as_longlong(minpiv));
    if (bad) atomicAdd(&p.stats[1], (unsigned long long)bad);
  }
}

template <typename T, int MY>
__global__ void __launch_bounds__(64 * kWavesY) k_fwd_y(ProbDev p) {
  extern __shared__ double smem_raw[];
  T* smem = reinterpret_cast<T*>(smem_raw);
  constexpr int NS = Tx<MY>::NS;
  const int w = threadIdx.x >> 6, lane = threadIdx.x & 63;
  const int n = blockIdx.x * kWavesY + w + 1, r = blockIdx.y;
  if (n > p.nx) return;  // whole wave leaves; no workgroup barrier below
  const int reg = region_elems<T, MY>(p.ny);
  T* buf = smem + w * reg;
  const double ctn = p.ctx[n - 1];
  int mpos[NS];
  double cph[NS], cp[NS], dp[NS];
#pragma unroll
  for (int s = 0; s < NS; ++s) {
    mpos[s] = line_mode<MY>(lane, s, p.ny);
    cph[s] = mpos[s] > 0 ? p.cty[mpos[s] - 1] : 0.0;
    cp[s] = 0.0;
    dp[s] = 0.0;
  }
  double minpiv = 1.0e308;
  unsigned bad = 0;
  T* Gr = reinterpret_cast<T*>(p.G) + r * p.G_stride;
  const bool write_c = (r == 0);
  for (int l = 1; l <= p.nz; ++l) {
    T* line = Gr + ((long long)(l - 1) * p.nx + (n - 1)) * p.ldy;
    for (int e = lane; e < p.ldy && e <= p.ny; e += 64) buf[e] = line[e];
    wave_sync();
    T out[NS];
    line_dst<T, MY>(buf, p.ny, out, lane, p.twy, p.siny);
    // lambda^o = beta^o + s_m alpha^o with beta = Z + s_n B, alpha = C + A s_n
    const double* Ll = p.LC + (l - 1) * 12;
    const double bm = Ll[0] + ctn * Ll[1], am = Ll[2] + Ll[3] * ctn;
    const double b0 = Ll[4] + ctn * Ll[5], a0 = Ll[6] + Ll[7] * ctn;
    const double bp = Ll[8] + ctn * Ll[9], ap = Ll[10] + Ll[11] * ctn;
    double* Cl = p.C + ((long long)(l - 1) * p.nx + (n - 1)) * p.ldy;
#pragma unroll
    for (int s = 0; s < NS; ++s) {
      if (mpos[s] > 0) {
        const double lm = am * cph[s] + bm, l0 = a0 * cph[s] + b0, lp = ap * cph[s] + bp;
        const double piv = l0 - lm * cp[s];
        record_pivot(piv, minpiv, bad);
        const double inv = 1.0 / piv;
        cp[s] = lp * inv;
        dp[s] = ((double)out[s] - lm * dp[s]) * inv;
        line[mpos[s]] = (T)dp[s];
        if (write_c) Cl[mpos[s]] = cp[s];
      }
    }
    wave_sync();
  }
  flush_stats(p, minpiv, bad);
}

// ---------------------------------------------------------------------------
// K3: back substitution + inverse DST along y (one wave per x-mode).
// ---------------------------------------------------------------------------
template <typename T, int MY>
__global__ void __launch_bounds__(64 * kWavesY) k_back_y(ProbDev p) {
  extern __shared__ double smem_raw[];
  T* smem = reinterpret_cast<T*>(smem_raw);
  constexpr int NS = Tx<MY>::NS;
  const int w = threadIdx.x >> 6, lane = threadIdx.x & 63;
  const int n = blockIdx.x * kWavesY + w + 1, r = blockIdx.y;
  if (n > p.nx) return;
  const int reg = region_elems<T, MY>(p.ny);
  T* buf = smem + w * reg;
  int mpos[NS];
  double Wn[NS];
#pragma unroll
  for (int s = 0; s < NS; ++s) {
    mpos[s] = line_mode<MY>(lane, s, p.ny);
    Wn[s] = 0.0;
  }
  T* Gr = reinterpret_cast<T*>(p.G) + r * p.G_stride;
  for (int l = p.nz; l >= 1; --l) {
    T* line = Gr + ((long long)(l - 1) * p.nx + (n - 1)) * p.ldy;
    const double* Cl = p.C + ((long long)(l - 1) * p.nx + (n - 1)) * p.ldy;
#pragma unroll
    for (int s = 0; s < NS; ++s) {
      if (mpos[s] > 0) {
        Wn[s] = (double)line[mpos[s]] - Cl[mpos[s]] * Wn[s];
        buf[mpos[s]] = (T)Wn[s];
      }
    }
    if (lane == 0) buf[0] = (T)0;
    wave_sync();
    T out[NS];
    line_dst<T, MY>(buf, p.ny, out, lane, p.twy, p.siny);
#pragma unroll
    for (int s = 0; s < NS; ++s)
      if (mpos[s] > 0) line[mpos[s]] = out[s];
    wave_sync();
  }
}

// ---------------------------------------------------------------------------
// K4: transposed load of 16 y-lines, inverse DST along x, scale, store u.
// ---------------------------------------------------------------------------
template <typename T, int MX>
__global__ void __launch_bounds__(1024) k_inv_x(ProbDev p) {
  extern __shared__ double smem_raw[];
  T* smem = reinterpret_cast<T*>(smem_raw);
  constexpr int NS = Tx<MX>::NS;
  constexpr int NV = 16;  // ceil(1024/64) column values per lane
  const int jt = blockIdx.x, l = blockIdx.y + 1, r = blockIdx.z;
  const int w = threadIdx.x >> 6, lane = threadIdx.x & 63;
  const T* G = reinterpret_cast<const T*>(p.G) + r * p.G_stride + (long long)(l - 1) * p.nx * p.ldy +
               jt * kTileJ;
  for (int idx = threadIdx.x; idx < p.nx * kTileJ; idx += blockDim.x) {
    const int n0 = idx / kTileJ, jj = idx % kTileJ;
    smem[n0 * kTileJ + (jj ^ (n0 & 15))] = G[(long long)n0 * p.ldy + jj];
  }
  __syncthreads();
  const int j = jt * kTileJ + w;
  const bool active = (j >= 1 && j <= p.ny);
  T col[NV];
#pragma unroll
  for (int k = 0; k < NV; ++k) {
    const int n = 1 + lane + 64 * k;
    col[k] = (active && n <= p.nx) ? smem[(n - 1) * kTileJ + (w ^ ((n - 1) & 15))] : (T)0;
  }
  __syncthreads();
  if (!active) return;
  const int reg = region_elems<T, MX>(p.nx);
  T* buf = smem + w * reg;
#pragma unroll
  for (int k = 0; k < NV; ++k) {
    const int n = 1 + lane + 64 * k;
    if (n <= p.nx) buf[n] = col[k];
  }
  if (lane == 0) buf[0] = (T)0;
  wave_sync();
  T out[NS];
  line_dst<T, MX>(buf, p.nx, out, lane, p.twx, p.sinx);
  double* u = p.u + r * p.u_stride + (long long)p.nx * ((j - 1) + (long long)p.ny * (l - 1));
#pragma unroll
  for (int s = 0; s < NS; ++s) {
    const int i = line_mode<MX>(lane, s, p.nx);
    if (i > 0) u[i - 1] = p.scale * (double)out[s];
  }
}

// ---------------------------------------------------------------------------
// FP64 residual r = F - A U of eq. stencil27 (z-face data as boundary planes).
// ---------------------------------------------------------------------------
__global__ void __launch_bounds__(256) k_residual(ProbDev p, const double* __restrict__ U,
                                                  double* __restrict__ R) {
  const int i = blockIdx.x * 64 + (threadIdx.x & 63) + 1;
  const int j = blockIdx.y * 4 + (threadIdx.x >> 6) + 1;
  const int l = blockIdx.z % p.nz + 1, r = blockIdx.z / p.nz;
  if (i > p.nx || j > p.ny) return;
  const double F = assembled_rhs(p, r, i, j, l);  // lifted for l = 1, nz
  const double* Ur = U + r * p.u_stride;
  double acc = 0.0;
  for (int o = -1; o <= 1; ++o) {
    const int ll = l + o;
    if (ll < 1 || ll > p.nz) continue;  // boundary planes are in the lift
    const double* w = p.W + (l - 1) * 12 + (o + 1) * 4;
    const double* P = Ur + (long long)p.nx * p.ny * (ll - 1);
    double s = 0.0;
    for (int dj = -1; dj <= 1; ++dj) {
      const int jj = j + dj;
      if (jj < 1 || jj > p.ny) continue;
      for (int di = -1; di <= 1; ++di) {
        const int ii = i + di;
        if (ii < 1 || ii > p.nx) continue;
        const double wt = (di && dj) ? w[0] : (di ? w[1] : (dj ? w[2] : w[3]));
        s += wt * P[(ii - 1) + (long long)p.nx * (jj - 1)];
      }
    }
    acc += s;
  }
  R[r * p.u_stride + (i - 1) + (long long)p.nx * ((j - 1) + (long long)p.ny * (l - 1))] = F - acc;
}

__global__ void k_stats_reset(unsigned long long* s) {
  if (threadIdx.x == 0) {
    s[0] = 0x7FEFFFFFFFFFFFFFull;  // bits of DBL_MAX
    s[1] = 0ull;
  }
}

}  // namespace cs3d
