// kernels.hpp - the streaming passes of the direct solve (Section 3.6) on CDNA4.
//
//  K0 rhs     : RHS operator of the scheme (Sections 3.2-3.5) + z-face lift, written as
//               the interior array F (into the caller's output buffer).  Workgroups
//               march along z over a 64 x 64 tile (64 x 16 in the batch), with a ring of
//               four halo planes in LDS and the thread's own column of five planes in
//               registers, so f is read from HBM about once; the corrections on the
//               faces of the box follow in small per-axis passes.
//  K1 fwd_x   : DST-I along x of 8 x-lines of F per workgroup (two such tiles in turn,
//               sharing the 128-byte lines of G, for FP64 lines of 512 and 1024 points);
//               the results are transposed through LDS and stored as y-lines G[l][n][j]
//               (j fastest).
//  K2 fwd_y   : one line group (one or two wavefronts) per x-mode n marches l = 1..N_z:
//               DST-I along y of G[l][n][:], modal eigenvalues lambda^{-,0,+} built on the
//               fly, forward elimination of the N_y tridiagonal systems (one mode m per
//               lane slot).  d'_l is stored in place, c'_l once per plan column in C.
//  K3 back_y  : the same line groups march l = N_z..1: back substitution
//               W_l = d'_l - c'_l W_{l+1}, inverse DST-I along y, stored in place.
//  K4 inv_x   : 8 y-lines per workgroup are transposed back through LDS, inverse
//               DST-I along x, scaled by 4/((N_x+1)(N_y+1)) and stored as u (x fastest).
//
// The DST-I is its own inverse up to the factor (N+1)/2, so all line transforms are
// the same routine and the orthonormal V of Section 3.6 is recovered by the single
// final scale.
#pragma once
#include <type_traits>

#include "wave_dst.hpp"

namespace cs3d {

enum SchemeId : int { kHelm2 = 2, kHelm4 = 4, kHelm6 = 6, kCd4 = 14, kWeights = 99 };

#ifndef CS3D_TILEJ
#define CS3D_TILEJ 8
#endif
constexpr int kTileJ = CS3D_TILEJ;  // y-lines per K1/K4 workgroup (one wavefront each)
constexpr int kBlockY = 256;  // threads per K2/K3 workgroup

struct ProbDev {
  int nx, ny, nz;
  int Mx, My;          // N+1 per axis
  int fx, fy;          // FFT length per axis (N+1 when a power of two in 64..1024), 0 = dense sine sums
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
  const double2* twx;  // exp(-i pi k/Mx), k < Mx  (FFT path)
  const double2* twy;
  const double* sinx;  // sin(pi r/Mx), r < 2 Mx      (dense path)
  const double* siny;
  // data (per right-hand side strides in elements)
  const double* f;     // closed grid f (K0 input)
  long long f_stride;
  const double* glo;   // closed planes or null
  const double* ghi;
  long long g_stride;
  const double* F;     // interior right-hand side (K1 input)
  double* u;           // interior solution (K4 output; K0 writes F here)
  long long u_stride;
  void* G;             // [nrhs][nz][nx][ldy] of the transform type
  long long G_stride;
  double* C;           // [nz][nx][ldy]   c' of the tridiagonal LU
  unsigned long long* stats;  // [0] = bits of min |pivot|, [1] = count of bad pivots
  int accumulate;      // K4: u += result (refinement corrections) instead of u = result
  int f32_input;       // K1: F holds FP32 values (the residuals of the mixed path)
  int zchunk;          // planes per workgroup of the z-marching passes (K0, residual)
  // complex k (absorbing media): imaginary parts; a complex right-hand side q occupies the
  // real slots 2q (real part) and 2q+1 (imaginary part) of f, F, u, G and the z-face data
  const double* Wi;    // [nz][3][4] imaginary parts of the row weights
  const double* LCi;   // [nz][3][4] imaginary parts of (Z, B, C, A)
  const double* k2i;   // [nz+2] Im k^2
  const double* k2zi;  // [nz+2] Im (k^2)_z
  double* Ci;          // [nz][nx][ldy] Im c'
  // Robin z faces: nz counts the system's planes z_0..z_{nz-1} (the face nodes are
  // unknowns); the first and last modal rows take the ghost-plane elimination
  //   row 0:    lambda^0 += (rb[0] + rb[1] mu) lambda^-,  lambda^+ += lambda^-
  //   row nz-1: lambda^0 += (rb[2] + rb[3] mu) lambda^+,  lambda^- += lambda^+
  // with mu = -2 s_n/hx^2 - 2 s_m/hy^2 the eigenvalue of the in-plane 5-point Laplacian;
  // ralpha, rbeta: the conditions alpha u_z + beta u = g of the two faces
  int robin;
  double rb[4];
  double ralpha[2], rbeta[2];
};

// ---------------------------------------------------------------------------
// Line transform selection: the FFT length M (N+1 for the sine transform, N-1 for the
// cosine transform of Neumann sides), 0 for dense sums; KIND kDst or kDct.
// ---------------------------------------------------------------------------
template <int M, int WPL, int KIND = kDst>
struct Tx {
  static constexpr int NS = fft_out_slots<M, WPL, KIND>();
};
template <int WPL, int KIND>
struct Tx<0, WPL, KIND> {
  static constexpr int NS = kDenseSlots;
};

template <typename T, int M, int WPL, int KIND = kDst>
using TxOut = T[Tx<M, WPL, KIND>::NS];

template <typename T, int M, int WPL, bool BLOCK_SYNC = false, int KIND = kDst, bool PAIR = false>
__device__ __forceinline__ void line_dst(T* buf, int N, TxOut<T, M, WPL, KIND>& out, int tl, const cx<T>* tab,
                                         const double* trig, const T* src = nullptr) {
  if constexpr (M == 0) {
    dst_dense<T, KIND>(buf, N, out, tl, trig, src);
    if constexpr (BLOCK_SYNC) __syncthreads();
  } else {
    dst_fft<T, M, WPL, KIND, BLOCK_SYNC, PAIR>(buf, out, tl, tab, src);
  }
}

template <int M, int WPL, int KIND = kDst>
__device__ __forceinline__ int line_mode(int tl, int s, int N) {
  if constexpr (M == 0) {
    return dense_mode(tl, s, N);
  } else {
    return fft_mode<M, WPL, KIND>(tl, s);
  }
}

// elements of T in one line buffer (it also holds the line at positions 0..N)
template <typename T, int M, int WPL, bool PAIR = false>
__host__ __device__ constexpr int line_buf_elems(int N) {
  const int line = ((N + 1 + 63) / 64) * 64;
  return M ? (fft_buf_elems<T, M, WPL, PAIR>() > line ? fft_buf_elems<T, M, WPL, PAIR>() : line) : line;
}

// twiddle table bytes (FFT path only)
template <typename T, int M>
__host__ __device__ constexpr int tw_bytes() {
  return M ? tw_entries<M>() * (int)sizeof(cx<T>) : 0;
}

// row stride (>= nx + 1, = 32 / tj mod 32) of the K1/K4 transpose tile of tj (8, 16 or 32)
// rows: the transposed accesses (tj rows x 32 / tj columns per half-wave) then hit 32
// distinct bank pairs
__host__ __device__ constexpr int tile_stride(int nx, int tj = kTileJ) {
  return ((nx + 1 - 32 / tj + 31) / 32) * 32 + 32 / tj;
}

// ---------------------------------------------------------------------------
// Hide a value from loop-invariant code motion (an empty asm statement that claims to
// change it): per-thread offsets derived from it are then recomputed where used instead
// of being hoisted out of a persistent loop as one live register pair per access.
template <typename V>
__device__ __forceinline__ V opaque(V v) {
  asm volatile("" : "+v"(v));
  return v;
}

// Settle prefetched registers: the wait for their loads happens here instead of where they
// are first used.  Placed after a transform and before a phase of stores, it keeps the
// wait (which also waits for every older memory operation) from covering those stores,
// so they stay in flight while the next line or tile is filled.
template <typename V, int N>
__device__ __forceinline__ void settle(V (&a)[N]) {
#pragma unroll
  for (int k = 0; k < N; ++k) a[k] = opaque(a[k]);
}


// ---------------------------------------------------------------------------
// XCD-aware work order.  The 8 XCDs of the chip each have their own L2, and
// workgroups are handed to them round-robin by linear index.  xcd_order maps the
// linear index L of a grid of n workgroups to a work index so that every XCD receives
// one contiguous range of work indices: neighbouring tiles, which share cache lines
// (x passes) or stencil halos (z-marching passes), then meet in the same L2.
// ---------------------------------------------------------------------------
constexpr int kXcds = 8;

__device__ __forceinline__ int xcd_order(int L, int n) {
  const int q = n / kXcds;
  return L < q * kXcds ? (L % kXcds) * q + L / kXcds : L;
}

__device__ __forceinline__ int linear_block() {
  return blockIdx.x + gridDim.x * (blockIdx.y + gridDim.y * blockIdx.z);
}

// ---------------------------------------------------------------------------
// K0: RHS operator + lift.  Tile 64 (x) x RY (y) interior points, 16 RY threads; thread
// (lane, wave) owns column x0 + lane, rows y0 + 4 wave .. + 3.  The workgroup marches
// over a z-chunk with a four-plane ring of halo tiles in LDS (the planes l-1, l, l+1
// and the next one) and two further planes in flight in registers; every thread keeps
// its own column of the five planes l-2 .. l+2 in registers, so the z-differences and
// the y-differences inside its rows cost no LDS reads.
// ---------------------------------------------------------------------------
constexpr int kRX = 64, kRH = 2, kZChunk = 32;  // kZChunk: default planes per workgroup
constexpr int kSX = kRX + 2 * kRH;
constexpr int kRSlots = 4;  // LDS planes

__device__ __forceinline__ double d4_onesided(const double* c, long long s, bool low) {
  // fourth difference at the first (low) or last interior layer: one-sided 6-point
  // formula from the boundary point and the next five points
  return low ? 2.0 * c[-s] - 9.0 * c[0] + 16.0 * c[s] - 14.0 * c[2 * s] + 6.0 * c[3 * s] - c[4 * s]
             : 2.0 * c[s] - 9.0 * c[0] + 16.0 * c[-s] - 14.0 * c[-2 * s] + 6.0 * c[-3 * s] - c[-4 * s];
}

// in-plane 9-point stencil of weights w = (a, b, c, d) on a closed plane at (i, j)
__device__ __forceinline__ double plane9(const double* __restrict__ w, const double* __restrict__ P,
                                         int nx, int i, int j) {
  const long long sy = nx + 2;
  const double* c = P + i + sy * j;
  return w[0] * (c[-sy - 1] + c[-sy + 1] + c[sy - 1] + c[sy + 1]) + w[1] * (c[-1] + c[1]) +
         w[2] * (c[-sy] + c[sy]) + w[3] * c[0];
}

// Correction of F at a point (i, j, l) on the faces of the interior box normal to `axis`
// (0: x, 1: y, 2: z): for the 6th-order operator the one-sided fourth difference along the
// axis in place of the zero-padded central one the RHS pass formed; on the z faces also
// minus the lift of the z-face data (both faces when nz = 1).  No contraction here: the
// per-axis face passes and the batch's inline loop then add the same value bit for bit,
// whatever the caller's context lets the compiler fuse.
__device__ __forceinline__ double face_corr(const ProbDev& p, int r, int i, int j, int l, int axis) {
#pragma clang fp contract(off)
  const long long sy = p.nx + 2, sz = (long long)(p.nx + 2) * (p.ny + 2);
  const double hz2 = p.hz * p.hz;
  double F = 0.0;
  if (p.scheme == kHelm6) {
    const double* c = p.f + r * p.f_stride + i + sy * j + sz * l;
    const long long st = axis == 0 ? 1 : (axis == 1 ? sy : sz);
    const int n = axis == 0 ? p.nx : (axis == 1 ? p.ny : p.nz);
    const int at = axis == 0 ? i : (axis == 1 ? j : l);
    const bool low = at == 1, hi = at == n;
    // the central difference as the RHS pass formed it (values beyond the grid are zero)
    const double pad = (low ? 0.0 : c[-2 * st]) + (hi ? 0.0 : c[2 * st]) - 4.0 * (c[-st] + c[st]) + 6.0 * c[0];
    F = -hz2 * (d4_onesided(c, st, low) - pad) * (1.0 / 240.0);
  }
  if (axis == 2) {
    // the weights through vector loads (an opaque offset): a uniform read here would
    // otherwise become a scalar load, the kind of read under which plans created after
    // others had been destroyed once gave wrong results (cause not isolated)
    const int o = opaque(0);
    if (l == 1 && p.glo) F -= plane9(p.W + o, p.glo + r * p.g_stride, p.nx, i, j);
    if (l == p.nz && p.ghi) F -= plane9(p.W + (p.nz - 1) * 12 + 8 + o, p.ghi + r * p.g_stride, p.nx, i, j);
  }
  return F;
}

// RHS tiles of 64 x RY points, four rows per thread: 16 RY threads.  The plan's pass takes
// 64 x 64 tiles (one workgroup of 16 waves per CU, 156 KB of LDS): their halo re-reads
// 1.09x the closed grid where 64 x 16 tiles re-read 1.30x (measured at 1023^3 x 4, FETCH_SIZE;
// 17.0 against 17.3 ms).  The batch keeps 64 x 16 tiles (its members are small, and the
// larger tile spills in the batch kernel).
template <int RY>
struct RTile {
  static constexpr int Y = RY, ROWS = 4, THREADS = 64 * RY / ROWS, SY = RY + 2 * kRH;
  static constexpr int LOADS = (SY * kSX + THREADS - 1) / THREADS;  // plane-tile elements per thread
};
constexpr int kRYPlan = 64, kRYBatch = 16;
constexpr int kRThreadsPlan = RTile<kRYPlan>::THREADS, kRThreadsBatch = RTile<kRYBatch>::THREADS;
constexpr int kZMax = 512;  // largest z-chunk of the z-marching passes (the tuning range)

// one 64 x 16 tile (bx, by) over the z-chunk zc of right-hand side r.  FACES: add the
// corrections of the points on the faces of the box here (else k_rhs_faces does it)
template <int RY, bool FACES>
__device__ __forceinline__ void rhs_block(const ProbDev& p, int bx, int by, int zc, int r,
                                          double (*win)[RTile<RY>::SY * kSX], double* kt) {
  constexpr int kRY = RY, kSY = RTile<RY>::SY, kRThreads = RTile<RY>::THREADS;
  constexpr int kRRows = RTile<RY>::ROWS, kRLoads = RTile<RY>::LOADS;
  const int tx = threadIdx.x & 63, ty = threadIdx.x >> 6;
  const int x0 = 1 + bx * kRX, y0 = 1 + by * kRY;
  const int lb = 1 + zc * p.zchunk;
  const int le = min(p.nz, lb + p.zchunk - 1);
  // k^2 and (k^2)_z of the chunk's planes in LDS (kt[0..), kt[kZMax..)): read there, the
  // per-plane samples cost no vector load, whose wait would also wait for the prefetched
  // planes.  The barrier keeps a previous call's readers off the table.
  __syncthreads();
  for (int q = threadIdx.x; q <= le - lb; q += kRThreads) {
    kt[q] = p.k2[lb + q];
    kt[kZMax + q] = p.k2z[lb + q];
  }
  const long long sy = p.nx + 2, sz = (long long)(p.nx + 2) * (p.ny + 2);
  const double* __restrict__ f = p.f + r * p.f_stride;

  // this thread's share of a plane tile: in-plane offsets, fixed for every plane
  int off[kRLoads];
  bool ok[kRLoads];
#pragma unroll
  for (int k = 0; k < kRLoads; ++k) {
    const int e = threadIdx.x + kRThreads * k;
    const int yy = e / kSX, xx = e - yy * kSX;
    const int gx = x0 - kRH + xx, gy = y0 - kRH + yy;
    ok[k] = e < kSY * kSX && gx >= 0 && gx <= p.nx + 1 && gy >= 0 && gy <= p.ny + 1;
    off[k] = ok[k] ? gx + (int)sy * gy : 0;
  }
  auto fetch = [&](double(&pre)[kRLoads], int q) {
    const bool qok = q >= 0 && q <= p.nz + 1;
    const double* fq = f + sz * (qok ? q : 0);
#pragma unroll
    for (int k = 0; k < kRLoads; ++k) pre[k] = (qok && ok[k]) ? fq[off[k]] : 0.0;
  };
  auto slot = [](int q) { return (q + 2 * kRSlots) % kRSlots; };
  auto stash = [&](const double(&pre)[kRLoads], int q) {
    double* w = win[slot(q)];
#pragma unroll
    for (int k = 0; k < kRLoads; ++k) {
      const int e = threadIdx.x + kRThreads * k;
      if (e < kSY * kSX) w[e] = pre[k];
    }
  };
  // tile index of this thread's row k
  const int cbase = (ty * kRRows + kRH) * kSX + tx + kRH;
  // own column of planes l-2 .. l+2
  double cz[5][kRRows];
  auto own = [&](double(&dst)[kRRows], int q) {
    const double* w = win[slot(q)];
#pragma unroll
    for (int k = 0; k < kRRows; ++k) dst[k] = w[cbase + k * kSX];
  };

  // prologue: planes lb-2 .. lb+1 into the ring and their own columns into registers,
  // then plane lb+2 over lb-2's slot; two further planes in flight in pa, pb (the step
  // of plane l stashes plane l+3 from the buffer (l - lb) mod 2 and refills that buffer
  // with plane l+5)
  double pa[kRLoads], pb[kRLoads];
  for (int q = lb - 2; q <= lb + 1; ++q) {
    fetch(pa, q);
    stash(pa, q);
  }
  fetch(pa, lb + 2);
  if (lb < le) fetch(pb, lb + 3);
  __syncthreads();
  own(cz[0], lb - 2);
  own(cz[1], lb - 1);
  own(cz[2], lb);
  own(cz[3], lb + 1);
  __syncthreads();
  stash(pa, lb + 2);
  if (lb + 1 < le) fetch(pa, lb + 4);
  __syncthreads();
  own(cz[4], lb + 2);

  const int i = x0 + tx;
  const double hz2 = p.hz * p.hz, h = p.hz;
  auto compute = [&](int l) {
    const double* P0 = win[slot(l)];
    const double* Pm = win[slot(l - 1)];
    const double* Pp = win[slot(l + 1)];
    const double kl = kt[l - lb], kzl = kt[kZMax + l - lb];
    // y-neighbours: own registers inside the thread's rows, LDS outside
    auto y0v = [&](int k, int d) -> double {
      const int kk = k + d;
      return (kk >= 0 && kk < kRRows) ? cz[2][kk] : P0[cbase + kk * kSX];
    };
    auto ymv = [&](int k, int d) -> double {
      const int kk = k + d;
      return (kk >= 0 && kk < kRRows) ? cz[1][kk] : Pm[cbase + kk * kSX];
    };
    auto ypv = [&](int k, int d) -> double {
      const int kk = k + d;
      return (kk >= 0 && kk < kRRows) ? cz[3][kk] : Pp[cbase + kk * kSX];
    };
#pragma unroll
    for (int k = 0; k < kRRows; ++k) {
      const int j = y0 + ty * kRRows + k;
      if (i > p.nx || j > p.ny) continue;
      const int c0 = cbase + k * kSX;
      const double f0 = cz[2][k];
      double F;
      if (p.scheme == kHelm2) {
        F = hz2 * f0;
      } else {
        // A: the 6 face neighbours
        const double ax = P0[c0 - 1] + P0[c0 + 1];
        const double ay = y0v(k, -1) + y0v(k, 1);
        const double az = cz[1][k] + cz[3][k];
        const double A = ax + ay + az;
        if (p.scheme == kHelm4) {
          // f + h^2/12 sum d2  =  f/2 + A/12
          F = hz2 * (0.5 * f0 + A * (1.0 / 12.0));
        } else if (p.scheme == kCd4) {
          // f + (d2x + d2y)/12 + (h gamma f_z + d2z)/12 with central f_z
          F = hz2 * (0.5 * f0 + A * (1.0 / 12.0) + p.hz * p.gamma * (cz[3][k] - cz[1][k]) * (1.0 / 24.0));
        } else {
          // 6th order: f + h^2/12 sum d2 - h^4/240 sum d4 + h^4/90 sum d2d2 - h^2 k^2 f/20
          // + h^4 (k^2)_z f_z/60, differences undivided, collected by stencil point:
          //   (67/120 - h^2 k^2/20) f + A/18 + E/90 - E2/240 + h^3 (k^2)_z (f_{l+1} - f_{l-1})/120
          // with E the 12 edge and E2 the 6 axis-distance-2 neighbours.  On the faces of
          // the interior box the axis-distance-2 values outside the grid are zeros here;
          // the one-sided fourth differences replace them below.
          const double e2 = P0[c0 - 2] + P0[c0 + 2] + y0v(k, -2) + y0v(k, 2) + cz[0][k] + cz[4][k];
          const double exy = P0[c0 - kSX - 1] + P0[c0 - kSX + 1] + P0[c0 + kSX - 1] + P0[c0 + kSX + 1];
          const double exz = Pm[c0 - 1] + Pm[c0 + 1] + Pp[c0 - 1] + Pp[c0 + 1];
          const double eyz = ymv(k, -1) + ymv(k, 1) + ypv(k, -1) + ypv(k, 1);
          const double E = exy + exz + eyz;
          F = hz2 * ((67.0 / 120.0 - h * h * kl * (1.0 / 20.0)) * f0 + A * (1.0 / 18.0) + E * (1.0 / 90.0) -
                     e2 * (1.0 / 240.0) + h * h * h * kzl * (cz[3][k] - cz[1][k]) * (1.0 / 120.0));
        }
      }
      p.u[r * p.u_stride + (i - 1) + (long long)p.nx * ((j - 1) + (long long)p.ny * (l - 1))] = F;
    }
    // FACES: the face corrections (face_corr), added axis by axis in the order of the
    // per-axis face passes, so both ways give the same result bit for bit (a rolled loop:
    // the rarely taken global reads cost no registers in the code above)
    if constexpr (FACES) {
      const bool h6 = p.scheme == kHelm6;
      const bool zface = l == 1 || l == p.nz;
      const bool lift = (l == 1 && p.glo) || (l == p.nz && p.ghi);
      const int jb = y0 + ty * kRRows;
      const bool yface = jb == 1 || (jb <= p.ny && p.ny <= jb + kRRows - 1);
      if (i <= p.nx && ((h6 && (zface || yface || i == 1 || i == p.nx)) || lift)) {
#pragma unroll 1
        for (int k = 0; k < kRRows; ++k) {
          const int j = jb + k;
          if (j > p.ny) break;
          double* u = p.u + r * p.u_stride + (i - 1) + (long long)p.nx * ((j - 1) + (long long)p.ny * (l - 1));
          if (h6 && (i == 1 || i == p.nx)) *u += face_corr(p, r, i, j, l, 0);
          if (h6 && (j == 1 || j == p.ny)) *u += face_corr(p, r, i, j, l, 1);
          if ((h6 && zface) || lift) *u += face_corr(p, r, i, j, l, 2);
        }
      }
    }
  };
  // step l: compute plane l; then plane l+3 replaces l-1 in the ring, its buffer is
  // refilled with plane l+5, and the own columns move up by one plane
  for (int l = lb; l <= le; l += 2) {
    compute(l);
    if (l == le) break;
    __syncthreads();
    stash(pb, l + 3);
    if (l + 2 < le) fetch(pb, l + 5);
    __syncthreads();
#pragma unroll
    for (int k = 0; k < kRRows; ++k) {
      cz[0][k] = cz[1][k];
      cz[1][k] = cz[2][k];
      cz[2][k] = cz[3][k];
      cz[3][k] = cz[4][k];
    }
    own(cz[4], l + 3);
    compute(l + 1);
    if (l + 1 == le) break;
    __syncthreads();
    stash(pa, l + 4);
    if (l + 3 < le) fetch(pa, l + 6);
    __syncthreads();
#pragma unroll
    for (int k = 0; k < kRRows; ++k) {
      cz[0][k] = cz[1][k];
      cz[1][k] = cz[2][k];
      cz[2][k] = cz[3][k];
      cz[3][k] = cz[4][k];
    }
    own(cz[4], l + 4);
  }
}

// grid: (x tiles) x (y tiles) x (z chunks x right-hand sides), taken in XCD order; the
// face corrections follow in k_rhs_faces
__global__ void __launch_bounds__(kRThreadsPlan) k_rhs(ProbDev p) {
  __shared__ double win[kRSlots][RTile<kRYPlan>::SY * kSX];
  __shared__ double kt[2 * kZMax];
  const int nzc = (p.nz + p.zchunk - 1) / p.zchunk;
  const int T = xcd_order(linear_block(), gridDim.x * gridDim.y * gridDim.z);
  const int bx = T % gridDim.x, by = (T / gridDim.x) % gridDim.y, bz = T / (gridDim.x * gridDim.y);
  rhs_block<kRYPlan, false>(p, bx, by, bz % nzc, bz / nzc, win, kt);
}

// Corrections of F on one pair of faces of the interior box (axis 0: x, 1: y, 2: z), one
// point per thread: for the 6th-order operator the one-sided fourth difference along the
// axis in place of the zero-padded central one k_rhs formed; on the z faces also minus the
// lift of the z-face data.  One launch per axis, so no point is updated twice at once.
// grid: (ceil(face points / 256), 2 faces, right-hand sides)
__global__ void __launch_bounds__(256) k_rhs_faces(ProbDev p, int axis) {
  const int e = blockIdx.x * 256 + threadIdx.x;
  const int high = blockIdx.y, r = blockIdx.z;
  int i, j, l;
  if (axis == 0) {
    if (e >= p.ny * p.nz) return;
    j = 1 + e % p.ny;
    l = 1 + e / p.ny;
    i = high ? p.nx : 1;
  } else if (axis == 1) {
    if (e >= p.nx * p.nz) return;
    i = 1 + e % p.nx;
    l = 1 + e / p.nx;
    j = high ? p.ny : 1;
  } else {
    if (e >= p.nx * p.ny) return;
    i = 1 + e % p.nx;
    j = 1 + e / p.nx;
    l = high ? p.nz : 1;
    if (high && p.nz == 1) return;  // a single plane: the low-face thread lifts both
  }
  const double F = face_corr(p, r, i, j, l, axis);
  p.u[r * p.u_stride + (i - 1) + (long long)p.nx * ((j - 1) + (long long)p.ny * (l - 1))] += F;
}

// ---------------------------------------------------------------------------
// Robin z faces: F on the face planes of the system (plane 0 at z_0, plane nz-1 at
// z_{N+1}; p.nz counts the system's planes, f has p.nz closed-grid planes), one node per
// thread:
//  - the scheme's RHS operator at the face node (Sections 3.2-3.4) with the z differences
//    one-sided into the box: delta_z^2 from (2, -5, 4, -1), delta_z^4 from
//    (3, -14, 26, -24, 11, -2), delta_z from (-3, 4, -1)/2 (raw differences);
//  - minus the face row's plane-offset weights applied to the data of the eliminated ghost
//    plane, R = (s/alpha)((-2h + (h^3/3) k^2) g + (h^3/3) D g) - (h^3/3) f_z with s = +1 on
//    the low face and -1 on the high face, D the in-plane 5-point Laplacian, f_z one-sided
//    of second order (zero beyond the x/y sides, where g and u vanish).
// grid: (ceil(nx ny / 256), 2 faces, right-hand sides)
// ---------------------------------------------------------------------------
__global__ void __launch_bounds__(256) k_robin_faces(ProbDev p) {
  const int e = blockIdx.x * 256 + threadIdx.x;
  if (e >= p.nx * p.ny) return;
  const int i = 1 + e % p.nx, j = 1 + e / p.nx;
  const int face = blockIdx.y, r = blockIdx.z;
  const long long sy = p.nx + 2, sz = sy * (p.ny + 2);
  const double* f = p.f + r * p.f_stride;
  const double sg = face ? -1.0 : 1.0;
  // plane q of f counted from the face into the box (q = 0: the face plane)
  auto fp = [&](int q) -> const double* { return f + sz * (face ? p.nz - 1 - q : q); };
  auto at = [&](const double* P, int ii, int jj) -> double { return P[ii + sy * jj]; };
  const double* f0 = fp(0);
  const double* f1 = fp(1);
  const double* f2 = fp(2);
  const double* f3 = fp(3);
  // one-sided second z difference (raw) at an in-plane node
  auto d2z = [&](int ii, int jj) -> double {
    return 2.0 * at(f0, ii, jj) - 5.0 * at(f1, ii, jj) + 4.0 * at(f2, ii, jj) - at(f3, ii, jj);
  };
  const double h = p.hz, h2 = h * h, h3 = h2 * h;
  const double c0 = at(f0, i, j);
  const double d2x = at(f0, i - 1, j) - 2.0 * c0 + at(f0, i + 1, j);
  const double d2y = at(f0, i, j - 1) - 2.0 * c0 + at(f0, i, j + 1);
  const double dzz = d2z(i, j);
  // sample index of the face plane: z_0 at 1, z_{N+1} at p.nz (samples from z_{-1})
  const int ks = face ? p.nz : 1;
  const double k2f = p.k2[ks], k2zf = p.k2z[ks];
  double F;
  if (p.scheme == kHelm2) {
    F = h2 * c0;
  } else if (p.scheme == kHelm4) {
    F = h2 * (c0 + (d2x + d2y + dzz) / 12.0);
  } else {
    // 6th order (uniform h): fourth differences in x and y with the one-sided formula on
    // the first and last interior lines, as in the interior planes
    const double* cc = f0 + i + sy * j;
    const double d4x = (i == 1 || i == p.nx) ? d4_onesided(cc, 1, i == 1)
                                             : cc[-2] - 4.0 * (cc[-1] + cc[1]) + 6.0 * cc[0] + cc[2];
    const double d4y = (j == 1 || j == p.ny) ? d4_onesided(cc, sy, j == 1)
                                             : cc[-2 * sy] - 4.0 * (cc[-sy] + cc[sy]) + 6.0 * cc[0] + cc[2 * sy];
    const double d4z = 3.0 * c0 - 14.0 * at(f1, i, j) + 26.0 * at(f2, i, j) - 24.0 * at(f3, i, j) +
                       11.0 * at(fp(4), i, j) - 2.0 * at(fp(5), i, j);
    const double d2xy = (at(f0, i - 1, j - 1) - 2.0 * at(f0, i, j - 1) + at(f0, i + 1, j - 1)) -
                        2.0 * d2x + (at(f0, i - 1, j + 1) - 2.0 * at(f0, i, j + 1) + at(f0, i + 1, j + 1));
    const double d2xz = d2z(i - 1, j) - 2.0 * dzz + d2z(i + 1, j);
    const double d2yz = d2z(i, j - 1) - 2.0 * dzz + d2z(i, j + 1);
    const double d1z = sg * (-3.0 * c0 + 4.0 * at(f1, i, j) - at(f2, i, j)) * 0.5;
    F = h2 * (c0 + (d2x + d2y + dzz) / 12.0 - (d4x + d4y + d4z) / 240.0 + (d2xy + d2xz + d2yz) / 90.0 -
              h2 * k2f * c0 / 20.0 + h3 * k2zf * d1z / 60.0);
  }
  // the ghost-plane data R at an interior in-plane node (zero beyond the sides)
  const double* g = face ? p.ghi : p.glo;
  const double* gr = g ? g + r * p.g_stride : nullptr;
  const double ia = 1.0 / p.ralpha[face];
  const double cg = -2.0 * h + (h3 / 3.0) * k2f;
  auto R = [&](int ii, int jj) -> double {
    if (ii < 1 || ii > p.nx || jj < 1 || jj > p.ny) return 0.0;
    double v = 0.0;
    if (gr) {
      const double gc = at(gr, ii, jj);
      const double lap = (at(gr, ii - 1, jj) - 2.0 * gc + at(gr, ii + 1, jj)) / (p.hx * p.hx) +
                         (at(gr, ii, jj - 1) - 2.0 * gc + at(gr, ii, jj + 1)) / (p.hy * p.hy);
      v = sg * ia * (cg * gc + (h3 / 3.0) * lap);
    }
    const double fz = (-3.0 * at(f0, ii, jj) + 4.0 * at(f1, ii, jj) - at(f2, ii, jj)) / (2.0 * h);
    return v - (h3 / 3.0) * fz;
  };
  // the face row's weights of the ghost side: row 0 offset -1, row nz-1 offset +1
  const int o = opaque(0);
  const double* w = p.W + (face ? (long long)(p.nz - 1) * 12 + 8 : 0) + o;
  const double lift = w[0] * (R(i - 1, j - 1) + R(i + 1, j - 1) + R(i - 1, j + 1) + R(i + 1, j + 1)) +
                      w[1] * (R(i - 1, j) + R(i + 1, j)) + w[2] * (R(i, j - 1) + R(i, j + 1)) + w[3] * R(i, j);
  p.u[r * p.u_stride + (long long)(face ? p.nz - 1 : 0) * p.nx * p.ny + (i - 1) + (long long)p.nx * (j - 1)] =
      F - lift;
}

// ---------------------------------------------------------------------------
// RHS operator for Neumann sides: p.nx, p.ny count the nodes of an x/y plane (the
// side nodes are unknowns), f is the closed grid with rows of p.nx values, and a
// value beyond a side is the mirror image about it (f_{-1} = f_1, f_{-2} = f_2).
// The x and y differences are therefore all central; the z ones as in k_rhs (the
// one-sided fourth difference on the first and last plane), then the lift of the
// z-face data through the in-plane 9-point weights, mirrored alike.
// One point per thread; grid: (ceil(nx ny / 256), nz, right-hand sides).
// ---------------------------------------------------------------------------
__device__ __forceinline__ int mirror(int i, int n) { return i < 0 ? -i : (i >= n ? 2 * (n - 1) - i : i); }

// Each thread owns a node (i, j) and marches over a chunk of kSidesChunk planes, keeping the
// 13-point neighbourhoods (centre, the 4 face and 4 edge neighbours, the 4 at distance 2) of
// the planes l-2..l+2 in a ring of registers: one new neighbourhood is loaded per plane.
// grid: (ceil(nx ny / 256), ceil(nz / kSidesChunk), right-hand sides)
constexpr int kSidesChunk = 60;  // a multiple of the ring's 5, so ring slots are compile-time

__global__ void __launch_bounds__(256) k_rhs_sides(ProbDev p) {
  const int e = blockIdx.x * 256 + threadIdx.x;
  if (e >= p.nx * p.ny) return;
  const int i = e % p.nx, j = e / p.nx, r = blockIdx.z;
  const int nx = p.nx, ny = p.ny, nz = p.nz;
  const int lb = 1 + blockIdx.y * kSidesChunk, le = min(nz, lb + kSidesChunk - 1);
  const double* f = p.f + r * p.f_stride;
  const long long P = (long long)nx * ny;
  // mirrored in-plane offsets, slot order: c, x-1, x+1, y-1, y+1, (x-1,y-1), (x+1,y-1),
  // (x-1,y+1), (x+1,y+1), x-2, x+2, y-2, y+2
  constexpr int DX[13] = {0, -1, 1, 0, 0, -1, 1, -1, 1, -2, 2, 0, 0};
  constexpr int DY[13] = {0, 0, 0, -1, 1, -1, -1, 1, 1, 0, 0, -2, 2};
  int off[13];
#pragma unroll
  for (int k = 0; k < 13; ++k) off[k] = mirror(i + DX[k], nx) + nx * mirror(j + DY[k], ny);
  double ring[5][13];
  auto load = [&](double(&v)[13], int q) {  // planes outside 0..nz+1 are never used
    const double* fq = f + P * (q < 0 ? 0 : (q > nz + 1 ? nz + 1 : q));
#pragma unroll
    for (int k = 0; k < 13; ++k) v[k] = fq[off[k]];
  };
  auto centre = [&](int q) { return f[P * q + off[0]]; };
  const double hz2 = p.hz * p.hz;
  // plane l sits in ring slot S = l mod 5 (lb = 1 mod 5)
  auto plane = [&](int l, auto slot) {
    constexpr int S = decltype(slot)::value;
    const double(&c)[13] = ring[S];
    const double(&m1)[13] = ring[(S + 4) % 5];
    const double(&p1)[13] = ring[(S + 1) % 5];
    const double f0 = c[0];
    double F;
    if (p.scheme == kHelm2) {
      F = hz2 * f0;
    } else {
      const double d2x = c[1] - 2.0 * f0 + c[2];
      const double d2y = c[3] - 2.0 * f0 + c[4];
      const double d2z = m1[0] - 2.0 * f0 + p1[0];
      if (p.scheme == kHelm4) {
        F = hz2 * (f0 + (d2x + d2y + d2z) * (1.0 / 12.0));
      } else if (p.scheme == kCd4) {
        const double d1z = 0.5 * (p1[0] - m1[0]);
        F = hz2 * (f0 + d2x * (1.0 / 12.0) + d2y * (1.0 / 12.0) + (p.hz * p.gamma * d1z + d2z) * (1.0 / 12.0));
      } else {
        // 6th order: f + sum d2/12 - sum d4/240 + sum d2d2/90 - h^2 k^2 f/20 + h^3 (k^2)_z d1z/60
        const double h = p.hz, kl = p.k2[l], kzl = p.k2z[l];
        const double d4x = c[9] - 4.0 * (c[1] + c[2]) + 6.0 * f0 + c[10];
        const double d4y = c[11] - 4.0 * (c[3] + c[4]) + 6.0 * f0 + c[12];
        double d4z;
        if (l == 1) {
          d4z = 2.0 * m1[0] - 9.0 * f0 + 16.0 * p1[0] - 14.0 * ring[(S + 2) % 5][0] + 6.0 * centre(l + 3) -
                centre(l + 4);
        } else if (l == nz) {
          d4z = 2.0 * p1[0] - 9.0 * f0 + 16.0 * m1[0] - 14.0 * ring[(S + 3) % 5][0] + 6.0 * centre(l - 3) -
                centre(l - 4);
        } else {
          d4z = ring[(S + 3) % 5][0] - 4.0 * (m1[0] + p1[0]) + 6.0 * f0 + ring[(S + 2) % 5][0];
        }
        // products of second differences over the three coordinate planes (the sums of the
        // 3 x 3 weights (1, -2, 1) x (1, -2, 1), taken row by row)
        const double sxy = (c[5] - 2.0 * c[3] + c[6]) - 2.0 * (c[1] - 2.0 * f0 + c[2]) + (c[7] - 2.0 * c[4] + c[8]);
        const double sxz = (m1[1] - 2.0 * m1[0] + m1[2]) - 2.0 * (c[1] - 2.0 * f0 + c[2]) + (p1[1] - 2.0 * p1[0] + p1[2]);
        const double syz = (m1[3] - 2.0 * m1[0] + m1[4]) - 2.0 * (c[3] - 2.0 * f0 + c[4]) + (p1[3] - 2.0 * p1[0] + p1[4]);
        const double sx = sxy + sxz + syz;
        const double d1z = 0.5 * (p1[0] - m1[0]);
        F = h * h * (f0 + (d2x + d2y + d2z) * (1.0 / 12.0) - (d4x + d4y + d4z) * (1.0 / 240.0) + sx * (1.0 / 90.0) -
                     h * h * kl * f0 * (1.0 / 20.0) + h * h * h * kzl * d1z * (1.0 / 60.0));
      }
    }
    // lift of the z-face data (both faces when nz = 1)
    auto plane9m = [&](const double* w, const double* Pl) -> double {
      return w[0] * (Pl[off[5]] + Pl[off[6]] + Pl[off[7]] + Pl[off[8]]) + w[1] * (Pl[off[1]] + Pl[off[2]]) +
             w[2] * (Pl[off[3]] + Pl[off[4]]) + w[3] * Pl[off[0]];
    };
    if (l == 1 && p.glo) F -= plane9m(p.W + 0, p.glo + r * p.g_stride);
    if (l == nz && p.ghi) F -= plane9m(p.W + (nz - 1) * 12 + 8, p.ghi + r * p.g_stride);
    p.u[r * p.u_stride + i + (long long)nx * (j + (long long)ny * (l - 1))] = F;
  };
  // planes lb-2 .. lb+1 into slots (lb-2) mod 5 .. (lb+1) mod 5 = 4, 0, 1, 2
  load(ring[4], lb - 2);
  load(ring[0], lb - 1);
  load(ring[1], lb);
  load(ring[2], lb + 1);
  using std::integral_constant;
  for (int l = lb; l <= le; l += 5) {
    load(ring[3], l + 2);
    plane(l, integral_constant<int, 1>{});
    if (l + 1 > le) break;
    load(ring[4], l + 3);
    plane(l + 1, integral_constant<int, 2>{});
    if (l + 2 > le) break;
    load(ring[0], l + 4);
    plane(l + 2, integral_constant<int, 3>{});
    if (l + 3 > le) break;
    load(ring[1], l + 5);
    plane(l + 3, integral_constant<int, 4>{});
    if (l + 4 > le) break;
    load(ring[2], l + 6);
    plane(l + 4, integral_constant<int, 0>{});
  }
}

// ---------------------------------------------------------------------------
// K1: DST along x of 8 lines of F, transposed store into y-lines.  Persistent:
// each workgroup walks tiles t = t0, t0 + gridDim.x, ... (t0 its XCD-ordered index; 8 y-lines
// of one plane of one right-hand side each) and loads the rows of its next tile
// into registers while it transforms the current one.
// LDS: 8 line buffers (the transpose tile overlays them) + twiddle table.
// ---------------------------------------------------------------------------
constexpr int kNV = 16;  // ceil(1023/64): row values per lane
constexpr int kXRows = 64 * kTileJ / kTileJ;  // tile rows one pass of an x-pass workgroup covers
constexpr int kMaxLine = 1023;                // longest x line of the x passes (interior points)

struct XTile {
  int jt, l, r, j;
  bool active;
};

__device__ __forceinline__ XTile decode_xtile(const ProbDev& p, int t, int w) {
  const int njt = p.ldy / kTileJ;
  XTile x;
  x.jt = t % njt;
  x.l = (t / njt) % p.nz + 1;
  x.r = t / (njt * p.nz);
  x.j = x.jt * kTileJ + w;
  x.active = x.j >= 1 && x.j <= p.ny;
  return x;
}

// K1 workgroups that take the tiles in pairs (see k_fwd_x); the host sizes the grid by it
template <typename T, int MX>
__host__ __device__ constexpr bool x_tile_pairs() {
  return sizeof(T) == 8 && MX >= 512;
}

// TI: element type of the input p.F (FP32 for the residuals of the mixed path)
template <typename T, int MX, int KIND = kDst, typename TI = double>
__global__ void __launch_bounds__(64 * kTileJ) k_fwd_x(ProbDev p, int ntiles) {
  extern __shared__ __align__(16) double smem_raw[];
  T* smem = reinterpret_cast<T*>(smem_raw);
  constexpr int NS = Tx<MX, 1, KIND>::NS;
  const int w = threadIdx.x >> 6, lane = threadIdx.x & 63;
  const int bufn = line_buf_elems<T, MX, 1>(p.nx);
  const int ts = tile_stride(p.nx);
  cx<T>* tab = lds_table(smem + kTileJ * (bufn > ts ? bufn : ts));  // after lines / tile
  if constexpr (MX != 0) load_twiddles<T, MX, 1>(tab, p.twx);
  T* buf = smem + w * bufn;
  TI pre[kNV];
  auto fetch = [&](int t) {
    const XTile x = decode_xtile(p, t, w);
    const int ln = opaque(lane);
    const TI* Fr = reinterpret_cast<const TI*>(p.F) + x.r * p.u_stride +
                   (long long)p.nx * ((x.j - 1) + (long long)p.ny * (x.l - 1)) + ln;
#pragma unroll
    for (int k = 0; k < kNV; ++k) pre[k] = (x.active && ln + 64 * k < p.nx) ? Fr[64 * k] : (TI)0;
  };
  auto fill = [&]() {
    if (lane == 0) buf[0] = (T)0;
#pragma unroll
    for (int k = 0; k < kNV; ++k) {
      const int i = 1 + lane + 64 * k;
      if (i <= p.nx) buf[i] = (T)pre[k];
    }
  };
  if constexpr (x_tile_pairs<T, MX>()) {
    // FP64 lines of 512 or more points: tiles 2q and 2q + 1 (y-lines jt 8 .. jt 8 + 15 of one
    // plane, jt even: the rows of G are a multiple of 16 long) fill the two halves of the same
    // 128-byte lines of G.  One workgroup transforms both, one after the other, and every
    // thread stores its values of the two back to back, so each line is written whole; with
    // one tile per workgroup the halves were written apart and 13 % more bytes than the field
    // reached HBM (K1 at 1023^3 x 4: 19.8-20.3 -> 18.1-18.3 ms).  Shorter lines keep one tile
    // per workgroup: the second tile's values raise their registers past four waves per SIMD.
    constexpr int NT = (kMaxLine + kXRows - 1) / kXRows;  // rows per thread for the longest line
    const int npairs = ntiles / 2;
    // x-transform of the tile whose rows pre holds, transposed into the LDS tile; thread
    // (n0, jj) then reads modes n0 + 1, n0 + 65, ... of line jj into v.  `next` is fetched
    // into pre once the rows are in the line buffers (-1: none).
    auto tile = [&](int t, int next, T(&v)[NT]) {
      const XTile x = decode_xtile(p, t, w);
      __syncthreads();  // every read of the previous tile is done with the LDS
      settle(pre);
      fill();
      if (next >= 0) fetch(next);  // in flight during the transform
      __syncthreads();              // also publishes the twiddle table on the first pass
      T out[NS];
      if (x.active) line_dst<T, MX, 1, false, KIND>(buf, p.nx, out, lane, tab, p.sinx);
      __syncthreads();
      if (x.active) {
#pragma unroll
        for (int s = 0; s < NS; ++s) {
          const int n = line_mode<MX, 1, KIND>(lane, s, p.nx);
          if (n > 0) smem[w * ts + n] = out[s];
        }
      } else {
        for (int n = 1 + lane; n <= p.nx; n += 64) smem[w * ts + n] = (T)0;
      }
      __syncthreads();
      const int tid = opaque((int)threadIdx.x);
      const int n0 = tid / kTileJ, jj = tid % kTileJ;
      const T* row = smem + jj * ts + n0 + 1;
#pragma unroll
      for (int k = 0; k < NT; ++k) v[k] = (n0 + kXRows * k < p.nx) ? row[kXRows * k] : (T)0;
    };
    int q = xcd_order(blockIdx.x, gridDim.x);
    if (q < npairs) fetch(2 * q);
    for (; q < npairs; q += gridDim.x) {
      const int qn = q + (int)gridDim.x;
      T va[NT], vb[NT];
      tile(2 * q, 2 * q + 1, va);
      tile(2 * q + 1, qn < npairs ? 2 * qn : -1, vb);
      const XTile x = decode_xtile(p, 2 * q, w);
      const int tid = opaque((int)threadIdx.x);
      const int n0 = tid / kTileJ, jj = tid % kTileJ;
      T* G = reinterpret_cast<T*>(p.G) + x.r * p.G_stride + (long long)(x.l - 1) * p.nx * p.ldy + x.jt * kTileJ +
             (long long)n0 * p.ldy + jj;
      const long long step = (long long)kXRows * p.ldy;
#pragma unroll
      for (int k = 0; k < NT; ++k) {
        if (n0 + kXRows * k < p.nx) {
          G[k * step] = va[k];
          G[k * step + kTileJ] = vb[k];
        }
      }
    }
    return;
  }
  int t = xcd_order(blockIdx.x, gridDim.x);
  if (t < ntiles) fetch(t);
  settle(pre);  // (every path into the loop arrives with settled rows)
  for (; t < ntiles; t += gridDim.x) {
    const XTile x = decode_xtile(p, t, w);
    __syncthreads();  // the previous tile's store phase is done with the LDS
    if (lane == 0) buf[0] = (T)0;
#pragma unroll
    for (int k = 0; k < kNV; ++k) {
      const int i = 1 + lane + 64 * k;
      if (i <= p.nx) buf[i] = (T)pre[k];
    }
    if (t + (int)gridDim.x < ntiles) fetch(t + gridDim.x);  // in flight during the transform
    __syncthreads();  // also publishes the twiddle table on the first pass
    T out[NS];
    if (x.active) line_dst<T, MX, 1, false, KIND>(buf, p.nx, out, lane, tab, p.sinx);
    __syncthreads();
    // tile[jj][n], n = 1..nx, odd row stride
    if (x.active) {
#pragma unroll
      for (int s = 0; s < NS; ++s) {
        const int n = line_mode<MX, 1, KIND>(lane, s, p.nx);
        if (n > 0) smem[w * ts + n] = out[s];
      }
    } else {
      for (int n = 1 + lane; n <= p.nx; n += 64) smem[w * ts + n] = (T)0;
    }
    __syncthreads();
    settle(pre);  // the next tile's rows, fetched before the transform
    // store phase.  FP64: thread (n0, jj) moves modes n0 + 1, n0 + 65, ... of line jj, all
    // of its LDS reads issued before its stores, so the LDS latency is paid once per tile
    // rather than once per element (K1 at 1023^3 x 4, one tile per workgroup: 20.6 -> 20.1
    // ms).  FP32 keeps the element loop, which measured faster there (39.5 against 43.5 ms
    // for the three launches of a mixed solve).
    if constexpr (sizeof(T) == 4) {
      T* G = reinterpret_cast<T*>(p.G) + x.r * p.G_stride + (long long)(x.l - 1) * p.nx * p.ldy + x.jt * kTileJ;
      for (int idx = threadIdx.x; idx < p.nx * kTileJ; idx += blockDim.x) {
        const int n0 = idx / kTileJ, jj = idx % kTileJ;
        G[(long long)n0 * p.ldy + jj] = smem[jj * ts + n0 + 1];
      }
    } else {
      const int tid = opaque((int)threadIdx.x);
      const int n0 = tid / kTileJ, jj = tid % kTileJ;
      const T* row = smem + jj * ts + n0 + 1;
      T* G = reinterpret_cast<T*>(p.G) + x.r * p.G_stride + (long long)(x.l - 1) * p.nx * p.ldy + x.jt * kTileJ +
             (long long)n0 * p.ldy + jj;
      const long long step = (long long)kXRows * p.ldy;
      constexpr int NT = (kMaxLine + kXRows - 1) / kXRows;  // rows per thread for the longest line
      T v[NT];
#pragma unroll
      for (int k = 0; k < NT; ++k) v[k] = (n0 + kXRows * k < p.nx) ? row[kXRows * k] : (T)0;
#pragma unroll
      for (int k = 0; k < NT; ++k) {
        if (n0 + kXRows * k < p.nx) G[k * step] = v[k];
      }
    }
  }
}

// ---------------------------------------------------------------------------
// K1 with two wavefronts per x-line (FFT lengths 512 and 1024): the same tiles of kTileJ
// y-lines, layout, transpose and stores as k_fwd_x, with 1024 threads per workgroup and
// half the values of a line per lane.  The registers of a lane then fit four waves per
// SIMD (one workgroup per CU: the LDS of the line buffers).  Every line of a workgroup
// runs the transform (its exchanges synchronise the workgroup); lines past N_y transform
// zeros and store zeros.
// ---------------------------------------------------------------------------
constexpr int kNV2 = 8;  // ceil(1023/128): row values per lane

template <typename T, int MX, int KIND = kDst, typename TI = double>
__global__ void __launch_bounds__(128 * kTileJ) k_fwd_x2(ProbDev p, int ntiles) {
  static_assert(MX >= 512, "two waves per line need M >= 512");
  extern __shared__ __align__(16) double smem_raw[];
  T* smem = reinterpret_cast<T*>(smem_raw);
  constexpr int NS = Tx<MX, 2, KIND>::NS;
  const int w = threadIdx.x >> 7, tl = threadIdx.x & 127;
  const int bufn = line_buf_elems<T, MX, 2>(p.nx);
  const int ts = tile_stride(p.nx);
  cx<T>* tab = lds_table(smem + kTileJ * (bufn > ts ? bufn : ts));  // after lines / tile
  load_twiddles<T, MX, 2>(tab, p.twx);
  T* buf = smem + w * bufn;
  TI pre[kNV2];
  auto fetch = [&](int t) {
    const XTile x = decode_xtile(p, t, w);
    const int ln = opaque(tl);
    const TI* Fr = reinterpret_cast<const TI*>(p.F) + x.r * p.u_stride +
                   (long long)p.nx * ((x.j - 1) + (long long)p.ny * (x.l - 1)) + ln;
#pragma unroll
    for (int k = 0; k < kNV2; ++k) pre[k] = (x.active && ln + 128 * k < p.nx) ? Fr[128 * k] : (TI)0;
  };
  int t = xcd_order(blockIdx.x, gridDim.x);
  if (t < ntiles) fetch(t);
  settle(pre);
  for (; t < ntiles; t += gridDim.x) {
    const XTile x = decode_xtile(p, t, w);
    __syncthreads();  // the previous tile's store phase is done with the LDS
    if (tl == 0) buf[0] = (T)0;
#pragma unroll
    for (int k = 0; k < kNV2; ++k) {
      const int i = 1 + tl + 128 * k;
      if (i <= p.nx) buf[i] = (T)pre[k];  // zeros for a line past N_y
    }
    if (t + (int)gridDim.x < ntiles) fetch(t + gridDim.x);  // in flight during the transform
    __syncthreads();  // also publishes the twiddle table on the first pass
    T out[NS];
    line_dst<T, MX, 2, false, KIND>(buf, p.nx, out, tl, tab, p.sinx);
    __syncthreads();
    // tile[jj][n], n = 1..nx
    if (x.active) {
#pragma unroll
      for (int s = 0; s < NS; ++s) {
        const int n = line_mode<MX, 2, KIND>(tl, s, p.nx);
        if (n > 0) smem[w * ts + n] = out[s];
      }
    } else {
      for (int n = 1 + tl; n <= p.nx; n += 128) smem[w * ts + n] = (T)0;
    }
    __syncthreads();
    settle(pre);  // the next tile's rows, fetched before the transform
    T* G = reinterpret_cast<T*>(p.G) + x.r * p.G_stride + (long long)(x.l - 1) * p.nx * p.ldy + x.jt * kTileJ;
    for (int idx = threadIdx.x; idx < p.nx * kTileJ; idx += blockDim.x) {
      const int n0 = idx / kTileJ, jj = idx % kTileJ;
      G[(long long)n0 * p.ldy + jj] = smem[jj * ts + n0 + 1];
    }
  }
}

// ---------------------------------------------------------------------------
// K2: DST along y + modal eigenvalues + forward elimination.
// ---------------------------------------------------------------------------
// Robin z faces: the first and last rows of a modal system (plane l of 1..nz) after the
// elimination of the ghost planes (the face rows of the system's first and last plane)
__device__ __forceinline__ void robin_rows(const ProbDev& p, int l, double sn, double sm, double& lm,
                                           double& l0, double& lp) {
  const double mu = -2.0 * sn / (p.hx * p.hx) - 2.0 * sm / (p.hy * p.hy);
  if (l == 1) {
    l0 += (p.rb[0] + p.rb[1] * mu) * lm;
    lp += lm;
  }
  if (l == p.nz) {
    l0 += (p.rb[2] + p.rb[3] * mu) * lp;
    lm += lp;
  }
}

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

// waves per line in the y passes (1, or 2 for M >= 512); the default is two for the
// 1024-point FFT and one otherwise, the autotuner may pick the other one
template <int MY>
constexpr int default_wpl() { return MY == 1024 ? 2 : 1; }

// PACK: the lines of 64- and 128-point transforms take the M/4 lanes their FFT uses, so
// a wave carries 4 or 2 lines (batches; see the batch tuning); else each line has whole waves
template <int MY, int WPL, bool PACK>
__host__ __device__ constexpr int ycfg_lanes() {
  if constexpr (PACK) {
    return FftGeom<MY, 1>::L;
  } else {
    return 64 * WPL;
  }
}

template <int MY, int WPL_ = default_wpl<MY>(), int KIND = kDst, bool PACK = false>
struct YCfg {
  static_assert(!PACK || ((MY == 64 || MY == 128) && WPL_ == 1 && KIND == kDst), "packed lines: 64 or 128 points");
  static constexpr int WPL = WPL_;
  static constexpr int LANES = ycfg_lanes<MY, WPL_, PACK>();
  static constexpr int LPB = kBlockY / LANES;  // lines (x-modes) per workgroup
  static constexpr int NS = Tx<MY, WPL, KIND>::NS;
  // line values loaded per lane (positions 0..N; N = M + 1 for the cosine transform)
  static constexpr int NLD = ((MY ? MY + (KIND == kDct ? 2 : 0) : 1024) + LANES - 1) / LANES;
  // most right-hand sides one workgroup carries: their tridiagonal systems share the
  // eigenvalues and pivots (formed once per plane and mode) and c' (read once in the
  // back pass); one where a lane holds 16 modes (register budget)
  static constexpr int NRMAX = (NS <= 8 && KIND == kDst) ? 4 : 1;
};

// Paired exchanges (wave_dst.hpp) in the real y passes, FP64 at M = 1024 with two waves per
// line; they double the line buffers (16-byte entries).  K2 (FWD) takes them: 21.9 -> 21.5
// ms at 1023^3 x 4.  K3 does not: no gain there (20.2-20.6 ms either way), and its larger
// buffers would cap it at two workgroups per CU.
#ifndef CS3D_PAIR_K2
#define CS3D_PAIR_K2 1
#endif
#ifndef CS3D_PAIR_K3
#define CS3D_PAIR_K3 0
#endif
template <typename T, int MY, int WPL, bool FWD>
__host__ __device__ constexpr bool ypair() {
  return pair_exchange_ok<T, MY, WPL>() && (FWD ? CS3D_PAIR_K2 : CS3D_PAIR_K3);
}

// twiddle tables of a y pass, loaded by the whole block (a barrier follows)
template <typename T, int MY, int WPL, bool PAIR = false>
__device__ __forceinline__ cx<T>* y_tables(const ProbDev& p, T* smem, bool load) {
  const int bufn = line_buf_elems<T, MY, WPL, PAIR>(p.ny);
  cx<T>* tab = lds_table(smem + YCfg<MY, WPL>::LPB * bufn);
  if constexpr (MY != 0) {
    if (load) load_twiddles<T, MY, WPL>(tab, p.twy);
  }
  __syncthreads();
  return tab;
}

// Lines n = g LPB + 1 .. of right-hand sides r0 .. r0 + nr - 1 (nr <= NR; tables already
// in LDS).  Per plane l the lines of the nr right-hand sides are transformed one after
// the other through the same line buffer; the modal eigenvalues, the pivot and c' of
// every mode are formed with the first of them and applied to all (the LU of Section
// 3.6 does not depend on the right-hand side).  The workgroup of r0 = 0 stores c' and
// records the pivots.
// ROBIN: Robin z faces, whose first and last modal rows change (robin_rows)
template <typename T, int MY, int WPL, int NR, int KIND = kDst, bool ROBIN = false, bool PACK = false>
__device__ __forceinline__ void yfwd_block(const ProbDev& p, int g, int r0, int nr, T* smem, const cx<T>* tab) {
  using C = YCfg<MY, WPL, KIND, PACK>;
  constexpr int NS = C::NS;
  const int bufn = line_buf_elems<T, MY, WPL, ypair<T, MY, WPL, true>()>(p.ny);
  const int line = threadIdx.x / C::LANES, tl = threadIdx.x % C::LANES;
  const int n = g * C::LPB + line + 1;
  const bool active = n <= p.nx;
  if constexpr (WPL == 1 && !PACK) {
    if (!active) return;  // no workgroup barrier below for single-wave lines
  }
  // (packed lines share a wave and its pivot reduction at the end: an inactive one runs on
  // zeros like the inactive lines of two-wave lines)
  T* buf = smem + line * bufn;
  const double ctn = active ? p.ctx[n - 1] : 0.0;
  // s_m of each slot's mode is the same on every plane: held in registers where they allow
  // it (FP64, one right-hand side per workgroup), else read per plane
  constexpr bool kHoistS = sizeof(T) == 8 && NR == 1;
  double cp[NS], dp[NR][NS], lmv[NS], inv[NS], smv[kHoistS ? NS : 1];
#pragma unroll
  for (int s = 0; s < NS; ++s) {
    cp[s] = 0.0;
#pragma unroll
    for (int r = 0; r < NR; ++r) dp[r][s] = 0.0;
    if constexpr (kHoistS) {
      const int m = line_mode<MY, WPL, KIND>(tl, s, p.ny);
      smv[s] = p.cty[(active && m > 0 ? m : 1) - 1];
    }
  }
  double minpiv = 1.0e308;
  unsigned bad = 0;
  const bool lead = (r0 == 0);  // stores c' and records the pivots
  const long long lstride = (long long)p.nx * p.ldy;
  const long long nbase = (long long)(active ? n - 1 : 0) * p.ldy;
  T* G0 = reinterpret_cast<T*>(p.G) + r0 * p.G_stride;
  // prefetch of the line of the next (plane, right-hand side) pair.  Every lane issues
  // every load and every store of a step (positions outside the line, and the whole of
  // an inactive line, go to position 0 of the row, which no pass reads as data), so the
  // number of memory operations in flight is fixed and the wait for the prefetched line
  // does not also wait for the stores of the step before.
  T pre[C::NLD];
  auto fetch = [&](int l, int r) {
    const T* row = G0 + r * p.G_stride + (long long)(l - 1) * lstride + nbase;
    const int tlo = opaque(tl);
#pragma unroll
    for (int s = 0; s < C::NLD; ++s) {
      const int e = tlo + C::LANES * s;
      if constexpr (kHoistS) {
        // (opaque: one load per slot, not a shared load of position 0 plus copies)
        pre[s] = row[opaque((active && e <= p.ny) ? e : 0)];  // an inactive line is filled with zeros below
      } else {
        pre[s] = (active && e <= p.ny) ? row[e] : (T)0;
      }
    }
  };
  fetch(1, 0);
  settle(pre);
  for (int l = 1; l <= p.nz; ++l) {
#pragma unroll
    for (int r = 0; r < NR; ++r) {
      if (r >= nr) break;
      T* line_p = G0 + r * p.G_stride + (long long)(l - 1) * lstride + nbase;
#pragma unroll
      for (int s = 0; s < C::NLD; ++s) {
        const int e = tl + C::LANES * s;
        if constexpr (MY != 0 && KIND == kDst) {
          buf[e] = active ? pre[s] : (T)0;  // e < M = N + 1: always a position of the line
        } else {
          if (e <= p.ny) buf[e] = active ? pre[s] : (T)0;
        }
      }
      line_sync<WPL>();
      if (r + 1 < nr) fetch(l, r + 1);
      else if (l < p.nz) fetch(l + 1, 0);
      T out[NS] = {};  // lanes past the FFT's own take part with zeros
      line_dst<T, MY, WPL, false, KIND, ypair<T, MY, WPL, true>()>(buf, p.ny, out, tl, tab, p.siny);
      settle(pre);  // the next line, fetched before the transform
      if (r == 0) {
        // lambda^o = beta^o + s_m alpha^o with beta = Z + s_n B, alpha = C + A s_n
        const double* Ll = p.LC + (l - 1) * 12;
        const double bm = Ll[0] + ctn * Ll[1], am = Ll[2] + Ll[3] * ctn;
        const double b0 = Ll[4] + ctn * Ll[5], a0 = Ll[6] + Ll[7] * ctn;
        const double bp = Ll[8] + ctn * Ll[9], ap = Ll[10] + Ll[11] * ctn;
        double* Cl = p.C + (long long)(l - 1) * lstride + nbase;
        if constexpr (kHoistS && NR == 1) {
          // one right-hand side: each mode's pivot is applied to d' at once, so no array of
          // eigenvalues and reciprocals stays live across the modes
#pragma unroll
          for (int s = 0; s < NS; ++s) {
            const int m = line_mode<MY, WPL, KIND>(tl, s, p.ny);
            const bool valid = active && m > 0;
            const double sm = smv[s];
            double lm = am * sm + bm, l0 = a0 * sm + b0, lpv = ap * sm + bp;
            if constexpr (ROBIN) robin_rows(p, l, ctn, sm, lm, l0, lpv);
            const double piv = l0 - lm * cp[s];
            if (lead && valid) record_pivot(piv, minpiv, bad);
            const double iv = 1.0 / piv;
            cp[s] = lpv * iv;
            if (lead) Cl[valid ? m : 0] = cp[s];
            dp[0][s] = ((double)out[s] - lm * dp[0][s]) * iv;
            line_p[valid ? m : 0] = (T)dp[0][s];
          }
        } else if constexpr (kHoistS) {
#pragma unroll
          for (int s = 0; s < NS; ++s) {
            const int m = line_mode<MY, WPL, KIND>(tl, s, p.ny);
            const bool valid = active && m > 0;
            const double sm = smv[s];
            double lm = am * sm + bm, l0 = a0 * sm + b0, lpv = ap * sm + bp;
            if constexpr (ROBIN) robin_rows(p, l, ctn, sm, lm, l0, lpv);
            const double piv = l0 - lm * cp[s];
            if (lead && valid) record_pivot(piv, minpiv, bad);
            inv[s] = 1.0 / piv;
            lmv[s] = lm;
            cp[s] = lpv * inv[s];
            if (lead) Cl[valid ? m : 0] = cp[s];
          }
        } else if (active) {
#pragma unroll
          for (int s = 0; s < NS; ++s) {
            const int m = line_mode<MY, WPL, KIND>(tl, s, p.ny);
            if (m > 0) {
              const double sm = p.cty[m - 1];
              double lm = am * sm + bm, l0 = a0 * sm + b0, lpv = ap * sm + bp;
              if constexpr (ROBIN) robin_rows(p, l, ctn, sm, lm, l0, lpv);
              const double piv = l0 - lm * cp[s];
              if (lead) record_pivot(piv, minpiv, bad);
              inv[s] = 1.0 / piv;
              lmv[s] = lm;
              cp[s] = lpv * inv[s];
              if (lead) Cl[m] = cp[s];
            }
          }
        }
      }
      if constexpr (kHoistS && NR == 1) {
        // (applied with the pivots above)
      } else if constexpr (kHoistS) {
#pragma unroll
        for (int s = 0; s < NS; ++s) {
          const int m = line_mode<MY, WPL, KIND>(tl, s, p.ny);
          const bool valid = active && m > 0;
          dp[r][s] = ((double)out[s] - lmv[s] * dp[r][s]) * inv[s];
          line_p[valid ? m : 0] = (T)dp[r][s];
        }
      } else if (active) {
#pragma unroll
        for (int s = 0; s < NS; ++s) {
          const int m = line_mode<MY, WPL, KIND>(tl, s, p.ny);
          if (m > 0) {
            dp[r][s] = ((double)out[s] - lmv[s] * dp[r][s]) * inv[s];
            line_p[m] = (T)dp[r][s];
          }
        }
      }
      line_sync<WPL>();
    }
  }
  if (lead && (active || WPL > 1 || PACK)) flush_stats(p, minpiv, bad);
}

// grid: (line groups, groups of NR right-hand sides)
template <typename T, int MY, int WPL, int NR, int KIND = kDst, bool ROBIN = false>
__global__ void __launch_bounds__(kBlockY) k_fwd_y(ProbDev p, int nrhs) {
  extern __shared__ __align__(16) double smem_raw[];
  T* smem = reinterpret_cast<T*>(smem_raw);
  const cx<T>* tab = y_tables<T, MY, WPL, ypair<T, MY, WPL, true>()>(p, smem, true);
  const int r0 = blockIdx.y * NR;
  yfwd_block<T, MY, WPL, NR, KIND, ROBIN>(p, blockIdx.x, r0, min(NR, nrhs - r0), smem, tab);
}

// ---------------------------------------------------------------------------
// K3: back substitution + inverse DST along y, the right-hand sides of a workgroup
// sharing each read of c'.
// ---------------------------------------------------------------------------
template <typename T, int MY, int WPL, int NR, int KIND = kDst, bool PACK = false>
__device__ __forceinline__ void yback_block(const ProbDev& p, int g, int r0, int nr, T* smem, const cx<T>* tab) {
  using C = YCfg<MY, WPL, KIND, PACK>;
  constexpr int NS = C::NS;
  const int bufn = line_buf_elems<T, MY, WPL, ypair<T, MY, WPL, false>()>(p.ny);
  const int line = threadIdx.x / C::LANES, tl = threadIdx.x % C::LANES;
  const int n = g * C::LPB + line + 1;
  const bool active = n <= p.nx;
  if constexpr (WPL == 1) {
    if (!active) return;
  }
  T* buf = smem + line * bufn;
  double Wn[NR][NS];
  int mpos[NS];
#pragma unroll
  for (int s = 0; s < NS; ++s) {
    mpos[s] = active ? line_mode<MY, WPL, KIND>(tl, s, p.ny) : -1;
#pragma unroll
    for (int r = 0; r < NR; ++r) Wn[r][s] = 0.0;
  }
  T* G0 = reinterpret_cast<T*>(p.G) + r0 * p.G_stride;
  const long long lstride = (long long)p.nx * p.ldy;
  const long long nbase = (long long)(active ? n - 1 : 0) * p.ldy;
  // prefetch: d' of the next (plane, right-hand side) pair, c' of the next plane
  T pd[NS];
  double pc[NS], pcn[NS];
  auto fetch_d = [&](int l, int r) {
    const T* src = G0 + r * p.G_stride + (long long)(l - 1) * lstride + nbase;
#pragma unroll
    for (int s = 0; s < NS; ++s) pd[s] = mpos[s] > 0 ? src[mpos[s]] : (T)0;
  };
  auto fetch_c = [&](int l, double(&dst)[NS]) {
    const double* src = p.C + (long long)(l - 1) * lstride + nbase;
#pragma unroll
    for (int s = 0; s < NS; ++s) dst[s] = mpos[s] > 0 ? src[mpos[s]] : 0.0;
  };
  fetch_d(p.nz, 0);
  fetch_c(p.nz, pc);
  settle(pd);
  settle(pc);
  for (int l = p.nz; l >= 1; --l) {
#pragma unroll
    for (int r = 0; r < NR; ++r) {
      if (r >= nr) break;
      T* line_p = G0 + r * p.G_stride + (long long)(l - 1) * lstride + nbase;
#pragma unroll
      for (int s = 0; s < NS; ++s)
        if (mpos[s] > 0) Wn[r][s] = (double)pd[s] - pc[s] * Wn[r][s];
      if constexpr (MY != 0 && KIND == kDst) {
        // modes 2q and 2q+1 of a lane are adjacent: one 16-byte store per pair (the
        // slot of mode 0 is written but never read)
        if (tl < FftGeom<MY, WPL>::L) {
#pragma unroll
          for (int s = 0; s < NS; s += 2) {
            using V2 = typename std::conditional<sizeof(T) == 8, double2, float2>::type;
            V2 w2;
            w2.x = (T)Wn[r][s];
            w2.y = (T)Wn[r][s + 1];
            *reinterpret_cast<V2*>(buf + 2 * (tl + FftGeom<MY, WPL>::L * (s >> 1))) = w2;
          }
        }
      } else {
#pragma unroll
        for (int s = 0; s < NS; ++s)
          if (mpos[s] > 0) buf[mpos[s]] = (T)Wn[r][s];
      }
      line_sync<WPL>();
      if (r + 1 < nr) {
        fetch_d(l, r + 1);
      } else if (l > 1) {
        fetch_d(l - 1, 0);
      }
      if (r == 0 && l > 1) fetch_c(l - 1, pcn);
      T out[NS];
      line_dst<T, MY, WPL, false, KIND, ypair<T, MY, WPL, false>()>(buf, p.ny, out, tl, tab, p.siny);
      settle(pd);  // d' and c' of the next step, fetched before the transform
      settle(pcn);
#pragma unroll
      for (int s = 0; s < NS; ++s)
        if (mpos[s] > 0) line_p[mpos[s]] = out[s];
      line_sync<WPL>();
    }
#pragma unroll
    for (int s = 0; s < NS; ++s) pc[s] = pcn[s];
  }
}

template <typename T, int MY, int WPL, int NR, int KIND = kDst>
__global__ void __launch_bounds__(kBlockY) k_back_y(ProbDev p, int nrhs) {
  extern __shared__ __align__(16) double smem_raw[];
  T* smem = reinterpret_cast<T*>(smem_raw);
  const cx<T>* tab = y_tables<T, MY, WPL, ypair<T, MY, WPL, false>()>(p, smem, true);
  // work index in XCD order, right-hand-side groups fastest: the workgroups of one line
  // group (every right-hand side) run at the same time on one XCD and march over the planes
  // together, so the c' rows they all read come from that XCD's L2 after the first
  const int nrg = gridDim.y;
  const int L = xcd_order(linear_block(), gridDim.x * nrg);
  const int r0 = (L % nrg) * NR;
  yback_block<T, MY, WPL, NR, KIND>(p, L / nrg, r0, min(NR, nrhs - r0), smem, tab);
}

// ---------------------------------------------------------------------------
// K4: transposed load of 8 y-lines, inverse DST along x, scale, store u.
// Persistent like K1: the next tile's y-line segments are loaded into registers
// while the current tile is transformed.
// ---------------------------------------------------------------------------
#ifndef CS3D_INV_PREFETCH
#define CS3D_INV_PREFETCH 1
#endif
// K4 register prefetch of the next tile (on: the loads of the next tile fly during the transform)
constexpr bool kInvPrefetch = CS3D_INV_PREFETCH != 0;

// ACC: u += the result (refinement corrections) instead of u = the result
template <typename T, int MX, int KIND = kDst, bool ACC = false>
__global__ void __launch_bounds__(64 * kTileJ) k_inv_x(ProbDev p, int ntiles) {
  extern __shared__ __align__(16) double smem_raw[];
  T* smem = reinterpret_cast<T*>(smem_raw);
  constexpr int NS = Tx<MX, 1, KIND>::NS;
  // FIXED: as in k_fwd_x, a fixed number of loads and stores per lane and tile (sine FFT of
  // 256..1024 points, plain stores)
  constexpr bool FIXED = KIND == kDst && MX >= 256 && !ACC;
  constexpr int NT = FIXED ? MX / 64 : (1023 * kTileJ + 64 * kTileJ - 1) / (64 * kTileJ);  // values per thread
  const int w = threadIdx.x >> 6, lane = threadIdx.x & 63;
  const int bufn = line_buf_elems<T, MX, 1>(p.nx);
  const int ts = tile_stride(p.nx);
  cx<T>* tab = lds_table(smem + kTileJ * (bufn > ts ? bufn : ts));  // after lines / tile
  if constexpr (MX != 0) load_twiddles<T, MX, 1>(tab, p.twx);
  T* buf = smem + w * bufn;
  T pre[NT];
  // thread (n0, jj) moves rows n0, n0 + 64, ... of column jj of the tile; the offsets
  // are rebuilt per tile from an opaque thread index (kept live across the tile loop,
  // one 64-bit offset per row would exhaust the registers)
  auto fetch = [&](int t) {
    const XTile x = decode_xtile(p, t, 0);
    const int tid = opaque((int)threadIdx.x);
    const int n0 = tid / kTileJ, jj = tid % kTileJ;
    if constexpr (FIXED) {
      const T* G = reinterpret_cast<const T*>(p.G) + x.r * p.G_stride + (long long)(x.l - 1) * p.nx * p.ldy +
                   x.jt * kTileJ + jj;
#pragma unroll
      for (int k = 0; k < NT; ++k) {
        const int row = n0 + kXRows * k;
        pre[k] = G[(long long)opaque(row < p.nx ? row : 0) * p.ldy];  // row M - 1: a valid stand-in
      }
    } else {
      const T* G = reinterpret_cast<const T*>(p.G) + x.r * p.G_stride + (long long)(x.l - 1) * p.nx * p.ldy +
                   x.jt * kTileJ + (long long)n0 * p.ldy + jj;
      const long long step = (long long)kXRows * p.ldy;
#pragma unroll
      for (int k = 0; k < NT; ++k) pre[k] = (n0 + kXRows * k < p.nx) ? G[k * step] : (T)0;
    }
  };
  int t = xcd_order(blockIdx.x, gridDim.x);
  if (kInvPrefetch && t < ntiles) fetch(t);
  settle(pre);
  for (; t < ntiles; t += gridDim.x) {
    const XTile x = decode_xtile(p, t, w);
    if (!kInvPrefetch) fetch(t);
    __syncthreads();  // the previous transform is done with the LDS
    {
      const int tid = opaque((int)threadIdx.x);
      const int n0 = tid / kTileJ, jj = tid % kTileJ;
      T* row = smem + jj * ts + n0 + 1;
#pragma unroll
      for (int k = 0; k < NT; ++k) {
        if constexpr (FIXED) {
          row[kXRows * k] = pre[k];  // position M of the tile row is not read by the transform
        } else {
          if (n0 + kXRows * k < p.nx) row[kXRows * k] = pre[k];
        }
      }
    }
    __syncthreads();  // also publishes the twiddle table on the first pass
    if (kInvPrefetch && t + (int)gridDim.x < ntiles) fetch(t + gridDim.x);  // in flight during the transform
    // the transform reads its input straight from tile row w; the workgroup barrier
    // inside separates those reads from the exchanges that overlay the tile
    T out[NS];
    line_dst<T, MX, 1, true, KIND>(buf, p.nx, out, lane, tab, p.sinx, smem + w * ts);
    if (kInvPrefetch) settle(pre);  // the next tile's segments, fetched before the transform
    if (x.active) {
      double* u = p.u + x.r * p.u_stride + (long long)p.nx * ((x.j - 1) + (long long)p.ny * (x.l - 1));
#pragma unroll
      for (int s = 0; s < NS; ++s) {
        const int i = line_mode<MX, 1, KIND>(lane, s, p.nx);
        if constexpr (FIXED) {
          // the one slot without a mode (lane 0, mode 0) writes u[0] with the value of its
          // own slot 1 (mode 1), which stores it too
          u[i > 0 ? i - 1 : 0] = p.scale * (double)(i > 0 ? out[s] : out[1]);
        } else if constexpr (ACC) {
          if (i > 0) u[i - 1] = u[i - 1] + p.scale * (double)out[s];
        } else {
          if (i > 0) u[i - 1] = p.scale * (double)out[s];
        }
      }
    }
  }
}

// ---------------------------------------------------------------------------
// K4 with two wavefronts per x-line (FFT lengths 512 and 1024): the tiles, transposes and
// stores of k_inv_x with 1024 threads per workgroup and half a line per lane.  Every line
// runs the transform (lines past N_y hold the zeros K1 stored there and store nothing).
// ---------------------------------------------------------------------------
template <typename T, int MX, int KIND = kDst, bool ACC = false>
__global__ void __launch_bounds__(128 * kTileJ) k_inv_x2(ProbDev p, int ntiles) {
  static_assert(MX >= 512, "two waves per line need M >= 512");
  extern __shared__ __align__(16) double smem_raw[];
  T* smem = reinterpret_cast<T*>(smem_raw);
  constexpr int NS = Tx<MX, 2, KIND>::NS;
  constexpr int XR = 128;  // tile rows one pass of the workgroup covers
  constexpr bool FIXED = KIND == kDst && !ACC;
  constexpr int NT = FIXED ? MX / XR : (1023 + XR - 1) / XR;  // values per thread
  const int w = threadIdx.x >> 7, tl = threadIdx.x & 127;
  const int bufn = line_buf_elems<T, MX, 2>(p.nx);
  const int ts = tile_stride(p.nx);
  cx<T>* tab = lds_table(smem + kTileJ * (bufn > ts ? bufn : ts));  // after lines / tile
  load_twiddles<T, MX, 2>(tab, p.twx);
  T* buf = smem + w * bufn;
  T pre[NT];
  // thread (n0, jj) moves rows n0, n0 + 128, ... of column jj of the tile (offsets rebuilt
  // per tile from an opaque thread index)
  auto fetch = [&](int t) {
    const XTile x = decode_xtile(p, t, 0);
    const int tid = opaque((int)threadIdx.x);
    const int n0 = tid / kTileJ, jj = tid % kTileJ;
    if constexpr (FIXED) {
      const T* G = reinterpret_cast<const T*>(p.G) + x.r * p.G_stride + (long long)(x.l - 1) * p.nx * p.ldy +
                   x.jt * kTileJ + jj;
#pragma unroll
      for (int k = 0; k < NT; ++k) {
        const int row = n0 + XR * k;
        pre[k] = G[(long long)opaque(row < p.nx ? row : 0) * p.ldy];  // row M - 1: a valid stand-in
      }
    } else {
      const T* G = reinterpret_cast<const T*>(p.G) + x.r * p.G_stride + (long long)(x.l - 1) * p.nx * p.ldy +
                   x.jt * kTileJ + (long long)n0 * p.ldy + jj;
      const long long step = (long long)XR * p.ldy;
#pragma unroll
      for (int k = 0; k < NT; ++k) pre[k] = (n0 + XR * k < p.nx) ? G[k * step] : (T)0;
    }
  };
  int t = xcd_order(blockIdx.x, gridDim.x);
  if (t < ntiles) fetch(t);
  settle(pre);
  for (; t < ntiles; t += gridDim.x) {
    const XTile x = decode_xtile(p, t, w);
    __syncthreads();  // the previous transform is done with the LDS
    {
      const int tid = opaque((int)threadIdx.x);
      const int n0 = tid / kTileJ, jj = tid % kTileJ;
      T* row = smem + jj * ts + n0 + 1;
#pragma unroll
      for (int k = 0; k < NT; ++k) {
        if constexpr (FIXED) {
          row[XR * k] = pre[k];  // position M of the tile row is not read by the transform
        } else {
          if (n0 + XR * k < p.nx) row[XR * k] = pre[k];
        }
      }
    }
    __syncthreads();  // also publishes the twiddle table on the first pass
    if (t + (int)gridDim.x < ntiles) fetch(t + gridDim.x);  // in flight during the transform
    // the transform reads its input straight from tile row w; the workgroup barrier
    // inside separates those reads from the exchanges that overlay the tile
    T out[NS];
    line_dst<T, MX, 2, true, KIND>(buf, p.nx, out, tl, tab, p.sinx, smem + w * ts);
    settle(pre);  // the next tile's segments, fetched before the transform
    if (x.active) {
      double* u = p.u + x.r * p.u_stride + (long long)p.nx * ((x.j - 1) + (long long)p.ny * (x.l - 1));
#pragma unroll
      for (int s = 0; s < NS; ++s) {
        const int i = line_mode<MX, 2, KIND>(tl, s, p.nx);
        if constexpr (FIXED) {
          // the one slot without a mode (lane 0, mode 0) writes u[0] with the value of its
          // own slot 1 (mode 1), which stores it too
          u[i > 0 ? i - 1 : 0] = p.scale * (double)(i > 0 ? out[s] : out[1]);
        } else if constexpr (ACC) {
          if (i > 0) u[i - 1] = u[i - 1] + p.scale * (double)out[s];
        } else {
          if (i > 0) u[i - 1] = p.scale * (double)out[s];
        }
      }
    }
  }
}

// ---------------------------------------------------------------------------
// Complex k (absorbing media).  The sine transforms are real, so K0 (per real slot,
// with Re k^2 and the real weights), K1 and K4 run unchanged over the 2 nrhs real
// slots; k_rhs_cx adds the terms that couple the real and imaginary parts, and the
// y passes carry both slots of a complex right-hand side and solve the complex
// tridiagonal systems.
// ---------------------------------------------------------------------------

// F of complex right-hand side q at the planes it touches: the Im k^2 terms of the
// 6th-order operator (every plane) and the Im W terms of the z-face lift (planes 1, nz).
// grid: (ceil(nx ny / 256), planes, complex right-hand sides)
__global__ void __launch_bounds__(256) k_rhs_cx(ProbDev p) {
  const int e = blockIdx.x * 256 + threadIdx.x;
  if (e >= p.nx * p.ny) return;
  const int i = 1 + e % p.nx, j = 1 + e / p.nx;
  const bool h6 = p.scheme == kHelm6;
  const int q = blockIdx.z;
  const long long sy = p.nx + 2, sz = (long long)(p.nx + 2) * (p.ny + 2);
  // 6th order: a z-march over a chunk of planes with f_{l-1}, f_l, f_{l+1} of both parts
  // in registers; otherwise the two lift planes (blockIdx.y = 0: plane 1, 1: plane nz)
  const int lb = h6 ? 1 + (int)blockIdx.y * kSidesChunk : (blockIdx.y == 0 ? 1 : p.nz);
  const int le = h6 ? min(p.nz, lb + kSidesChunk - 1) : lb;
  const double* fr = (h6 && p.f) ? p.f + (2 * q) * p.f_stride + i + sy * j : nullptr;
  const double* fi = fr ? fr + p.f_stride : nullptr;
  double rm = 0.0, r0 = 0.0, rp = 0.0, im = 0.0, i0 = 0.0, ip = 0.0;
  if (fr) {
    rm = fr[sz * (lb - 1)];
    r0 = fr[sz * lb];
    im = fi[sz * (lb - 1)];
    i0 = fi[sz * lb];
  }
  for (int l = lb; l <= le; ++l) {
    double dre = 0.0, dim = 0.0;  // corrections of Re F and Im F
    if (fr) {
      rp = fr[sz * (l + 1)];
      ip = fi[sz * (l + 1)];
      const double h = p.hz, hz2 = h * h;
      const double ki = p.k2i[l], kzi = p.k2zi[l];
      // -(h^2/20) k^2 f + (h^3/120) (k^2)_z (f_{l+1} - f_{l-1}), imaginary-part products
      dre = hz2 * (h * h * ki * i0 * (1.0 / 20.0) - h * h * h * kzi * (ip - im) * (1.0 / 120.0));
      dim = hz2 * (-h * h * ki * r0 * (1.0 / 20.0) + h * h * h * kzi * (rp - rm) * (1.0 / 120.0));
    }
    // lift: F -= W g with complex W and g; the real parts were lifted per slot
    if (l == 1 && p.glo) {
      const double* gr = p.glo + (2 * q) * p.g_stride;
      dre += plane9(p.Wi + 0, gr + p.g_stride, p.nx, i, j);
      dim -= plane9(p.Wi + 0, gr, p.nx, i, j);
    }
    if (l == p.nz && p.ghi) {
      const double* gr = p.ghi + (2 * q) * p.g_stride;
      const double* w = p.Wi + (p.nz - 1) * 12 + 8;
      dre += plane9(w, gr + p.g_stride, p.nx, i, j);
      dim -= plane9(w, gr, p.nx, i, j);
    }
    double* u = p.u + (2 * q) * p.u_stride + (i - 1) + (long long)p.nx * ((j - 1) + (long long)p.ny * (l - 1));
    u[0] += dre;
    u[p.u_stride] += dim;
    rm = r0;
    r0 = rp;
    im = i0;
    i0 = ip;
  }
}

__device__ __forceinline__ void record_pivot_c(double pr, double pi, double& minpiv, unsigned& bad) {
  const double a = hypot(pr, pi);
  if (!(a > 0.0) || !isfinite(a)) {
    ++bad;
  } else if (a < minpiv) {
    minpiv = a;
  }
}

// y-DST of the two slots of complex right-hand side q, complex modal eigenvalues and
// forward elimination (FP64 transforms)
template <int MY, int WPL>
__device__ __forceinline__ void yfwd_block_c(const ProbDev& p, int g, int q, double* smem, const cx<double>* tab) {
  using C = YCfg<MY, WPL>;
  constexpr int NS = C::NS;
  const int bufn = line_buf_elems<double, MY, WPL>(p.ny);
  const int line = threadIdx.x / C::LANES, tl = threadIdx.x % C::LANES;
  const int n = g * C::LPB + line + 1;
  const bool active = n <= p.nx;
  if constexpr (WPL == 1) {
    if (!active) return;
  }
  double* buf = smem + line * bufn;
  const double ctn = active ? p.ctx[n - 1] : 0.0;
  double cpr[NS], cpi[NS], dpr[NS], dpi[NS], orr[NS], smv[NS];
#pragma unroll
  for (int s = 0; s < NS; ++s) {
    cpr[s] = cpi[s] = dpr[s] = dpi[s] = 0.0;
    const int m = line_mode<MY, WPL>(tl, s, p.ny);
    smv[s] = p.cty[(active && m > 0 ? m : 1) - 1];  // s_m of the slot's mode, the same on every plane
  }
  double minpiv = 1.0e308;
  unsigned bad = 0;
  const bool lead = (q == 0);
  const long long lstride = (long long)p.nx * p.ldy;
  const long long nbase = (long long)(active ? n - 1 : 0) * p.ldy;
  double* G0 = reinterpret_cast<double*>(p.G) + (2 * q) * p.G_stride;
  double pre[C::NLD];
  auto fetch = [&](int l, int part) {
    const double* src = G0 + part * p.G_stride + (long long)(l - 1) * lstride + nbase + opaque(tl);
#pragma unroll
    for (int s = 0; s < C::NLD; ++s) pre[s] = (active && tl + C::LANES * s <= p.ny) ? src[C::LANES * s] : 0.0;
  };
  // the plane's coefficients Z, B, C, A (real parts, then imaginary), loaded just before
  // the second line's prefetch and settled with it: the elimination then waits for no load
  double Lc[24];
  fetch(1, 0);
  settle(pre);
  for (int l = 1; l <= p.nz; ++l) {
#pragma unroll
    for (int part = 0; part < 2; ++part) {
#pragma unroll
      for (int s = 0; s < C::NLD; ++s) {
        const int e = tl + C::LANES * s;
        if (e <= p.ny) buf[e] = pre[s];
      }
      line_sync<WPL>();
      if (part == 0) {
#pragma unroll
        for (int k = 0; k < 12; ++k) {
          Lc[k] = p.LC[(l - 1) * 12 + k];
          Lc[12 + k] = p.LCi[(l - 1) * 12 + k];
        }
        fetch(l, 1);
      } else if (l < p.nz) {
        fetch(l + 1, 0);
      }
      double out[NS];
      line_dst<double, MY, WPL>(buf, p.ny, out, tl, tab, p.siny);
      settle(pre);  // the next line, fetched before the transform
      if (part == 0) {
        settle(Lc);
#pragma unroll
        for (int s = 0; s < NS; ++s) orr[s] = out[s];
      } else if (active) {
        const double* Lr = Lc;
        const double* Li = Lc + 12;
        double* Cr = p.C + (long long)(l - 1) * lstride + nbase;
        double* Cim = p.Ci + (long long)(l - 1) * lstride + nbase;
        double* d0 = G0 + (long long)(l - 1) * lstride + nbase;
        double* d1 = d0 + p.G_stride;
#pragma unroll
        for (int s = 0; s < NS; ++s) {
          const int m = line_mode<MY, WPL>(tl, s, p.ny);
          if (m > 0) {
            const double sm = smv[s];
            // lambda^o = (Z + s_n B) + s_m (C + A s_n), real and imaginary parts
            const double lmr = (Lr[2] + Lr[3] * ctn) * sm + (Lr[0] + ctn * Lr[1]);
            const double lmi = (Li[2] + Li[3] * ctn) * sm + (Li[0] + ctn * Li[1]);
            const double l0r = (Lr[6] + Lr[7] * ctn) * sm + (Lr[4] + ctn * Lr[5]);
            const double l0i = (Li[6] + Li[7] * ctn) * sm + (Li[4] + ctn * Li[5]);
            const double lpr = (Lr[10] + Lr[11] * ctn) * sm + (Lr[8] + ctn * Lr[9]);
            const double lpi = (Li[10] + Li[11] * ctn) * sm + (Li[8] + ctn * Li[9]);
            // pivot = l0 - lm c'
            const double pr = l0r - (lmr * cpr[s] - lmi * cpi[s]);
            const double pim = l0i - (lmr * cpi[s] + lmi * cpr[s]);
            if (lead) record_pivot_c(pr, pim, minpiv, bad);
            const double den = 1.0 / (pr * pr + pim * pim);
            const double ir = pr * den, ii = -pim * den;  // 1 / pivot
            const double ncr = lpr * ir - lpi * ii, nci = lpr * ii + lpi * ir;
            // d' = (F - lm d'_prev) / pivot
            const double tr = orr[s] - (lmr * dpr[s] - lmi * dpi[s]);
            const double ti = out[s] - (lmr * dpi[s] + lmi * dpr[s]);
            dpr[s] = tr * ir - ti * ii;
            dpi[s] = tr * ii + ti * ir;
            cpr[s] = ncr;
            cpi[s] = nci;
            d0[m] = dpr[s];
            d1[m] = dpi[s];
            if (lead) {
              Cr[m] = ncr;
              Cim[m] = nci;
            }
          }
        }
      }
      line_sync<WPL>();
    }
  }
  if (lead && (active || WPL > 1)) flush_stats(p, minpiv, bad);
}

template <int MY, int WPL = default_wpl<MY>()>
__global__ void __launch_bounds__(kBlockY) k_fwd_y_c(ProbDev p) {
  extern __shared__ __align__(16) double smem_raw[];
  const cx<double>* tab = y_tables<double, MY, WPL>(p, smem_raw, true);
  yfwd_block_c<MY, WPL>(p, blockIdx.x, blockIdx.y, smem_raw, tab);
}

// complex back substitution, then the inverse y-DST of both slots
template <int MY, int WPL>
__device__ __forceinline__ void yback_block_c(const ProbDev& p, int g, int q, double* smem, const cx<double>* tab) {
  using C = YCfg<MY, WPL>;
  constexpr int NS = C::NS;
  const int bufn = line_buf_elems<double, MY, WPL>(p.ny);
  const int line = threadIdx.x / C::LANES, tl = threadIdx.x % C::LANES;
  const int n = g * C::LPB + line + 1;
  const bool active = n <= p.nx;
  if constexpr (WPL == 1) {
    if (!active) return;
  }
  double* buf = smem + line * bufn;
  double wr[NS], wi[NS], pdr[NS], pdi[NS], pcr[NS], pci[NS];
  int mpos[NS];
#pragma unroll
  for (int s = 0; s < NS; ++s) {
    mpos[s] = active ? line_mode<MY, WPL>(tl, s, p.ny) : -1;
    wr[s] = wi[s] = 0.0;
  }
  double* G0 = reinterpret_cast<double*>(p.G) + (2 * q) * p.G_stride;
  const long long lstride = (long long)p.nx * p.ldy;
  const long long nbase = (long long)(active ? n - 1 : 0) * p.ldy;
  auto fetch = [&](int l) {
    const long long o = (long long)(l - 1) * lstride + nbase;
#pragma unroll
    for (int s = 0; s < NS; ++s) {
      const bool v = mpos[s] > 0;
      pdr[s] = v ? G0[o + mpos[s]] : 0.0;
      pdi[s] = v ? G0[p.G_stride + o + mpos[s]] : 0.0;
      pcr[s] = v ? p.C[o + mpos[s]] : 0.0;
      pci[s] = v ? p.Ci[o + mpos[s]] : 0.0;
    }
  };
  fetch(p.nz);
  settle(pdr);
  settle(pdi);
  settle(pcr);
  settle(pci);
  for (int l = p.nz; l >= 1; --l) {
    // W_l = d'_l - c'_l W_{l+1}
#pragma unroll
    for (int s = 0; s < NS; ++s) {
      if (mpos[s] > 0) {
        const double nr = pdr[s] - (pcr[s] * wr[s] - pci[s] * wi[s]);
        const double ni = pdi[s] - (pcr[s] * wi[s] + pci[s] * wr[s]);
        wr[s] = nr;
        wi[s] = ni;
      }
    }
    if (l > 1) fetch(l - 1);
    double* line0 = G0 + (long long)(l - 1) * lstride + nbase;
#pragma unroll
    for (int part = 0; part < 2; ++part) {
#pragma unroll
      for (int s = 0; s < NS; ++s)
        if (mpos[s] > 0) buf[mpos[s]] = part == 0 ? wr[s] : wi[s];
      line_sync<WPL>();
      double out[NS];
      line_dst<double, MY, WPL>(buf, p.ny, out, tl, tab, p.siny);
      if (part == 0) {  // d' and c' of the next plane, fetched before the transforms
        settle(pdr);
        settle(pdi);
        settle(pcr);
        settle(pci);
      }
      double* dst = line0 + part * p.G_stride;
#pragma unroll
      for (int s = 0; s < NS; ++s)
        if (mpos[s] > 0) dst[mpos[s]] = out[s];
      line_sync<WPL>();
    }
  }
}

template <int MY, int WPL = default_wpl<MY>()>
__global__ void __launch_bounds__(kBlockY) k_back_y_c(ProbDev p) {
  extern __shared__ __align__(16) double smem_raw[];
  const cx<double>* tab = y_tables<double, MY, WPL>(p, smem_raw, true);
  // work order as in k_back_y: the right-hand sides of a line group side by side on one XCD
  const int nq = gridDim.y;
  const int L = xcd_order(linear_block(), gridDim.x * nq);
  yback_block_c<MY, WPL>(p, L / nq, L % nq, smem_raw, tab);
}

// ---------------------------------------------------------------------------
// FP64 residual r = F - A U of eq. stencil27 (the z-face data are in F through the
// lift; U vanishes on every face), with ||r||^2 accumulated into acc.  Tile 64 x 16
// interior points, 512 threads (two y-rows each), marching over kZChunk planes with a
// three-plane window of U (halo 1) in LDS and two planes in flight in registers.
// ---------------------------------------------------------------------------
constexpr int kQTX = 64, kQTY = 16, kQThreads = 512, kQRows = kQTY / (kQThreads / 64);
constexpr int kQWPlanes = 64;  // planes per refill of the residual's weight table (even)
constexpr int kQX = kQTX + 2, kQY = kQTY + 2;
constexpr int kQLoads = (kQX * kQY + kQThreads - 1) / kQThreads;

// TR: element type of r (FP32 where it only feeds an FP32 correction solve); STORE = false
// computes the norm alone (the last residual of a mixed solve)
// accF (may be null): also accumulates ||F||^2 over the same points
template <typename TR, bool STORE>
__global__ void __launch_bounds__(kQThreads) k_residual(ProbDev p, const double* __restrict__ Fi,
                                                        const double* __restrict__ U, TR* __restrict__ R,
                                                        double* acc, double* accF) {
  __shared__ double win[3][kQX * kQY];
  __shared__ double part[kQThreads / 64], partF[kQThreads / 64];
  // the weights of kQWPlanes planes at a time, in LDS (see kt in rhs_block)
  __shared__ double wt[12 * kQWPlanes];
  const int tx = threadIdx.x & 63, ty = threadIdx.x >> 6;
  const int T = xcd_order(linear_block(), gridDim.x * gridDim.y * gridDim.z);
  const int bx = T % gridDim.x, by = (T / gridDim.x) % gridDim.y, bz = T / (gridDim.x * gridDim.y);
  const int x0 = 1 + bx * kQTX, y0 = 1 + by * kQTY;
  const int nzc = (p.nz + p.zchunk - 1) / p.zchunk;
  const int zc = bz % nzc, r = bz / nzc;
  const int lb = 1 + zc * p.zchunk;
  const int le = min(p.nz, lb + p.zchunk - 1);
  const long long plane = (long long)p.nx * p.ny;
  const double* __restrict__ Ur = U + r * p.u_stride;
  long long off[kQLoads];
  bool ok[kQLoads];
#pragma unroll
  for (int k = 0; k < kQLoads; ++k) {
    const int e = threadIdx.x + kQThreads * k;
    const int yy = e / kQX, xx = e - yy * kQX;
    const int gx = x0 - 1 + xx, gy = y0 - 1 + yy;  // interior indices, 1-based
    ok[k] = e < kQX * kQY && gx >= 1 && gx <= p.nx && gy >= 1 && gy <= p.ny;
    off[k] = ok[k] ? (gx - 1) + (long long)p.nx * (gy - 1) : 0;
  }
  double pa[kQLoads], pb[kQLoads];
  auto fetch = [&](double(&pre)[kQLoads], int q) {
    const bool qok = q >= 1 && q <= p.nz;
#pragma unroll
    for (int k = 0; k < kQLoads; ++k) pre[k] = (qok && ok[k]) ? Ur[off[k] + plane * (q - 1)] : 0.0;
  };
  auto stash = [&](const double(&pre)[kQLoads], int q) {
    double* w = win[(q + 3) % 3];
#pragma unroll
    for (int k = 0; k < kQLoads; ++k) {
      const int e = threadIdx.x + kQThreads * k;
      if (e < kQX * kQY) w[e] = pre[k];
    }
  };
  fetch(pa, lb - 1);
  stash(pa, lb - 1);
  fetch(pa, lb);
  stash(pa, lb);
  fetch(pa, lb + 1);
  fetch(pb, lb + 2);
  const int i = x0 + tx;
  double ss = 0.0, sf = 0.0;
  // F of the rows a thread owns, fetched two planes ahead like U; the weights are read from
  // LDS, so no wait in the stencil phase holds up the prefetched planes
  double fA[kQRows], fB[kQRows];
  auto fetchF = [&](double(&dst)[kQRows], int q) {
#pragma unroll
    for (int k = 0; k < kQRows; ++k) {
      const int j = y0 + ty * kQRows + k;
      dst[k] = (q <= le && i <= p.nx && j <= p.ny)
                   ? Fi[r * p.u_stride + (i - 1) + (long long)p.nx * ((j - 1) + (long long)p.ny * (q - 1))]
                   : 0.0;
    }
  };
  fetchF(fA, lb);
  fetchF(fB, lb + 1);
  auto compute = [&](int l, const double(&fl)[kQRows]) {
    const double* Pm = win[(l + 2) % 3];
    const double* P0 = win[l % 3];
    const double* Pp = win[(l + 1) % 3];
    double w[12];
#pragma unroll
    for (int q = 0; q < 12; ++q) w[q] = wt[((l - lb) % kQWPlanes) * 12 + q];
#pragma unroll
    for (int k = 0; k < kQRows; ++k) {
      const int yl = ty * kQRows + k, j = y0 + yl;
      if (i > p.nx || j > p.ny) continue;
      const int c = (yl + 1) * kQX + tx + 1;
      double au = 0.0;
      const double* planes[3] = {Pm, P0, Pp};
#pragma unroll
      for (int o = 0; o < 3; ++o) {
        const double* P = planes[o];
        const double* wo = w + 4 * o;
        au += wo[0] * (P[c - kQX - 1] + P[c - kQX + 1] + P[c + kQX - 1] + P[c + kQX + 1]) +
              wo[1] * (P[c - 1] + P[c + 1]) + wo[2] * (P[c - kQX] + P[c + kQX]) + wo[3] * P[c];
      }
      const long long idx = r * p.u_stride + (i - 1) + (long long)p.nx * ((j - 1) + (long long)p.ny * (l - 1));
      const double rr = fl[k] - au;
      if constexpr (STORE) R[idx] = (TR)rr;
      ss += rr * rr;
      sf += fl[k] * fl[k];
    }
  };
  for (int l = lb; l <= le; l += 2) {
    if ((l - lb) % kQWPlanes == 0) {  // every reader of the previous block passed a barrier
      const int n = 12 * min(kQWPlanes, le - l + 1);
      for (int q = threadIdx.x; q < n; q += kQThreads) wt[q] = p.W[(l - 1) * 12 + q];
    }
    stash(pa, l + 1);
    __syncthreads();
    if (l + 2 <= le) fetch(pa, l + 3);
    compute(l, fA);
    if (l + 2 <= le) fetchF(fA, l + 2);
    __syncthreads();
    if (l + 1 <= le) {
      stash(pb, l + 2);
      __syncthreads();
      if (l + 3 <= le) fetch(pb, l + 4);
      compute(l + 1, fB);
      if (l + 3 <= le) fetchF(fB, l + 3);
      __syncthreads();
    }
  }
  for (int off2 = 32; off2 > 0; off2 >>= 1) {
    ss += __shfl_xor(ss, off2, 64);
    sf += __shfl_xor(sf, off2, 64);
  }
  if ((threadIdx.x & 63) == 0) {
    part[threadIdx.x >> 6] = ss;
    partF[threadIdx.x >> 6] = sf;
  }
  __syncthreads();
  if (threadIdx.x == 0 && acc) {
    double t = 0.0, tf = 0.0;
    for (int q = 0; q < kQThreads / 64; ++q) {
      t += part[q];
      tf += partF[q];
    }
    atomicAdd(acc, t);
    if (accF) atomicAdd(accF, tf);
  }
}

// statistics block: [0] bits of min |pivot|, [1] bad pivots, then doubles:
// [2] ||F||^2, [3 + s] ||r_s||^2 after refinement step s (s = 0 is the initial solve)
constexpr int kStatsWords = 16;

__global__ void k_stats_reset(unsigned long long* s) {
  if (threadIdx.x == 0) {
    s[0] = 0x7FEFFFFFFFFFFFFFull;  // bits of DBL_MAX
    s[1] = 0ull;
  }
  if (threadIdx.x >= 2 && threadIdx.x < kStatsWords) s[threadIdx.x] = 0ull;  // +0.0
}

}  // namespace cs3d
