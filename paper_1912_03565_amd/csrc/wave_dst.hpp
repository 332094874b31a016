// wave_dst.hpp - DST-I of one grid line per wavefront (CDNA4, wave64).
//
// The 2-D sine transform of Section 3.6 is applied as 1-D DST-I sums along x
// and along y:  S_k = sum_{n=1}^{N} x_n sin(pi k n / M),  M = N + 1.
//
// FFT path (M a power of two, 64 <= M <= 1024).  With x_0 = x_M = 0 define, for
// n = 0..M-1,
//     u_n = x_n - x_{M-n},   z_n = x_n + x_{M-n},   w_n = u_n + i z_n e^{-i pi n/M}.
// Splitting the length-2M DFT of the odd extension of x into even and odd
// frequencies shows that the M-point DFT W of w carries the whole transform:
//     S_{2q} = -Im(W_q)/2,   S_{2q+1} = Re(W_q)/2,   q = 0..M/2-1.
// W is computed by a Stockham radix-4/8/16 FFT.  The line is spread over L lanes
// with R = M/L complex values per lane; element e lives in lane e mod L, slot
// e div L, both on input and on output, so butterflies run in registers and only
// the L-lane transposes between stages go through a per-wave LDS buffer of M
// elements (real and imaginary parts exchanged in turn for FP64, which keeps the
// buffer at M doubles).
//
// Dense path (any N <= 1024).  Each lane sums S_k for its modes k directly,
// using a table sin(pi r/M), r < 2M.
#pragma once
#include <hip/hip_runtime.h>

namespace cs3d {

template <typename T>
struct cx {
  T re, im;
};

template <typename T>
__device__ __forceinline__ cx<T> cadd(cx<T> a, cx<T> b) { return {a.re + b.re, a.im + b.im}; }
template <typename T>
__device__ __forceinline__ cx<T> csub(cx<T> a, cx<T> b) { return {a.re - b.re, a.im - b.im}; }
template <typename T>
__device__ __forceinline__ cx<T> cmul(cx<T> a, cx<T> b) {
  return {a.re * b.re - a.im * b.im, a.re * b.im + a.im * b.re};
}
// multiply by -i
template <typename T>
__device__ __forceinline__ cx<T> cmi(cx<T> a) { return {a.im, -a.re}; }

// Compiler-level ordering point for LDS traffic inside one wavefront.  LDS
// instructions of a wave execute in program order, so a wave-private buffer
// needs no hardware barrier, only that the compiler keeps the order.
__device__ __forceinline__ void wave_sync() {
  __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
  __builtin_amdgcn_wave_barrier();
  __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
}

// ---------------------------------------------------------------------------
// Small forward DFTs (sign -1) on registers, output in natural order.
// ---------------------------------------------------------------------------
template <typename T>
__device__ __forceinline__ void dft2(cx<T>* a) {
  cx<T> t = a[0];
  a[0] = cadd(t, a[1]);
  a[1] = csub(t, a[1]);
}

template <typename T>
__device__ __forceinline__ void dft4(cx<T>& a0, cx<T>& a1, cx<T>& a2, cx<T>& a3) {
  cx<T> t0 = cadd(a0, a2), t1 = csub(a0, a2);
  cx<T> t2 = cadd(a1, a3), t3 = cmi(csub(a1, a3));
  a0 = cadd(t0, t2);
  a2 = csub(t0, t2);
  a1 = cadd(t1, t3);
  a3 = csub(t1, t3);
}

template <typename T>
__device__ __forceinline__ void dft4(cx<T>* a) { dft4(a[0], a[1], a[2], a[3]); }

template <typename T>
__device__ __forceinline__ void dft8(cx<T>* a) {
  // even/odd split, two 4-point DFTs, combine with w8^k
  cx<T> e0 = a[0], e1 = a[2], e2 = a[4], e3 = a[6];
  cx<T> o0 = a[1], o1 = a[3], o2 = a[5], o3 = a[7];
  dft4(e0, e1, e2, e3);
  dft4(o0, o1, o2, o3);
  const T h = (T)0.70710678118654752440084436210485;
  // w8^1 = (h, -h), w8^2 = -i, w8^3 = (-h, -h)
  cx<T> p1 = {h * (o1.re + o1.im), h * (o1.im - o1.re)};
  cx<T> p2 = cmi(o2);
  cx<T> p3 = {h * (o3.im - o3.re), -h * (o3.re + o3.im)};
  a[0] = cadd(e0, o0);
  a[4] = csub(e0, o0);
  a[1] = cadd(e1, p1);
  a[5] = csub(e1, p1);
  a[2] = cadd(e2, p2);
  a[6] = csub(e2, p2);
  a[3] = cadd(e3, p3);
  a[7] = csub(e3, p3);
}

template <typename T>
__device__ __forceinline__ void dft16(cx<T>* a) {
  // 16 = 4 x 4: n = 4 n1 + n2, k = k1 + 4 k2
  cx<T> b[4][4];
#pragma unroll
  for (int n2 = 0; n2 < 4; ++n2) {
    b[n2][0] = a[n2];
    b[n2][1] = a[4 + n2];
    b[n2][2] = a[8 + n2];
    b[n2][3] = a[12 + n2];
    dft4(b[n2][0], b[n2][1], b[n2][2], b[n2][3]);  // -> index k1
  }
  // twiddles w16^{n2 k1}
  const T c1 = (T)0.92387953251128675612818318939679;  // cos(pi/8)
  const T s1 = (T)0.38268343236508977172845998403040;  // sin(pi/8)
  const T h = (T)0.70710678118654752440084436210485;
  // n2 = 1: k1 = 1,2,3 -> w^1, w^2, w^3
  b[1][1] = cmul(b[1][1], cx<T>{c1, -s1});
  b[1][2] = cmul(b[1][2], cx<T>{h, -h});
  b[1][3] = cmul(b[1][3], cx<T>{s1, -c1});
  // n2 = 2: w^2, w^4, w^6
  b[2][1] = cmul(b[2][1], cx<T>{h, -h});
  b[2][2] = cmi(b[2][2]);
  b[2][3] = cmul(b[2][3], cx<T>{-h, -h});
  // n2 = 3: w^3, w^6, w^9
  b[3][1] = cmul(b[3][1], cx<T>{s1, -c1});
  b[3][2] = cmul(b[3][2], cx<T>{-h, -h});
  b[3][3] = cmul(b[3][3], cx<T>{-c1, s1});
#pragma unroll
  for (int k1 = 0; k1 < 4; ++k1) {
    cx<T> x0 = b[0][k1], x1 = b[1][k1], x2 = b[2][k1], x3 = b[3][k1];
    dft4(x0, x1, x2, x3);
    a[k1] = x0;
    a[k1 + 4] = x1;
    a[k1 + 8] = x2;
    a[k1 + 12] = x3;
  }
}

template <typename T, int RS>
__device__ __forceinline__ void dft(cx<T>* a) {
  if constexpr (RS == 2) dft2(a);
  else if constexpr (RS == 4) dft4(a);
  else if constexpr (RS == 8) dft8(a);
  else dft16(a);
}

// ---------------------------------------------------------------------------
// FFT geometry per line length M.
// ---------------------------------------------------------------------------
template <int M>
struct FftGeom {
  static_assert(M == 64 || M == 128 || M == 256 || M == 512 || M == 1024, "unsupported M");
  static constexpr int R = (M / 64 < 4) ? 4 : M / 64;  // complex values per lane
  static constexpr int L = M / R;                       // lanes per line
  static constexpr int NS = R;                          // output slots per lane
};

// twiddle table: tw[k] = exp(-i pi k / M), k < 2M, stored as (re, im) doubles
template <typename T>
__device__ __forceinline__ cx<T> twid(const double2* __restrict__ tw, int k) {
  double2 t = tw[k];
  return {(T)t.x, (T)t.y};
}

// One Stockham stage of radix RS and span NSP on the register layout.
template <typename T, int M, int RS, int NSP>
__device__ __forceinline__ void fft_stage(cx<T> (&v)[FftGeom<M>::R], int tl,
                                          const double2* __restrict__ tw) {
  constexpr int R = FftGeom<M>::R, L = FftGeom<M>::L, NB = R / RS;
#pragma unroll
  for (int b = 0; b < NB; ++b) {
    cx<T> u[RS];
#pragma unroll
    for (int r = 0; r < RS; ++r) u[r] = v[b + r * NB];
    if constexpr (NSP > 1) {
      const int jm = (tl + L * b) & (NSP - 1);
      constexpr int step = 2 * (M / (NSP * RS));
#pragma unroll
      for (int r = 1; r < RS; ++r) u[r] = cmul(u[r], twid<T>(tw, step * jm * r));
    }
    dft<T, RS>(u);
#pragma unroll
    for (int r = 0; r < RS; ++r) v[b + r * NB] = u[r];
  }
}

// Transpose between stage (RS, NSP) and a following stage of radix RS2 through LDS.
template <typename T, int M, int RS, int NSP, int RS2>
__device__ __forceinline__ void fft_exchange(cx<T> (&v)[FftGeom<M>::R], T* buf, int tl) {
  constexpr int R = FftGeom<M>::R, L = FftGeom<M>::L, NB = R / RS, NB2 = R / RS2;
  int opos[R], ipos[R];
#pragma unroll
  for (int b = 0; b < NB; ++b)
#pragma unroll
    for (int r = 0; r < RS; ++r) {
      const int j = tl + L * b;
      opos[b + r * NB] = (j / NSP) * NSP * RS + (j & (NSP - 1)) + r * NSP;
    }
#pragma unroll
  for (int b = 0; b < NB2; ++b)
#pragma unroll
    for (int r = 0; r < RS2; ++r) ipos[b + r * NB2] = tl + L * b + r * (M / RS2);
  if constexpr (sizeof(T) == 4) {
    cx<T>* cb = reinterpret_cast<cx<T>*>(buf);
#pragma unroll
    for (int s = 0; s < R; ++s) cb[opos[s]] = v[s];
    wave_sync();
#pragma unroll
    for (int s = 0; s < R; ++s) v[s] = cb[ipos[s]];
    wave_sync();
  } else {
#pragma unroll
    for (int s = 0; s < R; ++s) buf[opos[s]] = v[s].re;
    wave_sync();
#pragma unroll
    for (int s = 0; s < R; ++s) v[s].re = buf[ipos[s]];
    wave_sync();
#pragma unroll
    for (int s = 0; s < R; ++s) buf[opos[s]] = v[s].im;
    wave_sync();
#pragma unroll
    for (int s = 0; s < R; ++s) v[s].im = buf[ipos[s]];
    wave_sync();
  }
}

template <typename T, int M>
__device__ __forceinline__ void fft_run(cx<T> (&v)[FftGeom<M>::R], T* buf, int tl,
                                        const double2* __restrict__ tw) {
  if constexpr (M == 64) {
    fft_stage<T, M, 4, 1>(v, tl, tw);
    fft_exchange<T, M, 4, 1, 4>(v, buf, tl);
    fft_stage<T, M, 4, 4>(v, tl, tw);
    fft_exchange<T, M, 4, 4, 4>(v, buf, tl);
    fft_stage<T, M, 4, 16>(v, tl, tw);
  } else if constexpr (M == 128) {
    fft_stage<T, M, 4, 1>(v, tl, tw);
    fft_exchange<T, M, 4, 1, 4>(v, buf, tl);
    fft_stage<T, M, 4, 4>(v, tl, tw);
    fft_exchange<T, M, 4, 4, 4>(v, buf, tl);
    fft_stage<T, M, 4, 16>(v, tl, tw);
    fft_exchange<T, M, 4, 16, 2>(v, buf, tl);
    fft_stage<T, M, 2, 64>(v, tl, tw);
  } else if constexpr (M == 256) {
    fft_stage<T, M, 4, 1>(v, tl, tw);
    fft_exchange<T, M, 4, 1, 4>(v, buf, tl);
    fft_stage<T, M, 4, 4>(v, tl, tw);
    fft_exchange<T, M, 4, 4, 4>(v, buf, tl);
    fft_stage<T, M, 4, 16>(v, tl, tw);
    fft_exchange<T, M, 4, 16, 4>(v, buf, tl);
    fft_stage<T, M, 4, 64>(v, tl, tw);
  } else if constexpr (M == 512) {
    fft_stage<T, M, 8, 1>(v, tl, tw);
    fft_exchange<T, M, 8, 1, 8>(v, buf, tl);
    fft_stage<T, M, 8, 8>(v, tl, tw);
    fft_exchange<T, M, 8, 8, 8>(v, buf, tl);
    fft_stage<T, M, 8, 64>(v, tl, tw);
  } else {
    fft_stage<T, M, 16, 1>(v, tl, tw);
    fft_exchange<T, M, 16, 1, 16>(v, buf, tl);
    fft_stage<T, M, 16, 16>(v, tl, tw);
    fft_exchange<T, M, 16, 16, 4>(v, buf, tl);
    fft_stage<T, M, 4, 256>(v, tl, tw);
  }
}

// DST-I of the line held in buf[1..M-1] (buf[0] is ignored).  On return, lane
// lane < L holds out[s] = S_m for m = fft_mode<M>(lane, s); buf is clobbered.
template <typename T, int M>
__device__ __forceinline__ void dst_fft(T* buf, T (&out)[FftGeom<M>::R], int lane,
                                        const double2* __restrict__ tw) {
  constexpr int R = FftGeom<M>::R, L = FftGeom<M>::L;
  cx<T> v[R];
  if (lane < L) {
#pragma unroll
    for (int s = 0; s < R; ++s) {
      const int n = lane + L * s;
      if (n == 0) {
        v[s] = {(T)0, (T)0};
      } else {
        const T a = buf[n], b = buf[M - n];
        const T u = a - b, z = a + b;
        const cx<T> t = twid<T>(tw, n);  // (cos, -sin)(pi n/M)
        v[s] = {u - z * t.im, z * t.re};
      }
    }
  }
  wave_sync();
  if (lane < L) {
    fft_run<T, M>(v, buf, lane, tw);
#pragma unroll
    for (int s = 0; s < R / 2; ++s) {
      out[2 * s] = (T)-0.5 * v[s].im;
      out[2 * s + 1] = (T)0.5 * v[s].re;
    }
  }
}

template <int M>
__device__ __forceinline__ int fft_mode(int lane, int s) {
  constexpr int L = FftGeom<M>::L;
  if (lane >= L) return -1;
  const int m = 2 * (lane + L * (s >> 1)) + (s & 1);
  return (m >= 1 && m <= M - 1) ? m : -1;
}

// ---------------------------------------------------------------------------
// Dense path: any N <= 1024.  out[s] = S_k, k = 1 + lane + 64 s.
// sintab[r] = sin(pi r/M), r < 2M.
// ---------------------------------------------------------------------------
constexpr int kDenseSlots = 16;

template <typename T>
__device__ __forceinline__ void dst_dense(const T* buf, int N, T (&out)[kDenseSlots], int lane,
                                          const double* __restrict__ sintab) {
  const int twoM = 2 * (N + 1);
#pragma unroll
  for (int s = 0; s < kDenseSlots; ++s) {
    const int k = 1 + lane + 64 * s;
    T acc = (T)0;
    if (k <= N) {
      int idx = 0;
      for (int n = 1; n <= N; ++n) {
        idx += k;
        if (idx >= twoM) idx -= twoM;
        acc += buf[n] * (T)sintab[idx];
      }
    }
    out[s] = acc;
  }
}

__device__ __forceinline__ int dense_mode(int lane, int s, int N) {
  const int k = 1 + lane + 64 * s;
  return k <= N ? k : -1;
}

}  // namespace cs3d
