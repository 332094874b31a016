// wave_dst.hpp - DST-I of one grid line per group of wavefronts (CDNA4, wave64).
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
// W is computed by a Stockham FFT of radix 2..16.  A line is spread over L lanes
// (one or two wavefronts) with R = M/L complex values per lane; element e lives in
// lane e mod L, slot e div L, on input and on output, so butterflies run in
// registers and only the transposes between stages go through LDS.
//
// LDS layout.  The LDS of gfx950 serves 64 banks of 4 bytes; an 8-byte access of a
// wavefront is conflict-free when, within each half-wave, the 8-byte slot indices are
// distinct modulo 32 (measured: contiguous runs and odd strides are free, a stride of
// 2^k slots costs 2^k-fold).  The line input is stored unpadded (contiguous and
// mirrored reads are then free); every Stockham exchange uses its own index map of the
// buffer (pad one slot per 2^a, or an XOR of the low five bits with higher ones),
// chosen per transform size so that the stage's writes and the next stage's reads are
// conflict-free or nearly so.  FP64 exchanges move the real and then the imaginary
// parts through the buffer, FP32 exchanges move complex pairs in one go.
//
// Twiddles live in LDS, filled once per workgroup: tab[n] = exp(-i pi n/M), n < M, for
// the pre-processing, and after it one table per Stockham stage (radix RS, span NSP)
// laid out [r - 1][jm] = exp(-2 pi i jm r/(NSP RS)), so that the lanes of a wave read
// consecutive or identical entries (conflict-free) instead of entries a power of two
// apart.
//
// Dense path (any N <= 1024).  Each lane sums S_k for its modes k directly, using a
// table sin(pi r/M), r < 2M, in global memory.
//
// DCT-I (Neumann sides).  With unknowns on the side nodes too, a line holds
// x_0..x_M (N = M + 1 values) and the even reflection about its end nodes is
// diagonalised by C_k = sum_{n=0}^{M} e_n x_n cos(pi k n/M), k = 0..M, with
// e_0 = e_M = 1/2 and e_n = 1 otherwise; C applied twice is M/2 times the identity.
// For n = 0..M-1 let a_n = x_n + x_{M-n}, b_n = x_n - x_{M-n} (a_0 = x_0 + x_M) and
// w_n = a_n + i b_n e^{-i pi n/M}.  The even frequencies of the length-2M DFT of the
// even extension give C_{2q} = Re(W_q)/2, the odd ones C_{2q+1} = Im(W_q)/2 (the
// imaginary part of the odd sum cancels between n and M - n), with the same M-point
// FFT as the sine transform.  Mode M comes from W_{M/2}, an extra slot of lane 0.
// Both kinds keep a line at buffer positions 1..N: for the sine transform position n
// holds x_n, for the cosine transform x_{n-1}; outputs go to the same positions.
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

// A complex table in LDS at p, which must sit at a multiple of 2 sizeof(T) bytes, with that
// alignment made known to the compiler: an FP64 entry is then read with one 16-byte access.
// (Without it the compiler reads the two halves with one paired 8-byte instruction, whose
// lanes 16 bytes apart cost the LDS four times the cycles of a 16-byte read.)
template <typename T>
__device__ __forceinline__ cx<T>* lds_table(T* p) {
  return reinterpret_cast<cx<T>*>(__builtin_assume_aligned(p, 2 * sizeof(T)));
}

// index maps of a line buffer: identity, one pad slot per 2^a (a = 3, 4, 5), XOR of the
// low five bits with bits 4..8 (a bijection inside each aligned block of 32)
constexpr int kLayId = 0, kLayPad3 = 3, kLayPad4 = 4, kLayPad5 = 5, kLayXor4 = 14;

template <int LAY>
__host__ __device__ constexpr int lay(int p) {
  if constexpr (LAY == kLayId) {
    return p;
  } else if constexpr (LAY == kLayXor4) {
    return p ^ ((p >> 4) & 31);
  } else {
    return p + (p >> LAY);
  }
}

// slots a map needs for M elements
template <int LAY>
__host__ __device__ constexpr int lay_slots(int M) {
  return (LAY == kLayId || LAY == kLayXor4) ? M : M + (M >> LAY);
}

// Compiler-level ordering point for LDS traffic inside one wavefront.  LDS
// instructions of a wave execute in program order, so a wave-private buffer
// needs no hardware barrier, only that the compiler keeps the order.
__device__ __forceinline__ void wave_sync() {
  __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
  __builtin_amdgcn_wave_barrier();
  __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
}

// Ordering point for a line spread over WPL wavefronts of the same workgroup.
// With WPL > 1 the workgroup must consist of lines that all run the transform.
template <int WPL>
__device__ __forceinline__ void line_sync() {
  if constexpr (WPL == 1) {
    wave_sync();
  } else {
    __syncthreads();
  }
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
  // 16 = 4 x 4, in place: n = n2 + 4 n1, k = k1 + 4 k2.  Column DFTs over n1 leave
  // (n2, k1) in a[n2 + 4 k1]; after the twiddles w16^{n2 k1}, row DFTs over n2 leave
  // X[k1 + 4 k2] in a[4 k1 + k2]; a final register renaming restores natural order.
#pragma unroll
  for (int n2 = 0; n2 < 4; ++n2) dft4(a[n2], a[n2 + 4], a[n2 + 8], a[n2 + 12]);
  const T c1 = (T)0.92387953251128675612818318939679;  // cos(pi/8)
  const T s1 = (T)0.38268343236508977172845998403040;  // sin(pi/8)
  const T h = (T)0.70710678118654752440084436210485;
  a[1 + 4] = cmul(a[1 + 4], cx<T>{c1, -s1});
  a[1 + 8] = cmul(a[1 + 8], cx<T>{h, -h});
  a[1 + 12] = cmul(a[1 + 12], cx<T>{s1, -c1});
  a[2 + 4] = cmul(a[2 + 4], cx<T>{h, -h});
  a[2 + 8] = cmi(a[2 + 8]);
  a[2 + 12] = cmul(a[2 + 12], cx<T>{-h, -h});
  a[3 + 4] = cmul(a[3 + 4], cx<T>{s1, -c1});
  a[3 + 8] = cmul(a[3 + 8], cx<T>{-h, -h});
  a[3 + 12] = cmul(a[3 + 12], cx<T>{-c1, s1});
#pragma unroll
  for (int k1 = 0; k1 < 4; ++k1) dft4(a[4 * k1], a[4 * k1 + 1], a[4 * k1 + 2], a[4 * k1 + 3]);
  // a[4 k1 + k2] -> a[k1 + 4 k2]: transpose of the 4 x 4 index grid
  cx<T> t;
  t = a[1]; a[1] = a[4]; a[4] = t;
  t = a[2]; a[2] = a[8]; a[8] = t;
  t = a[3]; a[3] = a[12]; a[12] = t;
  t = a[6]; a[6] = a[9]; a[9] = t;
  t = a[7]; a[7] = a[13]; a[13] = t;
  t = a[11]; a[11] = a[14]; a[14] = t;
}

template <typename T, int RS>
__device__ __forceinline__ void dft(cx<T>* a) {
  if constexpr (RS == 2) dft2(a);
  else if constexpr (RS == 4) dft4(a);
  else if constexpr (RS == 8) dft8(a);
  else dft16(a);
}

// ---------------------------------------------------------------------------
// FFT geometry: WPL wavefronts per line (1, or 2 for M >= 512).
// ---------------------------------------------------------------------------
template <int M, int WPL>
struct FftGeom {
  static_assert(M == 64 || M == 128 || M == 256 || M == 512 || M == 1024, "unsupported M");
  static_assert(WPL == 1 || (WPL == 2 && M >= 512), "two waves per line need M >= 512");
  static constexpr int L = (M >= 256) ? 64 * WPL : M / 4;   // lanes per line
  static constexpr int R = M / L;                          // complex values per lane
  static constexpr int NS = R;                             // output slots per lane
};

// register arrays of one line: complex values and real output slots per lane
template <typename T, int M, int WPL>
using LineRegs = cx<T>[FftGeom<M, WPL>::R];
template <typename T, int M, int WPL>
using LineOut = T[FftGeom<M, WPL>::R];

// index map of exchange k of the stage plan of (M, WPL) (see fft_run)
template <int M, int WPL, int K>
__host__ __device__ constexpr int exch_lay() {
  if constexpr (M == 64) return K == 0 ? kLayPad4 : kLayPad3;
  else if constexpr (M == 128 || M == 256) return K == 0 ? kLayPad5 : (K == 1 ? kLayXor4 : kLayId);
  else if constexpr (M == 512 && WPL == 1) return K == 0 ? kLayPad5 : kLayPad3;
  else if constexpr (M == 512) return K == 0 ? kLayPad5 : (K == 1 ? kLayXor4 : kLayId);
  else if constexpr (WPL == 1) return K == 0 ? kLayPad5 : kLayXor4;
  else return K == 0 ? kLayPad5 : (K == 1 ? kLayPad3 : kLayId);
}

// Paired exchanges (FP64, M = 1024, two waves per line): the real and imaginary parts of a
// value move through the buffer together as one 16-byte entry, so an exchange takes one
// write, one read and two barriers per value instead of two, two and four.  The entry maps
// of exchanges 0, 1, 2 (one pad entry per 16; an XOR of the low four bits with bits 3..6;
// identity) make every quarter-wave's 16-byte accesses fall on distinct 16-byte bank groups.
template <typename T, int M, int WPL>
__host__ __device__ constexpr bool pair_exchange_ok() {
  return sizeof(T) == 8 && M == 1024 && WPL == 2;
}

template <int K>
__host__ __device__ constexpr int pair_lay(int p) {
  if constexpr (K == 0) {
    return p + (p >> 4);
  } else if constexpr (K == 1) {
    return p ^ ((p >> 3) & 15);
  } else {
    return p;
  }
}

constexpr int kPairEntries = 1024 + 1024 / 16;  // entries the maps above need at M = 1024

template <int M, int WPL>
__host__ __device__ constexpr int fft_slots() {
  constexpr int a = lay_slots<exch_lay<M, WPL, 0>()>(M), b = lay_slots<exch_lay<M, WPL, 1>()>(M),
                c = lay_slots<exch_lay<M, WPL, 2>()>(M), d = lay_slots<exch_lay<M, WPL, 3>()>(M);
  constexpr int ab = a > b ? a : b, cd = c > d ? c : d;
  return ab > cd ? ab : cd;
}

// LDS elements of T in one line buffer
template <typename T, int M, int WPL, bool PAIR = false>
__host__ __device__ constexpr int fft_buf_elems() {
  static_assert(!PAIR || pair_exchange_ok<T, M, WPL>(), "paired exchanges: FP64, M = 1024, two waves");
  if constexpr (PAIR) return 2 * kPairEntries;
  return sizeof(T) == 8 ? fft_slots<M, WPL>() : 2 * fft_slots<M, WPL>();
}

// LDS complex entries of the twiddle tables of one FFT size
template <int M>
__host__ __device__ constexpr int tw_entries() {
  return 2 * M;
}

// Fill the stage table of stage (RS, NSP) at stab + OFF from the global table
// tw[k] = exp(-i pi k/M), k < 2M (every thread of the block takes part).
template <typename T, int M, int RS, int NSP, int OFF>
__device__ __forceinline__ void fill_stage(cx<T>* stab, const double2* __restrict__ tw) {
  constexpr int step = 2 * (M / (NSP * RS));
  for (int e = threadIdx.x; e < (RS - 1) * NSP; e += blockDim.x) {
    const int r = 1 + e / NSP, jm = e % NSP;
    const double2 t = tw[step * jm * r];
    stab[OFF + e] = {(T)t.x, (T)t.y};
  }
}

template <typename T, int M, int WPL>
__device__ __forceinline__ void fill_stage_tables(cx<T>* stab, const double2* __restrict__ tw);

// Fill tab[0..M) and the stage tables behind it (a barrier must follow before use).
template <typename T, int M, int WPL>
__device__ __forceinline__ void load_twiddles(cx<T>* tab, const double2* __restrict__ tw) {
  for (int k = threadIdx.x; k < M; k += blockDim.x) {
    const double2 t = tw[k];
    tab[k] = {(T)t.x, (T)t.y};
  }
  fill_stage_tables<T, M, WPL>(tab + M, tw);
}

// One Stockham stage of radix RS and span NSP on the register layout; its twiddles
// are stab[OFF + (r - 1) NSP + jm].
template <typename T, int M, int WPL, int RS, int NSP, int OFF>
__device__ __forceinline__ void fft_stage(LineRegs<T, M, WPL>& v, int tl, const cx<T>* stab) {
  constexpr int R = FftGeom<M, WPL>::R, L = FftGeom<M, WPL>::L, NB = R / RS;
#pragma unroll
  for (int b = 0; b < NB; ++b) {
    cx<T> u[RS];
#pragma unroll
    for (int r = 0; r < RS; ++r) u[r] = v[b + r * NB];
    if constexpr (NSP > 1) {
      const int jm = (tl + L * b) & (NSP - 1);
#pragma unroll
      for (int r = 1; r < RS; ++r) u[r] = cmul(u[r], stab[OFF + (r - 1) * NSP + jm]);
    }
    dft<T, RS>(u);
#pragma unroll
    for (int r = 0; r < RS; ++r) v[b + r * NB] = u[r];
  }
}

// LDS positions of the transpose between stage (RS, NSP) and a following stage of
// radix RS2 (recomputed where used, so they do not occupy registers)
template <int M, int WPL, int RS, int NSP, int LAY>
__device__ __forceinline__ int fft_opos(int tl, int s) {
  constexpr int L = FftGeom<M, WPL>::L, NB = FftGeom<M, WPL>::R / RS;
  const int b = s % NB, r = s / NB;
  const int j = tl + L * b;
  return lay<LAY>((j / NSP) * NSP * RS + (j & (NSP - 1)) + r * NSP);
}

template <int M, int WPL, int RS2, int LAY>
__device__ __forceinline__ int fft_ipos(int tl, int s) {
  constexpr int L = FftGeom<M, WPL>::L, NB2 = FftGeom<M, WPL>::R / RS2;
  const int b = s % NB2, r = s / NB2;
  return lay<LAY>(tl + L * b + r * (M / RS2));
}

// exchange K of the plan: after stage (RS, NSP), before a stage of radix RS2
template <typename T, int M, int WPL, int RS, int NSP, int RS2, int K, bool PAIR = false>
__device__ __forceinline__ void fft_exchange(LineRegs<T, M, WPL>& v, T* buf, int tl) {
  constexpr int R = FftGeom<M, WPL>::R;
  constexpr int LAY = exch_lay<M, WPL, K>();
  if constexpr (PAIR) {
    static_assert(pair_exchange_ok<T, M, WPL>(), "paired exchanges: FP64, M = 1024, two waves");
    cx<T>* cb = lds_table(buf);
#pragma unroll
    for (int s = 0; s < R; ++s) cb[pair_lay<K>(fft_opos<M, WPL, RS, NSP, kLayId>(tl, s))] = v[s];
    line_sync<WPL>();
#pragma unroll
    for (int s = 0; s < R; ++s) v[s] = cb[pair_lay<K>(fft_ipos<M, WPL, RS2, kLayId>(tl, s))];
    line_sync<WPL>();
  } else if constexpr (sizeof(T) == 4) {
    cx<T>* cb = reinterpret_cast<cx<T>*>(buf);
#pragma unroll
    for (int s = 0; s < R; ++s) cb[fft_opos<M, WPL, RS, NSP, LAY>(tl, s)] = v[s];
    line_sync<WPL>();
#pragma unroll
    for (int s = 0; s < R; ++s) v[s] = cb[fft_ipos<M, WPL, RS2, LAY>(tl, s)];
    line_sync<WPL>();
  } else {
#pragma unroll
    for (int s = 0; s < R; ++s) buf[fft_opos<M, WPL, RS, NSP, LAY>(tl, s)] = v[s].re;
    line_sync<WPL>();
#pragma unroll
    for (int s = 0; s < R; ++s) v[s].re = buf[fft_ipos<M, WPL, RS2, LAY>(tl, s)];
    line_sync<WPL>();
#pragma unroll
    for (int s = 0; s < R; ++s) buf[fft_opos<M, WPL, RS, NSP, LAY>(tl, s)] = v[s].im;
    line_sync<WPL>();
#pragma unroll
    for (int s = 0; s < R; ++s) v[s].im = buf[fft_ipos<M, WPL, RS2, LAY>(tl, s)];
    line_sync<WPL>();
  }
}

// Stage plans: (radix, span, offset of the stage's twiddle table).  Offsets
// accumulate (RS - 1) NSP entries per stage; every plan uses fewer than M entries.
template <typename T, int M, int WPL>
__device__ __forceinline__ void fill_stage_tables(cx<T>* st, const double2* __restrict__ tw) {
  constexpr int R = FftGeom<M, WPL>::R;
  if constexpr (R == 4 && M == 64) {
    fill_stage<T, M, 4, 4, 0>(st, tw);
    fill_stage<T, M, 4, 16, 12>(st, tw);
  } else if constexpr (R == 4 && M == 128) {
    fill_stage<T, M, 4, 4, 0>(st, tw);
    fill_stage<T, M, 4, 16, 12>(st, tw);
    fill_stage<T, M, 2, 64, 60>(st, tw);
  } else if constexpr (R == 4 && M == 256) {
    fill_stage<T, M, 4, 4, 0>(st, tw);
    fill_stage<T, M, 4, 16, 12>(st, tw);
    fill_stage<T, M, 4, 64, 60>(st, tw);
  } else if constexpr (R == 4 && M == 512) {
    fill_stage<T, M, 4, 4, 0>(st, tw);
    fill_stage<T, M, 4, 16, 12>(st, tw);
    fill_stage<T, M, 4, 64, 60>(st, tw);
    fill_stage<T, M, 2, 256, 252>(st, tw);
  } else if constexpr (R == 8 && M == 512) {
    fill_stage<T, M, 8, 8, 0>(st, tw);
    fill_stage<T, M, 8, 64, 56>(st, tw);
  } else if constexpr (R == 8 && M == 1024) {
    fill_stage<T, M, 8, 8, 0>(st, tw);
    fill_stage<T, M, 8, 64, 56>(st, tw);
    fill_stage<T, M, 2, 512, 504>(st, tw);
  } else {
    static_assert(R == 16 && M == 1024, "no stage plan");
    fill_stage<T, M, 16, 16, 0>(st, tw);
    fill_stage<T, M, 4, 256, 240>(st, tw);
  }
}

template <typename T, int M, int WPL, bool PAIR = false>
__device__ __forceinline__ void fft_run(LineRegs<T, M, WPL>& v, T* buf, int tl, const cx<T>* st) {
  constexpr int R = FftGeom<M, WPL>::R;
  if constexpr (R == 4 && M == 64) {
    fft_stage<T, M, WPL, 4, 1, 0>(v, tl, st);
    fft_exchange<T, M, WPL, 4, 1, 4, 0>(v, buf, tl);
    fft_stage<T, M, WPL, 4, 4, 0>(v, tl, st);
    fft_exchange<T, M, WPL, 4, 4, 4, 1>(v, buf, tl);
    fft_stage<T, M, WPL, 4, 16, 12>(v, tl, st);
  } else if constexpr (R == 4 && M == 128) {
    fft_stage<T, M, WPL, 4, 1, 0>(v, tl, st);
    fft_exchange<T, M, WPL, 4, 1, 4, 0>(v, buf, tl);
    fft_stage<T, M, WPL, 4, 4, 0>(v, tl, st);
    fft_exchange<T, M, WPL, 4, 4, 4, 1>(v, buf, tl);
    fft_stage<T, M, WPL, 4, 16, 12>(v, tl, st);
    fft_exchange<T, M, WPL, 4, 16, 2, 2>(v, buf, tl);
    fft_stage<T, M, WPL, 2, 64, 60>(v, tl, st);
  } else if constexpr (R == 4 && M == 256) {
    fft_stage<T, M, WPL, 4, 1, 0>(v, tl, st);
    fft_exchange<T, M, WPL, 4, 1, 4, 0>(v, buf, tl);
    fft_stage<T, M, WPL, 4, 4, 0>(v, tl, st);
    fft_exchange<T, M, WPL, 4, 4, 4, 1>(v, buf, tl);
    fft_stage<T, M, WPL, 4, 16, 12>(v, tl, st);
    fft_exchange<T, M, WPL, 4, 16, 4, 2>(v, buf, tl);
    fft_stage<T, M, WPL, 4, 64, 60>(v, tl, st);
  } else if constexpr (R == 4 && M == 512) {
    fft_stage<T, M, WPL, 4, 1, 0>(v, tl, st);
    fft_exchange<T, M, WPL, 4, 1, 4, 0>(v, buf, tl);
    fft_stage<T, M, WPL, 4, 4, 0>(v, tl, st);
    fft_exchange<T, M, WPL, 4, 4, 4, 1>(v, buf, tl);
    fft_stage<T, M, WPL, 4, 16, 12>(v, tl, st);
    fft_exchange<T, M, WPL, 4, 16, 4, 2>(v, buf, tl);
    fft_stage<T, M, WPL, 4, 64, 60>(v, tl, st);
    fft_exchange<T, M, WPL, 4, 64, 2, 3>(v, buf, tl);
    fft_stage<T, M, WPL, 2, 256, 252>(v, tl, st);
  } else if constexpr (R == 8 && M == 512) {
    fft_stage<T, M, WPL, 8, 1, 0>(v, tl, st);
    fft_exchange<T, M, WPL, 8, 1, 8, 0>(v, buf, tl);
    fft_stage<T, M, WPL, 8, 8, 0>(v, tl, st);
    fft_exchange<T, M, WPL, 8, 8, 8, 1>(v, buf, tl);
    fft_stage<T, M, WPL, 8, 64, 56>(v, tl, st);
  } else if constexpr (R == 8 && M == 1024) {
    fft_stage<T, M, WPL, 8, 1, 0>(v, tl, st);
    fft_exchange<T, M, WPL, 8, 1, 8, 0, PAIR>(v, buf, tl);
    fft_stage<T, M, WPL, 8, 8, 0>(v, tl, st);
    fft_exchange<T, M, WPL, 8, 8, 8, 1, PAIR>(v, buf, tl);
    fft_stage<T, M, WPL, 8, 64, 56>(v, tl, st);
    fft_exchange<T, M, WPL, 8, 64, 2, 2, PAIR>(v, buf, tl);
    fft_stage<T, M, WPL, 2, 512, 504>(v, tl, st);
  } else {
    static_assert(R == 16 && M == 1024, "no stage plan");
    fft_stage<T, M, WPL, 16, 1, 0>(v, tl, st);
    fft_exchange<T, M, WPL, 16, 1, 16, 0>(v, buf, tl);
    fft_stage<T, M, WPL, 16, 16, 0>(v, tl, st);
    fft_exchange<T, M, WPL, 16, 16, 4, 1>(v, buf, tl);
    fft_stage<T, M, WPL, 4, 256, 240>(v, tl, st);
  }
}

// DST-I of a line.  The input x_n (1 <= n < M) is read from src[n] (src may alias
// nothing the exchanges write before the first sync) or, when src is null, from
// buf[n] (unpadded).  BLOCK_SYNC makes the sync after the input has been read a
// workgroup barrier, for callers whose line buffers overlay a shared input tile.
// tl is the lane index within the line (0 <= tl < 64 WPL).  On return, lane tl < L
// holds out[s] = S_m for m = fft_mode<M, WPL>(tl, s); buf is clobbered.  All lanes
// of the line's waves must call it (lanes tl >= L only take part in the syncs).
// transform kinds: DST-I (Dirichlet sides) and DCT-I (Neumann sides)
constexpr int kDst = 0, kDct = 1;

// output slots per lane of the FFT path: R, and for the cosine transform one more (mode M)
template <int M, int WPL, int KIND>
__host__ __device__ constexpr int fft_out_slots() {
  return FftGeom<M, WPL>::R + (KIND == kDct ? 1 : 0);
}

template <typename T, int M, int WPL, int KIND, bool BLOCK_SYNC = false, bool PAIR = false>
__device__ __forceinline__ void dst_fft(T* buf, T (&out)[fft_out_slots<M, WPL, KIND>()], int tl,
                                        const cx<T>* tab, const T* src = nullptr) {
  constexpr int R = FftGeom<M, WPL>::R, L = FftGeom<M, WPL>::L;
  LineRegs<T, M, WPL> v;
  if (tl < L) {
#pragma unroll
    for (int s = 0; s < R; ++s) {
      const int n = tl + L * s;
      if constexpr (KIND == kDst) {
        if (n == 0) {
          v[s] = {(T)0, (T)0};
        } else {
          const T a = src ? src[n] : buf[n];
          const T b = src ? src[M - n] : buf[M - n];
          const T u = a - b, z = a + b;
          const cx<T> t = tab[n];  // (cos, -sin)(pi n/M)
          v[s] = {u - z * t.im, z * t.re};
        }
      } else {
        // x_n at position n + 1
        const T a = src ? src[1 + n] : buf[1 + n];
        const T b = src ? src[1 + M - n] : buf[1 + M - n];
        const T z = a + b, u = a - b;
        const cx<T> t = tab[n];
        v[s] = {z - u * t.im, u * t.re};
      }
    }
  }
  if constexpr (BLOCK_SYNC) {
    __syncthreads();
  } else {
    line_sync<WPL>();
  }
  if (tl < L) {
    fft_run<T, M, WPL, PAIR>(v, buf, tl, tab + M);
#pragma unroll
    for (int s = 0; s < R / 2; ++s) {
      if constexpr (KIND == kDst) {
        out[2 * s] = (T)-0.5 * v[s].im;
        out[2 * s + 1] = (T)0.5 * v[s].re;
      } else {
        out[2 * s] = (T)0.5 * v[s].re;
        out[2 * s + 1] = (T)0.5 * v[s].im;
      }
    }
    if constexpr (KIND == kDct) out[R] = (T)0.5 * v[R / 2].re;  // C_M (lane 0: W_{M/2})
  }
}

// buffer position of output slot s of lane tl (-1: no mode)
template <int M, int WPL, int KIND = kDst>
__device__ __forceinline__ int fft_mode(int tl, int s) {
  constexpr int L = FftGeom<M, WPL>::L, R = FftGeom<M, WPL>::R;
  if (tl >= L) return -1;
  if constexpr (KIND == kDct) {
    if (s == R) return tl == 0 ? M + 1 : -1;
    return 2 * (tl + L * (s >> 1)) + (s & 1) + 1;
  } else {
    const int m = 2 * (tl + L * (s >> 1)) + (s & 1);
    return (m >= 1 && m <= M - 1) ? m : -1;
  }
}

// ---------------------------------------------------------------------------
// Dense path: any N <= 1024, one wave per line.  out[s] = S_k, k = 1 + lane + 64 s.
// sintab[r] = sin(pi r/M), r < 2M.  The line is read from buf[n].
// ---------------------------------------------------------------------------
constexpr int kDenseSlots = 16;

// KIND = kDct: out[s] = C_k, k = lane + 64 s (position k + 1), with trig[r] = cos(pi r/M),
// M = N - 1; x_n is read from position n + 1.
template <typename T, int KIND = kDst>
__device__ __forceinline__ void dst_dense(const T* buf, int N, T (&out)[kDenseSlots], int lane,
                                          const double* __restrict__ trig, const T* src = nullptr) {
  const int M = KIND == kDst ? N + 1 : N - 1;
  const int twoM = 2 * M;
#pragma unroll
  for (int s = 0; s < kDenseSlots; ++s) {
    const int pos = 1 + lane + 64 * s;
    T acc = (T)0;
    if (pos <= N) {
      const int k = KIND == kDst ? pos : pos - 1;
      int idx = 0;
      if constexpr (KIND == kDst) {
        for (int n = 1; n <= N; ++n) {
          idx += k;
          if (idx >= twoM) idx -= twoM;
          acc += (src ? src[n] : buf[n]) * (T)trig[idx];
        }
      } else {
        // end nodes with weight 1/2: x_0 (cos 0 = 1) and x_M (cos(pi k) = (-1)^k)
        const T x0 = src ? src[1] : buf[1], xm = src ? src[N] : buf[N];
        acc = (T)0.5 * (x0 + ((k & 1) ? -xm : xm));
        for (int n = 1; n < M; ++n) {
          idx += k;
          if (idx >= twoM) idx -= twoM;
          acc += (src ? src[1 + n] : buf[1 + n]) * (T)trig[idx];
        }
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
