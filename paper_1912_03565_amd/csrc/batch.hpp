// batch.hpp - grouped passes over many independent problems (batches).
//
// A batch of members (problems of any size, scheme and coefficients, one right-hand
// side each) is solved by one launch per pass.  Every pass has a work list: the k-th
// member of the pass's order, perm[k], owns items start[k] .. start[k+1]-1 (tiles of
// the x passes and of the z-marching RHS pass, line groups of the y passes).
// Workgroups are resident and walk the items t0, t0 + gridDim.x, ... (t0 the
// XCD-ordered index of the workgroup, so each XCD takes neighbouring items);
// each item finds its member by binary search in start[] and runs the same per-item
// code as a single solve, dispatched on the member's line-transform size.  With the
// members ordered by decreasing cost per item, the long items are taken first.
#pragma once
#include <type_traits>

#include "kernels.hpp"

namespace cs3d {

struct BatchArgs {
  const ProbDev* P;  // [n] member descriptors (device)
  const int* start;  // [n + 1] item prefix sums of this pass, in the pass's member order (device)
  const int* perm;   // [n] member of each position of that order (device)
  int n;
  int total;
};

// The work lists and member descriptors are read with vector loads (an opaque offset),
// then made uniform again with readfirstlane.  As uniform reads the compiler would turn
// them into scalar loads; with plan tables read that way, plans created after others
// had been destroyed gave wrong results (the cause was not isolated: a stale scalar-cache
// line is one reading, a read of uninitialised workspace another), and these lists are
// rewritten in place by a re-tune, so they stay on the vector path.
__device__ __forceinline__ int vload_int(const int* a) {
  return __builtin_amdgcn_readfirstlane(a[opaque(0)]);
}

__device__ __forceinline__ ProbDev vload_desc(const ProbDev* a) {
  static_assert(sizeof(ProbDev) % 4 == 0, "descriptor of whole words");
  constexpr int N = sizeof(ProbDev) / 4;
  const int* w = reinterpret_cast<const int*>(a) + opaque(0);
  union {
    ProbDev d;
    int u[N];
  } v;
#pragma unroll
  for (int k = 0; k < N; ++k) v.u[k] = __builtin_amdgcn_readfirstlane(w[k]);
  return v.d;
}

// position k of the work list holding `item` (start[k] <= item < start[k+1])
__device__ __forceinline__ int find_slot(const BatchArgs& b, int item) {
  int lo = 0, hi = b.n - 1;
  while (lo < hi) {
    const int mid = (lo + hi + 1) >> 1;
    if (vload_int(b.start + mid) <= item) lo = mid;
    else hi = mid - 1;
  }
  return lo;
}

// statistics blocks of all members
__global__ void kb_stats_reset(unsigned long long* s, int n) {
  const int e = blockIdx.x * blockDim.x + threadIdx.x;
  if (e >= n * kStatsWords) return;
  const int w = e % kStatsWords;
  s[e] = w == 0 ? 0x7FEFFFFFFFFFFFFFull : 0ull;  // bits of DBL_MAX, then zeros
}

// Packed lines (batch tuning `pack`): the FFT of 64 or 128 points keeps M/4 lanes busy
// (4 complex values each), so with packing a wave carries 256/M lines of such a member in
// the x and y passes instead of one; the arithmetic of every line is unchanged.
__host__ __device__ constexpr int pack_lines(int f, int pack) { return (pack && (f == 64 || f == 128)) ? 256 / f : 1; }
// x-pass items: tiles of 8 P y-lines of one plane (P lines per wave); the last tile of a
// plane may reach past the row length ldy, whose positions it neither reads nor writes
__host__ __device__ constexpr int x_tile_lines(int fx, int pack) { return kTileJ * pack_lines(fx, pack); }
__host__ __device__ inline int x_items(int ldy, int nz, int tj) { return ((ldy + tj - 1) / tj) * nz; }
// y-pass items: groups of LPB lines (x-modes)
__host__ __device__ inline int y_items(int nx, int lpb) { return (nx + lpb - 1) / lpb; }
// lanes per line of a y pass (the host's work lists and LDS sizes use it; the kernels
// take it from YCfg, which the assertions below tie to it)
__host__ __device__ constexpr int y_lanes(int fy, int pack) {
  return pack_lines(fy, pack) > 1 ? fy / 4 : 64 * (fy == 1024 ? default_wpl<1024>() : 1);
}
static_assert(y_lanes(64, 1) == YCfg<64, 1, kDst, true>::LANES && y_lanes(128, 1) == YCfg<128, 1, kDst, true>::LANES,
              "packed y lanes");
static_assert(y_lanes(0, 0) == YCfg<0>::LANES && y_lanes(64, 0) == YCfg<64>::LANES &&
                  y_lanes(256, 1) == YCfg<256>::LANES && y_lanes(512, 1) == YCfg<512>::LANES &&
                  y_lanes(1024, 1) == YCfg<1024>::LANES,
              "y lanes of the default waves per line");
static_assert(x_tile_lines(64, 1) == 4 * kTileJ && x_tile_lines(128, 1) == 2 * kTileJ && x_tile_lines(256, 1) == kTileJ &&
                  x_tile_lines(64, 0) == kTileJ,
              "x tile lines");
// RHS items: 64 x 16 tiles times z-chunks
__host__ __device__ inline int rhs_items(int nx, int ny, int nz, int zchunk) {
  return ((nx + kRX - 1) / kRX) * ((ny + kRYBatch - 1) / kRYBatch) * ((nz + zchunk - 1) / zchunk);
}

// Call fn(std::integral_constant<int, M>) for the member's transform size: FFT lengths up
// to MAXM, 0 for the dense sine sums when DENSE (a variant without them keeps the
// register budget of the FFT code; the host picks it only when no member needs them).
template <int MAXM, bool DENSE, typename Fn>
__device__ __forceinline__ void dispatch_m(int M, Fn&& fn) {
  switch (M) {
    case 64: fn(std::integral_constant<int, 64>{}); break;
    case 128: fn(std::integral_constant<int, 128>{}); break;
    case 256: fn(std::integral_constant<int, 256>{}); break;
    case 512:
      if constexpr (MAXM >= 512) fn(std::integral_constant<int, 512>{});
      break;
    case 1024:
      if constexpr (MAXM >= 1024) fn(std::integral_constant<int, 1024>{});
      break;
    default:
      if constexpr (DENSE) fn(std::integral_constant<int, 0>{});
      break;
  }
}

// ---------------------------------------------------------------------------
// RHS pass
// ---------------------------------------------------------------------------
__global__ void __launch_bounds__(kRThreadsBatch) kb_rhs(BatchArgs b) {
  __shared__ double win[kRSlots][RTile<kRYBatch>::SY * kSX];
  __shared__ double kt[2 * kZMax];
  for (int item = xcd_order(blockIdx.x, gridDim.x); item < b.total; item += gridDim.x) {
    const int k = find_slot(b, item);
    const ProbDev p = vload_desc(b.P + vload_int(b.perm + k));
    const int t = item - vload_int(b.start + k);
    const int nbx = (p.nx + kRX - 1) / kRX, nby = (p.ny + kRYBatch - 1) / kRYBatch;
    rhs_block<kRYBatch, true>(p, t % nbx, (t / nbx) % nby, t / (nbx * nby), 0, win, kt);
  }
}

// ---------------------------------------------------------------------------
// x passes: the twiddle tables sit at the start of the LDS, the line buffers after them.
// An item is a tile of TJ = 8 P y-lines of one plane: wave w transforms tile rows
// w P .. w P + P - 1 (lane group sub = lane / LL, LL lanes per line), and the tile is
// transposed through the LDS (row stride tile_stride(nx, TJ)).
// ---------------------------------------------------------------------------
struct XItem {
  int jt, l, row, j, jmax;  // tile, plane, tile row of this lane group, its line, rows inside ldy
  bool active;
};

template <int P>
__device__ __forceinline__ XItem decode_xitem(const ProbDev& p, int t, int row) {
  constexpr int TJ = kTileJ * P;
  const int njt = (p.ldy + TJ - 1) / TJ;
  XItem x;
  x.jt = t % njt;
  x.l = t / njt + 1;
  x.row = row;
  x.j = x.jt * TJ + row;
  x.jmax = min(TJ, p.ldy - x.jt * TJ);
  x.active = x.j >= 1 && x.j <= p.ny;
  return x;
}

template <typename T, int MX, int P>
__device__ __forceinline__ void xfwd_item(const ProbDev& p, int t, T* lines, const cx<T>* tab) {
  constexpr int NS = Tx<MX, 1>::NS;
  constexpr int TJ = kTileJ * P, LL = 64 / P;
  const int w = threadIdx.x >> 6, lane = threadIdx.x & 63;
  const int sub = lane / LL, tl = lane % LL;
  const int bufn = line_buf_elems<T, MX, 1>(p.nx);
  const int ts = tile_stride(p.nx, TJ);
  const XItem x = decode_xitem<P>(p, t, w * P + sub);
  T* buf = lines + x.row * bufn;
  if (x.active) {
    const double* Fr = p.F + (long long)p.nx * ((x.j - 1) + (long long)p.ny * (x.l - 1));
    if (tl == 0) buf[0] = (T)0;
    for (int i = 1 + tl; i <= p.nx; i += LL) buf[i] = (T)Fr[i - 1];
  }
  __syncthreads();
  T out[NS];
  if (x.active) line_dst<T, MX, 1>(buf, p.nx, out, tl, tab, p.sinx);
  __syncthreads();
  if (x.active) {
#pragma unroll
    for (int s = 0; s < NS; ++s) {
      const int n = line_mode<MX, 1>(tl, s, p.nx);
      if (n > 0) lines[x.row * ts + n] = out[s];
    }
  } else {
    for (int n = 1 + tl; n <= p.nx; n += LL) lines[x.row * ts + n] = (T)0;
  }
  __syncthreads();
  T* G = reinterpret_cast<T*>(p.G) + (long long)(x.l - 1) * p.nx * p.ldy + x.jt * TJ;
  for (int idx = threadIdx.x; idx < p.nx * TJ; idx += blockDim.x) {
    const int n0 = idx / TJ, jj = idx % TJ;
    if (jj < x.jmax) G[(long long)n0 * p.ldy + jj] = lines[jj * ts + n0 + 1];
  }
  __syncthreads();
}

template <typename T, int MX, int P>
__device__ __forceinline__ void xinv_item(const ProbDev& p, int t, T* lines, const cx<T>* tab) {
  constexpr int NS = Tx<MX, 1>::NS;
  constexpr int TJ = kTileJ * P, LL = 64 / P;
  const int w = threadIdx.x >> 6, lane = threadIdx.x & 63;
  const int sub = lane / LL, tl = lane % LL;
  const int bufn = line_buf_elems<T, MX, 1>(p.nx);
  const int ts = tile_stride(p.nx, TJ);
  const XItem x = decode_xitem<P>(p, t, w * P + sub);
  T* buf = lines + x.row * bufn;
  const T* G = reinterpret_cast<const T*>(p.G) + (long long)(x.l - 1) * p.nx * p.ldy + x.jt * TJ;
  for (int idx = threadIdx.x; idx < p.nx * TJ; idx += blockDim.x) {
    const int n0 = idx / TJ, jj = idx % TJ;
    lines[jj * ts + n0 + 1] = jj < x.jmax ? G[(long long)n0 * p.ldy + jj] : (T)0;
  }
  __syncthreads();
  T out[NS];
  line_dst<T, MX, 1, true>(buf, p.nx, out, tl, tab, p.sinx, lines + x.row * ts);
  if (x.active) {
    double* u = p.u + (long long)p.nx * ((x.j - 1) + (long long)p.ny * (x.l - 1));
#pragma unroll
    for (int s = 0; s < NS; ++s) {
      const int i = line_mode<MX, 1>(tl, s, p.nx);
      if (i > 0) u[i - 1] = p.scale * (double)out[s];
    }
  }
  __syncthreads();
}

// PACK: lines of 64- and 128-point transforms packed 4 or 2 to a wave (a kernel of its own,
// so the unpacked kernel keeps its register budget)
template <typename T, int MAXM, bool DENSE, bool FWD, bool PACK>
__global__ void __launch_bounds__(64 * kTileJ) kb_x(BatchArgs b) {
  extern __shared__ __align__(16) double smem_raw[];
  T* smem = reinterpret_cast<T*>(smem_raw);
  cx<T>* tab = lds_table(smem);
  T* lines = smem + (size_t)tw_entries<MAXM>() * sizeof(cx<T>) / sizeof(T);
  int curM = -1;
  for (int item = xcd_order(blockIdx.x, gridDim.x); item < b.total; item += gridDim.x) {
    const int k = find_slot(b, item);
    const ProbDev p = vload_desc(b.P + vload_int(b.perm + k));
    const int t = item - vload_int(b.start + k);
    if (p.fx != curM) {  // uniform: reload the tables of this transform size
      __syncthreads();
      dispatch_m<MAXM, DENSE>(p.fx, [&](auto mc) {
        constexpr int MM = decltype(mc)::value;
        if constexpr (MM != 0) load_twiddles<T, MM, 1>(tab, p.twx);
      });
      __syncthreads();
      curM = p.fx;
    }
    dispatch_m<MAXM, DENSE>(p.fx, [&](auto mc) {
      constexpr int MM = decltype(mc)::value;
      constexpr int P = pack_lines(MM, PACK);
      if constexpr (FWD) xfwd_item<T, MM, P>(p, t, lines, tab);
      else xinv_item<T, MM, P>(p, t, lines, tab);
    });
  }
}

// ---------------------------------------------------------------------------
// y passes (default waves per line of each size)
// ---------------------------------------------------------------------------
template <typename T, int MAXM, bool DENSE, bool FWD, bool PACK>
__global__ void __launch_bounds__(kBlockY) kb_y(BatchArgs b) {
  extern __shared__ __align__(16) double smem_raw[];
  T* smem = reinterpret_cast<T*>(smem_raw);
  cx<T>* tab = lds_table(smem);
  T* lines = smem + (size_t)tw_entries<MAXM>() * sizeof(cx<T>) / sizeof(T);
  int curM = -1;
  for (int item = xcd_order(blockIdx.x, gridDim.x); item < b.total; item += gridDim.x) {
    const int k = find_slot(b, item);
    const ProbDev p = vload_desc(b.P + vload_int(b.perm + k));
    const int g = item - vload_int(b.start + k);
    __syncthreads();  // every line of the previous item is done with the LDS
    if (p.fy != curM) {
      dispatch_m<MAXM, DENSE>(p.fy, [&](auto mc) {
        constexpr int MM = decltype(mc)::value;
        if constexpr (MM != 0) load_twiddles<T, MM, default_wpl<MM>()>(tab, p.twy);
      });
      __syncthreads();
      curM = p.fy;
    }
    dispatch_m<MAXM, DENSE>(p.fy, [&](auto mc) {
      constexpr int MM = decltype(mc)::value;
      constexpr bool PK = PACK && (MM == 64 || MM == 128);
      if constexpr (FWD) yfwd_block<T, MM, default_wpl<MM>(), 1, kDst, false, PK>(p, g, 0, 1, lines, tab);
      else yback_block<T, MM, default_wpl<MM>(), 1, kDst, PK>(p, g, 0, 1, lines, tab);
    });
  }
}

}  // namespace cs3d
