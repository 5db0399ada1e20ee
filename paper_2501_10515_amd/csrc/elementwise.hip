// Element-wise and reduction kernels of the residual, the energy and the Jacobi/DIIS update.
//
// Reductions are deterministic: a fixed grid, a fixed per-thread stride pattern, a fixed
// wave64 shuffle tree and a fixed second stage, with no floating-point atomics, so the same
// inputs always give bitwise the same energy, norms and DIIS coefficients.
#include <algorithm>
#include <cmath>

#include <type_traits>

#include "internal.h"

namespace ascc {
namespace {

constexpr int kThreads = 256;
constexpr int kRedBlocks = 1024;  // first-stage blocks of every reduction

struct P4 {
  double* out;
  long os[4];
  int d[4];
  double c0;
  int nin;
  const double* in[4];
  long s[4][4];
  double coef[4];
};

__global__ __launch_bounds__(kThreads) void permute4_kernel(P4 p, long total) {
  for (long idx = blockIdx.x * (long)blockDim.x + threadIdx.x; idx < total; idx += (long)gridDim.x * blockDim.x) {
    long r = idx;
    const int i3 = r % p.d[3];
    r /= p.d[3];
    const int i2 = r % p.d[2];
    r /= p.d[2];
    const int i1 = r % p.d[1];
    const int i0 = r / p.d[1];
    double* o = p.out + i0 * p.os[0] + i1 * p.os[1] + i2 * p.os[2] + i3 * p.os[3];
    double v = (p.c0 == 0.0) ? 0.0 : p.c0 * *o;
#pragma unroll
    for (int t = 0; t < 4; ++t)
      if (t < p.nin) v += p.coef[t] * p.in[t][i0 * p.s[t][0] + i1 * p.s[t][1] + i2 * p.s[t][2] + i3 * p.s[t][3]];
    *o = v;
  }
}

// Same operation when the output is contiguous along i3 and some inputs are contiguous along
// another index t instead (a transposition): 32 x 32 tiles over (i_t, i3) for fixed (i_u, i_w);
// the transposed inputs (bit q of tmask) are summed into an LDS tile with reads along i_t, the
// others are read along i3 with the output row, so reads and writes are coalesced.
__global__ __launch_bounds__(kThreads) void permute4_tiled_kernel(P4 p, int t, int u, int w, int tiles3, int tmask) {
  __shared__ double tile[32][33];
  const int it0 = (blockIdx.x / tiles3) * 32, i30 = (blockIdx.x % tiles3) * 32;
  const long iu = blockIdx.y, iw = blockIdx.z;
  const int tx = threadIdx.x & 31, ty = threadIdx.x >> 5;  // 32 x 8
  const int dt = p.d[t], d3 = p.d[3];
#pragma unroll
  for (int k = 0; k < 4; ++k) {  // tile[i3 - i30][it - it0], reads along it
    const long i3 = i30 + ty + 8 * k, it = it0 + tx;
    double acc = 0.0;
    if (i3 < d3 && it < dt)
      for (int q = 0; q < p.nin; ++q)
        if ((tmask >> q) & 1)
          acc += p.coef[q] * p.in[q][iu * p.s[q][u] + iw * p.s[q][w] + it * p.s[q][t] + i3 * p.s[q][3]];
    tile[ty + 8 * k][tx] = acc;
  }
  __syncthreads();
#pragma unroll
  for (int k = 0; k < 4; ++k) {  // output along i3
    const long it = it0 + ty + 8 * k, i3 = i30 + tx;
    if (it < dt && i3 < d3) {
      double* o = p.out + iu * p.os[u] + iw * p.os[w] + it * p.os[t] + i3 * p.os[3];
      double v = (p.c0 == 0.0) ? 0.0 : p.c0 * *o;
      for (int q = 0; q < p.nin; ++q)
        if (!((tmask >> q) & 1)) v += p.coef[q] * p.in[q][iu * p.s[q][u] + iw * p.s[q][w] + it * p.s[q][t] + i3 * p.s[q][3]];
      *o = v + tile[tx][ty + 8 * k];
    }
  }
}

// Doubles residual, element (i,j,a,b) of the [o][o][v][v] output:
//   R = 1/2 (G1[iajb] + G1[jbia]) + 1/2 (RL[ijab] + RL[jiba]) + EM[ijab] + EM[jiba]
//       - 1/2 (P1[jbia] + P1[iajb]) + 1/2 (P2[jbia] + P2[iajb]) - (P1[ibja] + P1[jaib])
// (ovov arrays are [o][v][o][v]).  G1 and RL are pair-symmetric in exact arithmetic; taking their
// symmetric parts makes R[ijab] = R[jiba] whatever the rounding of the products behind them (a
// low-precision ladder is not), so amplitudes that start pair-symmetric stay so.  The part of t2
// odd under the joint (ij)(ab) swap is outside the closed-shell equations and barely damped by
// the Jacobi step; fed by rounding, it stalls the DIIS iteration of excited (ASCC) states.
// R2[ij][ab] = X(i,j,a,b) + X(j,i,b,a) with
//   X(i,j,a,b) = EM[ijab] + (RL[ijab] + G1[iajb]) / 2 - P1[iajb] / 2 + P2[iajb] / 2 - P1[jaib].
// One workgroup per pair i <= j and 32 x 32 blocks (A, B) of (a, b): it forms X(i,j) on A x B with
// reads along b and X(j,i) on B x A with reads along a (every term is contiguous in the index read
// along), keeps both tiles in LDS and writes R2[ij] on A x B and R2[ji] on B x A, so each input
// element is read once.  For i = j only A <= B runs; with A = B both tiles are the same block and
// the two writes of an element carry the same value.
__device__ __forceinline__ double assemble_x(const double* __restrict__ g1, const double* __restrict__ rl,
                                             const double* __restrict__ em, const double* __restrict__ p1,
                                             const double* __restrict__ p2, long x, long iajb, long jaib) {
  return 0.5 * (g1[iajb] + rl[x]) + em[x] - 0.5 * p1[iajb] + 0.5 * p2[iajb] - p1[jaib];
}

__global__ __launch_bounds__(kThreads) void assemble_r2_kernel(double* __restrict__ r2, const double* __restrict__ g1,
                                                              const double* __restrict__ rl,
                                                              const double* __restrict__ em,
                                                              const double* __restrict__ p1,
                                                              const double* __restrict__ p2, int o, int v) {
  __shared__ double t1[32][33], t2[32][33];  // t1[a - a0][b - b0] = X(i,j,a,b), t2[b - b0][a - a0] = X(j,i,b,a)
  const int tv = (v + 31) / 32;
  const int ta = blockIdx.y / tv, tb = blockIdx.y % tv;
  // pair p = j (j + 1) / 2 + i, i <= j
  const long p = blockIdx.x;
  int j = (int)((sqrt(8.0 * (double)p + 1.0) - 1.0) * 0.5);
  while ((long)j * (j + 1) / 2 > p) --j;
  while ((long)(j + 1) * (j + 2) / 2 <= p) ++j;
  const int i = (int)(p - (long)j * (j + 1) / 2);
  if (i == j && ta > tb) return;
  const int a0 = ta * 32, b0 = tb * 32;
  const int tx = threadIdx.x & 31, ty = threadIdx.x >> 5;  // 32 x 8
  auto ov = [&](int q, int x, int r, int y) -> long { return ((long)(q * v + x) * o + r) * v + y; };
  const long ij = ((long)i * o + j) * v * v, ji = ((long)j * o + i) * v * v;
  double x1[4], x2[4];
#pragma unroll
  for (int k = 0; k < 4; ++k) {
    const int r = ty + 8 * k;
    {  // X(i,j,a,b), a = a0 + r, b = b0 + tx: along b
      const int a = a0 + r, b = b0 + tx;
      x1[k] = (a < v && b < v) ? assemble_x(g1, rl, em, p1, p2, ij + (long)a * v + b, ov(i, a, j, b), ov(j, a, i, b))
                               : 0.0;
      t1[r][tx] = x1[k];
    }
    {  // X(j,i,b,a), b = b0 + r, a = a0 + tx: along a
      const int b = b0 + r, a = a0 + tx;
      x2[k] = (a < v && b < v) ? assemble_x(g1, rl, em, p1, p2, ji + (long)b * v + a, ov(j, b, i, a), ov(i, b, j, a))
                               : 0.0;
      t2[r][tx] = x2[k];
    }
  }
  __syncthreads();
#pragma unroll
  for (int k = 0; k < 4; ++k) {
    const int r = ty + 8 * k;
    {  // R2[ij][a][b] = X(i,j,a,b) + X(j,i,b,a)
      const int a = a0 + r, b = b0 + tx;
      if (a < v && b < v) r2[ij + (long)a * v + b] = x1[k] + t2[tx][r];
    }
    {  // R2[ji][b][a] = X(j,i,b,a) + X(i,j,a,b)
      const int b = b0 + r, a = a0 + tx;
      if (a < v && b < v) r2[ji + (long)b * v + a] = x2[k] + t1[tx][r];
    }
  }
}

__global__ void add_fvo_kernel(double* r1, const double* F, int o, int v) {
  const int idx = blockIdx.x * blockDim.x + threadIdx.x;
  if (idx < o * v) {
    const int i = idx / v, a = idx % v;
    r1[idx] += F[(long)(o + a) * (o + v) + i];
  }
}

// T1 dressing applied from the column correction: for each of the stacked n x n matrices,
//   b(x, q) = S[x][q] + (q < o ? Tc[x][q] : 0)   with Tc[x][i] = sum_a S[x][o + a] t1[i][a],
//   D[p][q] = b(p, q) - [p >= o] sum_{i < o} t1[i][p - o] b(i, q).
// One thread per column q of a 32-row chunk of one matrix: b(i, q) is read once per i and applied to
// all 32 rows; the t1 coefficients depend on the row only, so they are wave-uniform (scalar loads).
__global__ __launch_bounds__(kThreads) void dress_apply_kernel(double* __restrict__ D, const double* __restrict__ S,
                                                               const double* __restrict__ Tc,
                                                               const double* __restrict__ t1, int o, int v) {
  constexpr int RC = 32;
  const int n = o + v;
  const long nn = (long)n * n;
  const int z = blockIdx.z, r0 = blockIdx.x * RC, q = blockIdx.y * kThreads + threadIdx.x;
  if (q >= n) return;
  const double* Sz = S + z * nn;
  const double* Tz = Tc + (long)z * n * o;
  double* Dz = D + z * nn;
  const bool qlo = q < o;
  double acc[RC];
#pragma unroll
  for (int r = 0; r < RC; ++r) {
    const int p = r0 + r;
    acc[r] = p < n ? Sz[(long)p * n + q] + (qlo ? Tz[(long)p * o + q] : 0.0) : 0.0;
  }
  if (r0 + RC > o) {  // the chunk has rows p >= o
    for (int i = 0; i < o; ++i) {
      const double b = Sz[(long)i * n + q] + (qlo ? Tz[(long)i * o + q] : 0.0);
      const double* ti = t1 + (long)i * v;
#pragma unroll
      for (int r = 0; r < RC; ++r) {
        const int p = r0 + r;
        if (p >= o && p < n) acc[r] -= ti[p - o] * b;
      }
    }
  }
#pragma unroll
  for (int r = 0; r < RC; ++r) {
    const int p = r0 + r;
    if (p < n) Dz[(long)p * n + q] = acc[r];
  }
}

// The same dressing with the chunk's t1 coefficients staged in LDS first: for fixed i the 32
// coefficients t1[i][p - o] of the chunk's rows are contiguous, zero for rows p < o or p >= n, so
// the inner loop is branch-free and reads them as LDS broadcasts instead of one dependent scalar
// load per (i, row).
constexpr int kDressRows = 32;
__global__ __launch_bounds__(kThreads) void dress_apply_lds_kernel(double* __restrict__ D, const double* __restrict__ S,
                                                                   const double* __restrict__ Tc,
                                                                   const double* __restrict__ t1, int o, int v) {
  extern __shared__ double coef[];  // [o][kDressRows]
  const int n = o + v;
  const long nn = (long)n * n;
  const int z = blockIdx.z, r0 = blockIdx.x * kDressRows, q = blockIdx.y * kThreads + threadIdx.x;
  const bool lower = r0 + kDressRows > o;  // the chunk has rows p >= o
  if (lower) {
    for (int x = threadIdx.x; x < o * kDressRows; x += kThreads) {
      const int i = x / kDressRows, p = r0 + (x - i * kDressRows);
      coef[x] = (p >= o && p < n) ? t1[(long)i * v + (p - o)] : 0.0;
    }
    __syncthreads();
  }
  if (q >= n) return;
  const double* Sz = S + z * nn;
  const double* Tz = Tc + (long)z * n * o;
  double* Dz = D + z * nn;
  const bool qlo = q < o;
  double acc[kDressRows];
#pragma unroll
  for (int r = 0; r < kDressRows; ++r) {
    const int p = r0 + r;
    acc[r] = p < n ? Sz[(long)p * n + q] + (qlo ? Tz[(long)p * o + q] : 0.0) : 0.0;
  }
  if (lower) {
    for (int i = 0; i < o; ++i) {
      const double b = Sz[(long)i * n + q] + (qlo ? Tz[(long)i * o + q] : 0.0);
      const double* ci = coef + i * kDressRows;
#pragma unroll
      for (int r = 0; r < kDressRows; ++r) acc[r] -= ci[r] * b;
    }
  }
#pragma unroll
  for (int r = 0; r < kDressRows; ++r) {
    const int p = r0 + r;
    if (p < n) Dz[(long)p * n + q] = acc[r];
  }
}

// x -> (1 + c E_hp) x (1 - c E_hp) on each of nb stacked n x n matrices (E_hp: the unit matrix with a
// one at row h, column p): row h += c row p, then column p -= c column h of the result.  One
// workgroup per matrix; the two steps touch disjoint rows / columns of their own step.
__global__ __launch_bounds__(kThreads) void onebody_transform_kernel(double* __restrict__ X, int n, int h, int p,
                                                                     double c) {
  double* Xz = X + (long)blockIdx.x * n * n;
  for (int q = threadIdx.x; q < n; q += kThreads) Xz[(long)h * n + q] += c * Xz[(long)p * n + q];
  __syncthreads();
  for (int r = threadIdx.x; r < n; r += kThreads) Xz[(long)r * n + p] -= c * Xz[(long)r * n + h];
}

// t1 = 0 except t1[h][a] = s1; t2 = 0 except t2[h][h][a][a] = s2.
__global__ __launch_bounds__(kThreads) void initial_guess_kernel(double* __restrict__ t1, double* __restrict__ t2,
                                                                 long len1, long len2, long k1, long k2, double s1,
                                                                 double s2) {
  for (long x = blockIdx.x * (long)kThreads + threadIdx.x; x < len1 + len2; x += (long)gridDim.x * kThreads) {
    if (x < len1)
      t1[x] = (x == k1) ? s1 : 0.0;
    else
      t2[x - len1] = (x - len1 == k2) ? s2 : 0.0;
  }
}

__global__ void diag_trace_kernel(double* J, const double* Bh, int naux, int n, int no) {
  const int Q = blockIdx.x * blockDim.x + threadIdx.x;
  if (Q < naux) {
    const double* b = Bh + (long)Q * n * n;
    double s = 0.0;
    for (int k = 0; k < no; ++k) s += b[(long)k * n + k];
    J[Q] = s;
  }
}

__device__ __forceinline__ double wave_sum(double x) {
#pragma unroll
  for (int off = 32; off > 0; off >>= 1) x += __shfl_down(x, off, 64);
  return x;
}
__device__ __forceinline__ double wave_max(double x) {
#pragma unroll
  for (int off = 32; off > 0; off >>= 1) x = fmax(x, __shfl_down(x, off, 64));
  return x;
}

// Block sum of one value per thread; result valid in thread 0.
__device__ double block_sum(double x, double* sh) {
  x = wave_sum(x);
  const int lane = threadIdx.x & 63, w = threadIdx.x >> 6;
  __syncthreads();
  if (lane == 0) sh[w] = x;
  __syncthreads();
  double s = 0.0;
  if (threadIdx.x == 0)
    for (int k = 0; k < (int)(blockDim.x >> 6); ++k) s += sh[k];
  return s;
}
__device__ double block_max(double x, double* sh) {
  x = wave_max(x);
  const int lane = threadIdx.x & 63, w = threadIdx.x >> 6;
  __syncthreads();
  if (lane == 0) sh[w] = x;
  __syncthreads();
  double s = 0.0;
  if (threadIdx.x == 0)
    for (int k = 0; k < (int)(blockDim.x >> 6); ++k) s = fmax(s, sh[k]);
  return s;
}

__global__ __launch_bounds__(kThreads) void energy_stage1(double* partial, const double* __restrict__ t1,
                                                         const double* __restrict__ t2,
                                                         const double* __restrict__ L, int o, int v, long total) {
  __shared__ double sh[kThreads / 64];
  double acc = 0.0;
  const long vv = (long)v * v, ovv = (long)o * vv;
  for (long idx = blockIdx.x * (long)blockDim.x + threadIdx.x; idx < total; idx += (long)gridDim.x * blockDim.x) {
    const int i = idx / ovv;
    const int j = (idx / vv) % o;
    const int a = (idx / v) % v;
    const int b = idx % v;
    acc += (t2[idx] + t1[i * v + a] * t1[j * v + b]) * L[idx];
  }
  const double s = block_sum(acc, sh);
  if (threadIdx.x == 0) partial[blockIdx.x] = s;
}

__global__ __launch_bounds__(kThreads) void energy_stage2(double* e, const double* partial, int nblk,
                                                         const double* t1, const double* fov, int nov) {
  __shared__ double sh[kThreads / 64];
  double acc = 0.0;
  for (int k = threadIdx.x; k < nblk; k += blockDim.x) acc += partial[k];
  for (int k = threadIdx.x; k < nov; k += blockDim.x) acc += 2.0 * fov[k] * t1[k];
  const double s = block_sum(acc, sh);
  if (threadIdx.x == 0) *e = s;
}

// ---------------------------------------------------------------------------------------
// Jacobi step + DIIS.
//
// Element x of the amplitude vector t1 (+) t2 gets s = R/D, t_new = t + s.  When the call
// stores a DIIS pair, (t_new, s) go to history slot `head`, and the overlaps <s, e_k> with
// every stored error vector are accumulated (the new slot's own entry is <s, s>).
// Partial sums per block: [0] sum R^2, [1] max|R|, [2] non-finite count, [3 + k] <s, e_k>.

__device__ __forceinline__ double denom(long x, int o, int v, const double* eps, double shift) {
  const long ov = (long)o * v;
  if (x < ov) {
    const int i = x / v, a = x % v;
    return eps[i] - eps[o + a] - shift;
  }
  const long y = x - ov, vv = (long)v * v, ovv = (long)o * vv;
  const int i = y / ovv, j = (y / vv) % o, a = (y / v) % v, b = y % v;
  return eps[i] + eps[j] - eps[o + a] - eps[o + b] - shift;
}

struct UK {
  double* t1;
  double* t2;
  const double* r1;
  const double* r2;
  const double* eps;
  double* hist_t;
  double* hist_e;
  double* partial;
  const DiisState* st;
  int o, v, m, start, nstat;
  long len;
  double shift;
  long ss;         // byte stride between the slots of a batched update (0: one slot)
  const int* tab;  // slot of grid row blockIdx.y (nullptr: blockIdx.y)
};

// The same pointer in slot k of a batched update (slots at a fixed byte stride).
template <class T>
__device__ __forceinline__ T* in_slot(T* p, long k, long ss) {
  return reinterpret_cast<T*>(reinterpret_cast<char*>(const_cast<typename std::remove_const<T>::type*>(p)) + k * ss);
}

__global__ __launch_bounds__(kThreads) void update_stage1(UK p) {
  if (p.ss) {  // this grid row's slot
    const long k = p.tab ? p.tab[blockIdx.y] : blockIdx.y;
    p.t1 = in_slot(p.t1, k, p.ss);
    p.t2 = in_slot(p.t2, k, p.ss);
    p.r1 = in_slot(p.r1, k, p.ss);
    p.r2 = in_slot(p.r2, k, p.ss);
    p.eps = in_slot(p.eps, k, p.ss);
    p.hist_t = in_slot(p.hist_t, k, p.ss);
    p.hist_e = in_slot(p.hist_e, k, p.ss);
    p.partial = in_slot(p.partial, k, p.ss);
    p.st = in_slot(p.st, k, p.ss);
  }
  __shared__ double sh[kThreads / 64];
  const int head = p.st->head;
  const bool store = p.st->calls >= p.start;  // decided on the device, so a captured graph replays it
  bool valid[kMaxDiis];
  for (int k = 0; k < kMaxDiis; ++k) valid[k] = store && k < p.m && (k == head || p.st->slot_age[k] >= 0);
  double dots[kMaxDiis];
  for (int k = 0; k < kMaxDiis; ++k) dots[k] = 0.0;
  double rr = 0.0, rmax = 0.0, bad = 0.0;
  const long ov = (long)p.o * p.v;
  for (long x = blockIdx.x * (long)blockDim.x + threadIdx.x; x < p.len; x += (long)gridDim.x * blockDim.x) {
    const double r = (x < ov) ? p.r1[x] : p.r2[x - ov];
    double* tp = (x < ov) ? (p.t1 + x) : (p.t2 + (x - ov));
    const double s = r / denom(x, p.o, p.v, p.eps, p.shift);
    const double tn = *tp + s;
    *tp = tn;
    rr += r * r;
    rmax = fmax(rmax, fabs(r));
    if (!isfinite(r)) bad += 1.0;
    if (store) {
      for (int k = 0; k < kMaxDiis; ++k)
        if (valid[k]) dots[k] += s * ((k == head) ? s : p.hist_e[(long)k * p.len + x]);
      p.hist_t[(long)head * p.len + x] = tn;
      p.hist_e[(long)head * p.len + x] = s;
    }
  }
  double* out = p.partial + (long)blockIdx.x * p.nstat;
  double v = block_sum(rr, sh);
  if (threadIdx.x == 0) out[0] = v;
  v = block_max(rmax, sh);
  if (threadIdx.x == 0) out[1] = v;
  v = block_sum(bad, sh);
  if (threadIdx.x == 0) out[2] = v;
  for (int k = 0; k < p.m; ++k) {
    v = block_sum(dots[k], sh);
    if (threadIdx.x == 0) out[3 + k] = v;
  }
}

// Bordered DIIS system over the valid slots, oldest first; returns false if a pivot is tiny.
// A and xs: (kMaxDiis + 1) x (kMaxDiis + 2) and kMaxDiis + 1 doubles of the caller's LDS (one thread
// eliminates; LDS rather than private arrays, which would live in scratch memory).
__device__ bool diis_solve(DiisState* st, int m, double* A, double* xs) {
  int order[kMaxDiis];
  int nv = 0;
  for (int k = 0; k < m; ++k)
    if (st->slot_age[k] >= 0) order[nv++] = k;
  for (int x = 1; x < nv; ++x)  // insertion sort by age (oldest first)
    for (int y = x; y > 0 && st->slot_age[order[y - 1]] > st->slot_age[order[y]]; --y) {
      const int t = order[y];
      order[y] = order[y - 1];
      order[y - 1] = t;
    }
  constexpr int W = kMaxDiis + 2;
  const int nn = nv + 1;
  double scale = 0.0;
  for (int r = 0; r < nv; ++r)
    for (int c = 0; c < nv; ++c) scale = fmax(scale, fabs(st->Bm[order[r] * kMaxDiis + order[c]]));
  for (int r = 0; r < nn; ++r)
    for (int c = 0; c <= nn; ++c) {
      double x;
      if (c == nn)
        x = (r == nv) ? -1.0 : 0.0;
      else if (r < nv && c < nv)
        x = st->Bm[order[r] * kMaxDiis + order[c]];
      else if (r == nv && c == nv)
        x = 0.0;
      else
        x = -1.0;
      A[r * W + c] = x;
    }
  for (int c = 0; c < nn; ++c) {
    int piv = c;
    for (int r = c + 1; r < nn; ++r)
      if (fabs(A[r * W + c]) > fabs(A[piv * W + c])) piv = r;
    if (!(fabs(A[piv * W + c]) >= 1e-14 * scale)) return false;
    if (piv != c)
      for (int k = 0; k <= nn; ++k) {
        const double t = A[c * W + k];
        A[c * W + k] = A[piv * W + k];
        A[piv * W + k] = t;
      }
    for (int r = c + 1; r < nn; ++r) {
      const double f = A[r * W + c] / A[c * W + c];
      for (int k = c; k <= nn; ++k) A[r * W + k] -= f * A[c * W + k];
    }
  }
  for (int r = nn - 1; r >= 0; --r) {
    double acc = A[r * W + nn];
    for (int k = r + 1; k < nn; ++k) acc -= A[r * W + k] * xs[k];
    xs[r] = acc / A[r * W + r];
  }
  for (int k = 0; k < kMaxDiis; ++k) st->coef[k] = 0.0;
  for (int r = 0; r < nv; ++r) st->coef[order[r]] = xs[r];
  return true;
}

__global__ __launch_bounds__(kThreads) void update_stage2(DiisState* st, const double* partial, int nblk, int nstat,
                                                         int m, int start, const double* e, double* stats,
                                                         double shift, long ss, const int* tab) {
  if (ss) {  // this grid row's slot; its statistics block is row k of stats
    const long k = tab ? tab[blockIdx.y] : blockIdx.y;
    st = in_slot(st, k, ss);
    partial = in_slot(partial, k, ss);
    e = in_slot(e, k, ss);
    stats += 8 * k;
  }
  const bool store = st->calls >= start;
  __shared__ double sh[kThreads / 64];
  __shared__ double red[3 + kMaxDiis];
  __shared__ double sysA[(kMaxDiis + 1) * (kMaxDiis + 2)], sysx[kMaxDiis + 1];
  double a = 0.0;
  for (int k = threadIdx.x; k < nblk; k += blockDim.x) a += partial[(long)k * nstat + 0];
  double v = block_sum(a, sh);
  if (threadIdx.x == 0) red[0] = v;
  a = 0.0;
  for (int k = threadIdx.x; k < nblk; k += blockDim.x) a = fmax(a, partial[(long)k * nstat + 1]);
  v = block_max(a, sh);
  if (threadIdx.x == 0) red[1] = v;
  a = 0.0;
  for (int k = threadIdx.x; k < nblk; k += blockDim.x) a += partial[(long)k * nstat + 2];
  v = block_sum(a, sh);
  if (threadIdx.x == 0) red[2] = v;
  for (int q = 0; q < m; ++q) {
    a = 0.0;
    for (int k = threadIdx.x; k < nblk; k += blockDim.x) a += partial[(long)k * nstat + 3 + q];
    v = block_sum(a, sh);
    if (threadIdx.x == 0) red[3 + q] = v;
  }
  if (threadIdx.x != 0) return;

  const double E = *e;
  int flags = 0;
  if (red[2] > 0.0 || !isfinite(E) || !isfinite(red[0])) flags |= 1;
  if (store) {
    const int head = st->head;
    for (int k = 0; k < m; ++k)
      if (k == head || st->slot_age[k] >= 0) {
        st->Bm[head * kMaxDiis + k] = red[3 + k];
        st->Bm[k * kMaxDiis + head] = red[3 + k];
      }
    st->slot_age[head] = st->counter++;
    st->head = (head + 1) % m;
    int nvalid = 0;
    for (int k = 0; k < m; ++k) nvalid += (st->slot_age[k] >= 0);
    st->nvec = nvalid;
    for (int k = 0; k < kMaxDiis; ++k) st->coef[k] = 0.0;
    while (st->nvec >= 2 && !(flags & 1)) {
      if (diis_solve(st, m, sysA, sysx)) break;
      int oldest = -1;
      for (int k = 0; k < m; ++k)
        if (st->slot_age[k] >= 0 && (oldest < 0 || st->slot_age[k] < st->slot_age[oldest])) oldest = k;
      st->slot_age[oldest] = -1;
      st->nvec -= 1;
      flags |= 2;
      for (int k = 0; k < kMaxDiis; ++k) st->coef[k] = 0.0;
    }
  }
  stats[0] = E;
  stats[1] = st->has_prev ? E - st->e_prev : INFINITY;
  stats[2] = red[1];
  stats[3] = sqrt(red[0]);
  stats[4] = st->nvec;
  stats[5] = flags;
  stats[6] = st->calls;
  stats[7] = shift;
  st->e_prev = E;
  st->has_prev = 1;
  st->flags = flags;
  st->calls += 1;
}

// t <- sum_k coef[k] hist_t[k] once two or more pairs are stored (no-op otherwise).
__global__ __launch_bounds__(kThreads) void update_stage3(double* t1, double* t2, const double* hist_t,
                                                         const DiisState* st, int m, long ov, long len, long ss,
                                                         const int* tab) {
  if (ss) {
    const long k = tab ? tab[blockIdx.y] : blockIdx.y;
    t1 = in_slot(t1, k, ss);
    t2 = in_slot(t2, k, ss);
    hist_t = in_slot(hist_t, k, ss);
    st = in_slot(st, k, ss);
  }
  if (st->nvec < 2 || (st->flags & 1)) return;
  double c[kMaxDiis];
  for (int k = 0; k < kMaxDiis; ++k) c[k] = (k < m) ? st->coef[k] : 0.0;
  for (long x = blockIdx.x * (long)blockDim.x + threadIdx.x; x < len; x += (long)gridDim.x * blockDim.x) {
    double acc = 0.0;
    for (int k = 0; k < m; ++k)
      if (c[k] != 0.0) acc += c[k] * hist_t[(long)k * len + x];
    if (x < ov)
      t1[x] = acc;
    else
      t2[x - ov] = acc;
  }
}


// ---------------------------------------------------------------------------------------
// Pair packing for the particle-particle ladder.
//
// Pair index of i <= j among n: pidx(i, j) = i*n - i*(i-1)/2 + (j - i)  (row-major upper triangle).
__device__ __forceinline__ long pidx(long i, long j, long n) { return i * n - i * (i - 1) / 2 + (j - i); }

// t+-[p(i,j)][p(c,d)] for i <= j, c <= d:
//   t+ = (t_ij^cd + t_ij^dc)/2 (c < d), dscale * t_ij^cc (c = d);  t- = (t_ij^cd - t_ij^dc)/2 (c < d), 0 (c = d).
__global__ __launch_bounds__(kThreads) void pack_tpm_kernel(double* __restrict__ tplus, double* __restrict__ tminus,
                                                           const double* __restrict__ t2, int o, int v, double dscale) {
  const int i = blockIdx.y / o, j = blockIdx.y % o;
  if (i > j) return;
  const long Tv = (long)v * (v + 1) / 2, vv = (long)v * v;
  const double* src = t2 + ((long)i * o + j) * vv;
  const long p = pidx(i, j, o);
  double* plus = tplus + p * Tv;
  double* minus = tminus + p * Tv;
  for (long x = blockIdx.x * (long)blockDim.x + threadIdx.x; x < vv; x += (long)gridDim.x * blockDim.x) {
    const int c = x / v, d = x % v;
    if (c > d) continue;
    const double a = src[x], b = src[(long)d * v + c];
    const long k = pidx(c, d, v);
    plus[k] = (c == d) ? dscale * a : 0.5 * (a + b);
    minus[k] = (c == d) ? 0.0 : 0.5 * (a - b);
  }
}

// RL[i][j][a][b] from R+-[p][p(a,b)]: R^ab = R+ + R- (a <= b), R+ - R- (a > b), with R_ij = R_ji^T.
// One workgroup per pair i <= j and 32 x 32 block (A <= B) of (a, b): with u = R+ + R-, w = R+ - R-
// at the packed index p(a, b), a <= b, the four outputs are RL[i][j][a][b] = RL[j][i][b][a] = u and
// RL[i][j][b][a] = RL[j][i][a][b] = w (the residual's pair symmetry; R- vanishes on a = b).  Each
// packed element is read once; the transposed writes go through an LDS tile.
__global__ __launch_bounds__(kThreads) void unpack_rpm_kernel(double* __restrict__ RL, const double* __restrict__ Rplus,
                                                             const double* __restrict__ Rminus, int o, int v,
                                                             int nblk) {
  __shared__ double tu[32][33], tw[32][33];
  const long Tv = (long)v * (v + 1) / 2, vv = (long)v * v;
  // block pair (A, B), A <= B, from blockIdx.x
  int A = 0, rem = blockIdx.x;
  while (rem >= nblk - A) {
    rem -= nblk - A;
    ++A;
  }
  const int B = A + rem;
  int i = 0, prem = blockIdx.y;  // pair i <= j from blockIdx.y
  while (prem >= o - i) {
    prem -= o - i;
    ++i;
  }
  const int j = i + prem;
  const long p = pidx(i, j, o);
  const double* plus = Rplus + p * Tv;
  const double* minus = Rminus + p * Tv;
  double* dij = RL + ((long)i * o + j) * vv;
  double* dji = RL + ((long)j * o + i) * vv;
  const int a0 = 32 * A, b0 = 32 * B;
  const int tx = threadIdx.x & 31, ty = threadIdx.x >> 5;  // 32 x 8
  // read: rows a = a0 + ty + 8r, columns b = b0 + tx (contiguous in the packed row)
#pragma unroll
  for (int r = 0; r < 4; ++r) {
    const int la = ty + 8 * r, a = a0 + la, b = b0 + tx;
    double u = 0.0, w = 0.0;
    const bool in = a < v && b < v && a <= b;
    if (in) {
      const long k = pidx(a, b, v);
      const double x = plus[k], y = minus[k];
      u = x + y;
      w = x - y;
      dij[(long)a * v + b] = u;
      if (i != j) dji[(long)a * v + b] = (a == b) ? u : w;
    }
    tu[la][tx] = u;
    tw[la][tx] = w;
  }
  __syncthreads();
  // transposed writes: position (b, a), a = a0 + tx contiguous
#pragma unroll
  for (int r = 0; r < 4; ++r) {
    const int lb = ty + 8 * r, b = b0 + lb, a = a0 + tx;
    if (a < v && b < v && a < b) {
      dij[(long)b * v + a] = tw[tx][lb];
      if (i != j) dji[(long)b * v + a] = tu[tx][lb];
    }
  }
}

// V+-[p(a,b)][p(c,d)] for a in [a0, a1), b >= a, from W[a - a0][b][c][d] = (ac|bd):
//   V+ = W[.][c][d] + W[.][d][c] (c < d), W[.][c][c] (c = d);  V- = W[.][c][d] - W[.][d][c] (c < d), 0 (c = d).
__global__ __launch_bounds__(kThreads) void pack_vvvv_kernel(double* __restrict__ Vp, const double* __restrict__ W,
                                                            int a0, int v) {
  const int a = a0 + blockIdx.y / v, b = blockIdx.y % v;
  if (b < a) return;
  const long Tv = (long)v * (v + 1) / 2, vv = (long)v * v;
  const double* src = W + ((long)(a - a0) * v + b) * vv;
  const long r = pidx(a, b, v);
  double* plus = Vp + r * Tv;
  double* minus = Vp + (Tv + r) * Tv;
  for (long x = blockIdx.x * (long)blockDim.x + threadIdx.x; x < vv; x += (long)gridDim.x * blockDim.x) {
    const int c = x / v, d = x % v;
    if (c > d) continue;
    const double w1 = src[x], w2 = src[(long)d * v + c];
    const long k = pidx(c, d, v);
    plus[k] = (c == d) ? w1 : w1 + w2;
    minus[k] = (c == d) ? 0.0 : w1 - w2;
  }
}

// Pair order of the full (ac|bd) storage: R(a,b) = p(a,b) for a <= b, T(v) + strict pair index of
// (b,a) for a > b; pm[n] = R(b,a) for pair n = (a <= b) (n itself when a = b).
__device__ __forceinline__ long pair_order(long a, long b, long v) {
  const long Tv = v * (v + 1) / 2;
  return a <= b ? pidx(a, b, v) : Tv + pidx(b, a, v) - (b + 1);
}

__global__ __launch_bounds__(kThreads) void pair_minus_rows_kernel(int* __restrict__ pm, int v) {
  const int a = blockIdx.x * kThreads + threadIdx.x;
  if (a >= v) return;
  for (int b = a; b < v; ++b) pm[pidx(a, b, v)] = (int)pair_order(b, a, v);
}

// Full (ac|bd) in pair order: V[R(a,b)][R(c,d)] = W[a - a0][b][c][d] for a in [a0, a1).
__global__ __launch_bounds__(kThreads) void pack_full_kernel(double* __restrict__ V, const double* __restrict__ W,
                                                            int a0, int v) {
  const int a = a0 + blockIdx.y / v, b = blockIdx.y % v;
  const long vv = (long)v * v;
  const double* src = W + ((long)(a - a0) * v + b) * vv;
  double* dst = V + pair_order(a, b, v) * vv;
  for (long x = blockIdx.x * (long)blockDim.x + threadIdx.x; x < vv; x += (long)gridDim.x * blockDim.x) {
    const int c = x / v, d = x % v;
    dst[pair_order(c, d, v)] = src[x];
  }
}

inline int grid_for(long total) {
  long g = (total + kThreads - 1) / kThreads;
  if (g > 8192) g = 8192;
  if (g < 1) g = 1;
  return (int)g;
}

}  // namespace

static bool p4_in_bounds(const P4& p) {
  const char* names[4] = {"permute input 0", "permute input 1", "permute input 2", "permute input 3"};
  long lo = 0, hi = 0;
  for (int k = 0; k < 4; ++k) {
    const long d = (long)(p.d[k] - 1) * p.os[k];
    if (d < 0) lo += d; else hi += d;
  }
  if (!range_ok(p.out, lo, hi, sizeof(double), "permute output")) return false;
  for (int t = 0; t < p.nin; ++t) {
    lo = hi = 0;
    for (int k = 0; k < 4; ++k) {
      const long d = (long)(p.d[k] - 1) * p.s[t][k];
      if (d < 0) lo += d; else hi += d;
    }
    if (!range_ok(p.in[t], lo, hi, sizeof(double), names[t])) return false;
  }
  return true;
}

// Drops size-1 dimensions (the remaining ones keep their order, right-aligned), then takes the
// tiled kernel when the output is contiguous along its last index and some input is contiguous
// along another index of at least 16.
static hipError_t launch_permute(P4 p, long total, hipStream_t s) {
  P4 c = p;
  int k2 = 3;
  for (int k = 3; k >= 0; --k) {
    if (p.d[k] == 1) continue;
    c.d[k2] = p.d[k];
    c.os[k2] = p.os[k];
    for (int q = 0; q < p.nin; ++q) c.s[q][k2] = p.s[q][k];
    --k2;
  }
  for (; k2 >= 0; --k2) {
    c.d[k2] = 1;
    c.os[k2] = 0;
    for (int q = 0; q < p.nin; ++q) c.s[q][k2] = 0;
  }
  int t = -1, tmask = 0;
  if (c.os[3] == 1 && c.d[3] >= 16) {
    for (int k = 2; k >= 0 && t < 0; --k) {
      if (c.d[k] < 16) continue;
      int m = 0;
      for (int q = 0; q < c.nin; ++q)
        if (c.s[q][k] == 1 && c.s[q][3] != 1) m |= 1 << q;
      if (m) {
        t = k;
        tmask = m;
      }
    }
  }
  if (t >= 0) {
    int u = -1, w = -1;
    for (int k = 0; k < 3; ++k)
      if (k != t) (u < 0 ? u : w) = k;
    const long tiles_t = (c.d[t] + 31) / 32, tiles3 = (c.d[3] + 31) / 32;
    if (tiles_t * tiles3 <= 0x7fffffffL && c.d[u] <= 65535 && c.d[w] <= 65535) {
      hipLaunchKernelGGL(permute4_tiled_kernel, dim3((unsigned)(tiles_t * tiles3), (unsigned)c.d[u], (unsigned)c.d[w]),
                         dim3(kThreads), 0, s, c, t, u, w, (int)tiles3, tmask);
      return hipGetLastError();
    }
  }
  hipLaunchKernelGGL(permute4_kernel, dim3(grid_for(total)), dim3(kThreads), 0, s, p, total);
  return hipGetLastError();
}

hipError_t permute4(double* out, const int dims[4], double c0, const Perm4In* in, int nin, hipStream_t s) {
  // contiguous output with the given dims
  P4 p{};
  p.out = out;
  p.os[3] = 1;
  p.os[2] = dims[3];
  p.os[1] = (long)dims[3] * dims[2];
  p.os[0] = (long)dims[3] * dims[2] * dims[1];
  for (int k = 0; k < 4; ++k) p.d[k] = dims[k];
  p.c0 = c0;
  p.nin = nin;
  for (int t = 0; t < nin; ++t) {
    p.in[t] = in[t].p;
    p.coef[t] = in[t].coef;
    for (int k = 0; k < 4; ++k) p.s[t][k] = in[t].s[k];
  }
  const long total = (long)dims[0] * dims[1] * dims[2] * dims[3];
  if (total <= 0) return hipSuccess;
  if (bounds_checking() && !p4_in_bounds(p)) return hipErrorInvalidValue;
  if (dry_run()) return hipSuccess;
  return launch_permute(p, total, s);
}

hipError_t permute4_strided(double* out, const long ostr[4], const int dims[4], double c0, const Perm4In* in,
                            int nin, hipStream_t s) {
  P4 p{};
  p.out = out;
  for (int k = 0; k < 4; ++k) {
    p.os[k] = ostr[k];
    p.d[k] = dims[k];
  }
  p.c0 = c0;
  p.nin = nin;
  for (int t = 0; t < nin; ++t) {
    p.in[t] = in[t].p;
    p.coef[t] = in[t].coef;
    for (int k = 0; k < 4; ++k) p.s[t][k] = in[t].s[k];
  }
  const long total = (long)dims[0] * dims[1] * dims[2] * dims[3];
  if (total <= 0) return hipSuccess;
  if (bounds_checking() && !p4_in_bounds(p)) return hipErrorInvalidValue;
  if (dry_run()) return hipSuccess;
  return launch_permute(p, total, s);
}

hipError_t assemble_r2(double* r2, const double* g1, const double* rl, const double* em, const double* p1,
                       const double* p2, int no, int nv, hipStream_t s) {
  const long total = (long)no * no * nv * nv;
  const long ovov = (long)no * nv * no * nv;
  if (bounds_checking() &&
      !(range_ok(r2, 0, total - 1, 8, "assemble r2") && range_ok(g1, 0, ovov - 1, 8, "assemble g1") &&
        range_ok(rl, 0, total - 1, 8, "assemble rl") && range_ok(em, 0, total - 1, 8, "assemble em") &&
        range_ok(p1, 0, ovov - 1, 8, "assemble p1") && range_ok(p2, 0, ovov - 1, 8, "assemble p2")))
    return hipErrorInvalidValue;
  if (dry_run()) return hipSuccess;
  const long tv = (nv + 31) / 32, pairs = (long)no * (no + 1) / 2;
  if (tv * tv > 65535 || pairs > 0x7fffffffL) return hipErrorInvalidValue;
  hipLaunchKernelGGL(assemble_r2_kernel, dim3((unsigned)pairs, (unsigned)(tv * tv)), dim3(kThreads), 0, s, r2, g1, rl,
                     em, p1, p2, no, nv);
  return hipGetLastError();
}

hipError_t add_fvo(double* r1, const double* fhat, int no, int nv, hipStream_t s) {
  const int total = no * nv;
  const long n = no + nv;
  if (bounds_checking() && !(range_ok(r1, 0, total - 1, 8, "add_fvo r1") && range_ok(fhat, 0, n * n - 1, 8, "add_fvo F")))
    return hipErrorInvalidValue;
  if (dry_run()) return hipSuccess;
  hipLaunchKernelGGL(add_fvo_kernel, dim3((total + 255) / 256), dim3(256), 0, s, r1, fhat, no, nv);
  return hipGetLastError();
}

hipError_t dress_apply(double* D, const double* S, const double* Tc, const double* t1, int o, int v, int nb,
                       hipStream_t s) {
  const long n = o + v;
  if (o < 1 || v < 1 || nb < 1 || nb > 65535) return hipErrorInvalidValue;
  if (bounds_checking() && !(range_ok(D, 0, nb * n * n - 1, 8, "dress D") && range_ok(S, 0, nb * n * n - 1, 8, "dress S") &&
                             range_ok(Tc, 0, nb * n * o - 1, 8, "dress Tc") && range_ok(t1, 0, (long)o * v - 1, 8, "dress t1")))
    return hipErrorInvalidValue;
  if (dry_run()) return hipSuccess;
  if (o <= 256) {  // coefficients of one chunk: o * 32 doubles of LDS, 64 KB at most
    hipLaunchKernelGGL(dress_apply_lds_kernel,
                       dim3((unsigned)((n + kDressRows - 1) / kDressRows), (unsigned)((n + kThreads - 1) / kThreads),
                            (unsigned)nb),
                       dim3(kThreads), (size_t)o * kDressRows * sizeof(double), s, D, S, Tc, t1, o, v);
    return hipGetLastError();
  }
  hipLaunchKernelGGL(dress_apply_kernel, dim3((unsigned)((n + 31) / 32), (unsigned)((n + kThreads - 1) / kThreads), (unsigned)nb),
                     dim3(kThreads), 0, s, D, S, Tc, t1, o, v);
  return hipGetLastError();
}

hipError_t onebody_transform(double* X, long nb, int n, int h, int p, double c, hipStream_t s) {
  if (nb < 1 || n < 1) return hipSuccess;
  if (h < 0 || h >= n || p < 0 || p >= n || h == p || nb > 0x7fffffffL) return hipErrorInvalidValue;
  if (bounds_checking() && !range_ok(X, 0, nb * n * n - 1, 8, "one-body transform")) return hipErrorInvalidValue;
  if (dry_run()) return hipSuccess;
  hipLaunchKernelGGL(onebody_transform_kernel, dim3((unsigned)nb), dim3(kThreads), 0, s, X, n, h, p, c);
  return hipGetLastError();
}

hipError_t initial_guess(double* t1, double* t2, int no, int nv, int h, int a, double s1, double s2, hipStream_t s) {
  const long len1 = (long)no * nv, len2 = len1 * len1;
  if (h < 0 || h >= no || a < 0 || a >= nv) return hipErrorInvalidValue;
  if (bounds_checking() && !(range_ok(t1, 0, len1 - 1, 8, "guess t1") && range_ok(t2, 0, len2 - 1, 8, "guess t2")))
    return hipErrorInvalidValue;
  if (dry_run()) return hipSuccess;
  const long k1 = (long)h * nv + a, k2 = (((long)h * no + h) * nv + a) * nv + a;
  hipLaunchKernelGGL(initial_guess_kernel, dim3(grid_for(len1 + len2)), dim3(kThreads), 0, s, t1, t2, len1, len2, k1,
                     k2, s1, s2);
  return hipGetLastError();
}

// ---------------------------------------------------------------------------------------
// Cross index sets (internal.h): over r = i * nv + a (i < no, a < nv) the members i == h or
// a == pa, m = nv + no - 1 of them in the compact order k < nv -> (h, k), k = nv + q -> (i, pa)
// with i = q (q < h) or q + 1 (q >= h).
__device__ __forceinline__ long cross_row(const Cross& X, long k) {
  if (k < X.nv) return (long)X.h * X.nv + k;
  const long q = k - X.nv;
  return (q < X.h ? q : q + 1) * (long)X.nv + X.pa;
}
__device__ __forceinline__ bool cross_member(const Cross& X, long r) { return r / X.nv == X.h || r % X.nv == X.pa; }

// dst[k][c] = src[cross_row(k)][c] (c < ncols); with zero_diag, the entry whose row and column
// are both the cross's corner r = h * nv + pa is written as 0.
__global__ void cross_gather_rows_kernel(double* __restrict__ dst, long ldd, const double* __restrict__ src, long lds,
                                         long ncols, Cross X, int zero_diag) {
  const long m = X.m(), total = m * ncols, hp = (long)X.h * X.nv + X.pa;
  for (long x = blockIdx.x * (long)blockDim.x + threadIdx.x; x < total; x += (long)gridDim.x * blockDim.x) {
    const long k = x / ncols, c = x - k * ncols;
    const long r = cross_row(X, k);
    dst[k * ldd + c] = (zero_diag && r == hp && c == hp) ? 0.0 : src[r * lds + c];
  }
}

// dst[r][k] = src[r][cross_row(k)] for k < m and 0 for m <= k < ldd (padding); with zero_rows,
// rows r that are members of the row cross R are written as 0.
__global__ void cross_gather_cols_kernel(double* __restrict__ dst, long ldd, const double* __restrict__ src, long lds,
                                         long nrows, Cross X, Cross R, int zero_rows) {
  const long m = X.m(), total = nrows * ldd;
  for (long x = blockIdx.x * (long)blockDim.x + threadIdx.x; x < total; x += (long)gridDim.x * blockDim.x) {
    const long r = x / ldd, k = x - r * ldd;
    dst[x] = (k >= m || (zero_rows && cross_member(R, r))) ? 0.0 : src[r * lds + cross_row(X, k)];
  }
}

// dst[cross_row(k)][c] += alpha * src[k][c] (members are distinct: no two threads share a target).
__global__ void cross_scatter_add_rows_kernel(double* __restrict__ dst, long ldd, const double* __restrict__ src,
                                              long lds, long ncols, double alpha, Cross X) {
  const long m = X.m(), total = m * ncols;
  for (long x = blockIdx.x * (long)blockDim.x + threadIdx.x; x < total; x += (long)gridDim.x * blockDim.x) {
    const long k = x / ncols, c = x - k * ncols;
    dst[cross_row(X, k) * ldd + c] += alpha * src[k * lds + c];
  }
}

// dst[r][cross_row(k)] += alpha * src[r][k]   (r < nrows, k < m).
__global__ void cross_scatter_add_cols_kernel(double* __restrict__ dst, long ldd, const double* __restrict__ src,
                                              long lds, long nrows, double alpha, Cross X) {
  const long m = X.m(), total = nrows * m;
  for (long x = blockIdx.x * (long)blockDim.x + threadIdx.x; x < total; x += (long)gridDim.x * blockDim.x) {
    const long r = x / m, k = x - r * m;
    dst[r * ldd + cross_row(X, k)] += alpha * src[r * lds + k];
  }
}

// dst[cross_row(k1)][cross_row(k2)] += alpha * src[k1][k2].
__global__ void cross_scatter_add_block_kernel(double* __restrict__ dst, long ldd, const double* __restrict__ src,
                                               long lds, double alpha, Cross X) {
  const long m = X.m(), total = m * m;
  for (long x = blockIdx.x * (long)blockDim.x + threadIdx.x; x < total; x += (long)gridDim.x * blockDim.x) {
    const long k1 = x / m, k2 = x - k1 * m;
    dst[cross_row(X, k1) * ldd + cross_row(X, k2)] += alpha * src[k1 * lds + k2];
  }
}

// dst[k][c] = Y[cross_row(k)][c] - [cross_row(k) == hp] T[hp][hp] K[hp][c]  (square ld x ld operands,
// hp = h * nv + pa): the cross rows of (T with its corner entry removed) K, from Y = T K.
__global__ void cross_rows_without_corner_kernel(double* __restrict__ dst, long ldd, const double* __restrict__ Y,
                                                 const double* __restrict__ T, const double* __restrict__ K, long ld,
                                                 Cross X) {
  const long m = X.m(), total = m * ld, hp = (long)X.h * X.nv + X.pa;
  const double thp = T[hp * ld + hp];
  for (long x = blockIdx.x * (long)blockDim.x + threadIdx.x; x < total; x += (long)gridDim.x * blockDim.x) {
    const long k = x / ld, c = x - k * ld;
    const long r = cross_row(X, k);
    dst[k * ldd + c] = Y[r * ld + c] - (r == hp ? thp * K[hp * ld + c] : 0.0);
  }
}

// EM[ij][a][b] += tc[ij][v + q(a)] * A[b][pa] for a != pa (q(a) = a - [a > pa]): the part of
// sum_c t^M_ij^ac A[b][c] from the entries (a, pa) of rows ij outside the occupied cross, which
// tc holds (compact vv-cross columns, rows of the occupied cross zero).
__global__ void em_cross_column_kernel(double* __restrict__ em, const double* __restrict__ tc, long ldt,
                                       const double* __restrict__ A, int o, int v, int pa) {
  const long vv = (long)v * v, total = (long)o * o * vv;
  for (long x = blockIdx.x * (long)blockDim.x + threadIdx.x; x < total; x += (long)gridDim.x * blockDim.x) {
    const long ij = x / vv, ab = x - ij * vv;
    const int a = (int)(ab / v), b = (int)(ab % v);
    if (a == pa) continue;
    em[x] += tc[ij * ldt + v + (a < pa ? a : a - 1)] * A[(long)b * v + pa];
  }
}

// dst[i][j][a][b] = src[i][j][a][b] where the index set holds h (in i, j) or pa (in a, b) and is
// not all primary (the mixed doubles), else 0.
__global__ void mixed_doubles_kernel(double* __restrict__ dst, const double* __restrict__ src, int o, int v, int h,
                                     int pa) {
  const long vv = (long)v * v, total = (long)o * o * vv;
  for (long x = blockIdx.x * (long)blockDim.x + threadIdx.x; x < total; x += (long)gridDim.x * blockDim.x) {
    const long ij = x / vv, ab = x - ij * vv;
    const int i = (int)(ij / o), j = (int)(ij % o), a = (int)(ab / v), b = (int)(ab % v);
    const bool any = i == h || j == h || a == pa || b == pa;
    const bool all = i == h && j == h && a == pa && b == pa;
    dst[x] = (any && !all) ? src[x] : 0.0;
  }
}

// e0 = sum_{i<o} (h[i * hs] + f[i * fs]): one workgroup, fixed-order tree sum (o <= 256 per thread pass).
__global__ __launch_bounds__(kThreads) void reference_energy_kernel(double* e0, const double* h, long hs,
                                                                   const double* f, long fs, int o) {
  __shared__ double red[kThreads];
  double acc = 0.0;
  for (int i = threadIdx.x; i < o; i += kThreads) acc += h[(long)i * hs] + f[(long)i * fs];
  red[threadIdx.x] = acc;
  __syncthreads();
  for (int w = kThreads / 2; w > 0; w >>= 1) {
    if (threadIdx.x < w) red[threadIdx.x] += red[threadIdx.x + w];
    __syncthreads();
  }
  if (threadIdx.x == 0) e0[0] = red[0];
}

hipError_t reference_energy(double* e0, const double* h, long hs, long hlen, const double* f, long fs, long flen,
                            int o, hipStream_t s) {
  if (o < 1 || hs < 0 || fs < 0) return hipErrorInvalidValue;
  if (bounds_checking() && !(range_ok(e0, 0, 0, 8, "reference energy e0") &&
                             range_ok(h, 0, hlen - 1, 8, "reference energy h") && (o - 1) * hs < hlen &&
                             range_ok(f, 0, flen - 1, 8, "reference energy f") && (o - 1) * fs < flen))
    return hipErrorInvalidValue;
  if (dry_run()) return hipSuccess;
  hipLaunchKernelGGL(reference_energy_kernel, dim3(1), dim3(kThreads), 0, s, e0, h, hs, f, fs, o);
  return hipGetLastError();
}

namespace {
bool cross_ok(const Cross& X) { return X.no >= 1 && X.nv >= 1 && X.h >= 0 && X.h < X.no && X.pa >= 0 && X.pa < X.nv; }
unsigned ew_grid(long total) { return (unsigned)std::max<long>(1, std::min<long>((total + 255) / 256, 8192)); }
}  // namespace

hipError_t cross_gather_rows(double* dst, long ldd, const double* src, long lds, long src_rows, long ncols,
                             const Cross& X, bool zero_diag, hipStream_t s) {
  const long m = X.m();
  if (!cross_ok(X) || src_rows < X.n() || ncols < 1 || ncols > lds || ncols > ldd) return hipErrorInvalidValue;
  if (bounds_checking() && !(range_ok(dst, 0, (m - 1) * ldd + ncols - 1, 8, "cross gather rows dst") &&
                             range_ok(src, 0, (src_rows - 1) * lds + ncols - 1, 8, "cross gather rows src")))
    return hipErrorInvalidValue;
  if (dry_run()) return hipSuccess;
  hipLaunchKernelGGL(cross_gather_rows_kernel, dim3(ew_grid(m * ncols)), dim3(256), 0, s, dst, ldd, src, lds, ncols, X,
                     zero_diag ? 1 : 0);
  return hipGetLastError();
}

hipError_t cross_gather_cols(double* dst, long ldd, const double* src, long lds, long nrows, const Cross& X,
                             const Cross* zero_rows, hipStream_t s) {
  const long m = X.m();
  if (!cross_ok(X) || lds < X.n() || nrows < 1 || ldd < m || (zero_rows && (!cross_ok(*zero_rows) || zero_rows->n() < nrows)))
    return hipErrorInvalidValue;
  if (bounds_checking() && !(range_ok(dst, 0, nrows * ldd - 1, 8, "cross gather cols dst") &&
                             range_ok(src, 0, (nrows - 1) * lds + X.n() - 1, 8, "cross gather cols src")))
    return hipErrorInvalidValue;
  if (dry_run()) return hipSuccess;
  const Cross R = zero_rows ? *zero_rows : X;
  hipLaunchKernelGGL(cross_gather_cols_kernel, dim3(ew_grid(nrows * ldd)), dim3(256), 0, s, dst, ldd, src, lds, nrows, X,
                     R, zero_rows ? 1 : 0);
  return hipGetLastError();
}

hipError_t cross_scatter_add_rows(double* dst, long ldd, long dst_rows, const double* src, long lds, long ncols,
                                  double alpha, const Cross& X, hipStream_t s) {
  const long m = X.m();
  if (!cross_ok(X) || dst_rows < X.n() || ncols < 1 || ncols > ldd || ncols > lds) return hipErrorInvalidValue;
  if (bounds_checking() && !(range_ok(dst, 0, (dst_rows - 1) * ldd + ncols - 1, 8, "cross scatter rows dst") &&
                             range_ok(src, 0, (m - 1) * lds + ncols - 1, 8, "cross scatter rows src")))
    return hipErrorInvalidValue;
  if (dry_run()) return hipSuccess;
  hipLaunchKernelGGL(cross_scatter_add_rows_kernel, dim3(ew_grid(m * ncols)), dim3(256), 0, s, dst, ldd, src, lds, ncols,
                     alpha, X);
  return hipGetLastError();
}

hipError_t cross_scatter_add_cols(double* dst, long ldd, long nrows, const double* src, long lds, double alpha,
                                  const Cross& X, hipStream_t s) {
  const long m = X.m();
  if (!cross_ok(X) || ldd < X.n() || nrows < 1 || lds < m) return hipErrorInvalidValue;
  if (bounds_checking() && !(range_ok(dst, 0, (nrows - 1) * ldd + X.n() - 1, 8, "cross scatter cols dst") &&
                             range_ok(src, 0, (nrows - 1) * lds + m - 1, 8, "cross scatter cols src")))
    return hipErrorInvalidValue;
  if (dry_run()) return hipSuccess;
  hipLaunchKernelGGL(cross_scatter_add_cols_kernel, dim3(ew_grid(nrows * m)), dim3(256), 0, s, dst, ldd, src, lds, nrows,
                     alpha, X);
  return hipGetLastError();
}

hipError_t cross_scatter_add_block(double* dst, long ldd, const double* src, long lds, double alpha, const Cross& X,
                                   hipStream_t s) {
  const long m = X.m();
  if (!cross_ok(X) || ldd < X.n() || lds < m) return hipErrorInvalidValue;
  if (bounds_checking() && !(range_ok(dst, 0, (X.n() - 1) * ldd + X.n() - 1, 8, "cross scatter block dst") &&
                             range_ok(src, 0, (m - 1) * lds + m - 1, 8, "cross scatter block src")))
    return hipErrorInvalidValue;
  if (dry_run()) return hipSuccess;
  hipLaunchKernelGGL(cross_scatter_add_block_kernel, dim3(ew_grid(m * m)), dim3(256), 0, s, dst, ldd, src, lds, alpha, X);
  return hipGetLastError();
}

hipError_t cross_rows_without_corner(double* dst, long ldd, const double* Y, const double* T, const double* K,
                                     const Cross& X, hipStream_t s) {
  const long m = X.m(), ld = X.n();
  if (!cross_ok(X) || ldd < ld) return hipErrorInvalidValue;
  if (bounds_checking() && !(range_ok(dst, 0, (m - 1) * ldd + ld - 1, 8, "cross rows dst") &&
                             range_ok(Y, 0, ld * ld - 1, 8, "cross rows Y") && range_ok(T, 0, ld * ld - 1, 8, "cross rows T") &&
                             range_ok(K, 0, ld * ld - 1, 8, "cross rows K")))
    return hipErrorInvalidValue;
  if (dry_run()) return hipSuccess;
  hipLaunchKernelGGL(cross_rows_without_corner_kernel, dim3(ew_grid(m * ld)), dim3(256), 0, s, dst, ldd, Y, T, K, ld, X);
  return hipGetLastError();
}

hipError_t em_cross_column(double* em, const double* tc, long ldt, const double* A, int o, int v, int pa,
                           hipStream_t s) {
  const long total = (long)o * o * v * v, mv = 2L * v - 1;
  if (o < 1 || v < 1 || pa < 0 || pa >= v || ldt < mv) return hipErrorInvalidValue;
  if (bounds_checking() && !(range_ok(em, 0, total - 1, 8, "EM cross column em") &&
                             range_ok(tc, 0, ((long)o * o - 1) * ldt + mv - 1, 8, "EM cross column t") &&
                             range_ok(A, 0, (long)v * v - 1, 8, "EM cross column A")))
    return hipErrorInvalidValue;
  if (dry_run()) return hipSuccess;
  hipLaunchKernelGGL(em_cross_column_kernel, dim3(ew_grid(total)), dim3(256), 0, s, em, tc, ldt, A, o, v, pa);
  return hipGetLastError();
}

hipError_t mixed_doubles(double* dst, const double* src, int o, int v, int h, int pa, hipStream_t s) {
  const long total = (long)o * o * v * v;
  if (o < 1 || v < 1 || h < 0 || h >= o || pa < 0 || pa >= v) return hipErrorInvalidValue;
  if (bounds_checking() && !(range_ok(dst, 0, total - 1, 8, "mixed doubles dst") &&
                             range_ok(src, 0, total - 1, 8, "mixed doubles src")))
    return hipErrorInvalidValue;
  if (dry_run()) return hipSuccess;
  hipLaunchKernelGGL(mixed_doubles_kernel, dim3(ew_grid(total)), dim3(256), 0, s, dst, src, o, v, h, pa);
  return hipGetLastError();
}

hipError_t diag_trace(double* J, const double* Bh, int naux, int n, int no, hipStream_t s) {
  if (bounds_checking() && !(range_ok(J, 0, naux - 1, 8, "trace J") &&
                             range_ok(Bh, 0, (long)naux * n * n - 1, 8, "trace B")))
    return hipErrorInvalidValue;
  if (dry_run()) return hipSuccess;
  hipLaunchKernelGGL(diag_trace_kernel, dim3((naux + 255) / 256), dim3(256), 0, s, J, Bh, naux, n, no);
  return hipGetLastError();
}

hipError_t energy(double* e, double* partial, const double* t1, const double* t2, const double* Lijab,
                  const double* fov, int no, int nv, hipStream_t s) {
  const long total = (long)no * no * nv * nv;
  if (bounds_checking() &&
      !(range_ok(e, 0, 0, 8, "energy e") && range_ok(partial, 0, kRedBlocks - 1, 8, "energy partial") &&
        range_ok(t1, 0, (long)no * nv - 1, 8, "energy t1") && range_ok(t2, 0, total - 1, 8, "energy t2") &&
        range_ok(Lijab, 0, total - 1, 8, "energy L") && range_ok(fov, 0, (long)no * nv - 1, 8, "energy fov")))
    return hipErrorInvalidValue;
  if (dry_run()) return hipSuccess;
  hipLaunchKernelGGL(energy_stage1, dim3(kRedBlocks), dim3(kThreads), 0, s, partial, t1, t2, Lijab, no, nv, total);
  hipLaunchKernelGGL(energy_stage2, dim3(1), dim3(kThreads), 0, s, e, partial, kRedBlocks, t1, fov, no * nv);
  return hipGetLastError();
}


static bool chk(const void* p, long n, const char* what) { return range_ok(p, 0, n - 1, 8, what); }

hipError_t pack_tpm(double* tplus, double* tminus, const double* t2, int o, int v, double dscale, hipStream_t s) {
  const long To = (long)o * (o + 1) / 2, Tv = (long)v * (v + 1) / 2, vv = (long)v * v;
  if (bounds_checking() && !(chk(tplus, To * Tv, "pack_tpm plus") && chk(tminus, To * Tv, "pack_tpm minus") &&
                             chk(t2, (long)o * o * vv, "pack_tpm t2")))
    return hipErrorInvalidValue;
  if (dry_run()) return hipSuccess;
  dim3 grid((unsigned)std::min<long>((vv + kThreads - 1) / kThreads, 64), o * o);
  hipLaunchKernelGGL(pack_tpm_kernel, grid, dim3(kThreads), 0, s, tplus, tminus, t2, o, v, dscale);
  return hipGetLastError();
}

hipError_t unpack_rpm(double* RL, const double* Rplus, const double* Rminus, int o, int v, hipStream_t s) {
  const long To = (long)o * (o + 1) / 2, Tv = (long)v * (v + 1) / 2, vv = (long)v * v;
  if (bounds_checking() && !(chk(RL, (long)o * o * vv, "unpack_rpm RL") && chk(Rplus, To * Tv, "unpack_rpm plus") &&
                             chk(Rminus, To * Tv, "unpack_rpm minus")))
    return hipErrorInvalidValue;
  if (dry_run()) return hipSuccess;
  const int nblk = (v + 31) / 32;
  dim3 grid((unsigned)(nblk * (nblk + 1) / 2), (unsigned)To);
  hipLaunchKernelGGL(unpack_rpm_kernel, grid, dim3(kThreads), 0, s, RL, Rplus, Rminus, o, v, nblk);
  return hipGetLastError();
}

hipError_t pack_vvvv(double* Vp, const double* W, int a0, int a1, int v, hipStream_t s) {
  const long Tv = (long)v * (v + 1) / 2, vv = (long)v * v;
  if (a1 <= a0) return hipSuccess;
  if (bounds_checking() && !(chk(Vp, 2 * Tv * Tv, "pack_vvvv out") && chk(W, (long)(a1 - a0) * v * vv, "pack_vvvv in")))
    return hipErrorInvalidValue;
  if (dry_run()) return hipSuccess;
  dim3 grid((unsigned)std::min<long>((vv + kThreads - 1) / kThreads, 64), (a1 - a0) * v);
  hipLaunchKernelGGL(pack_vvvv_kernel, grid, dim3(kThreads), 0, s, Vp, W, a0, v);
  return hipGetLastError();
}

hipError_t pair_minus_rows(int* pm, int v, hipStream_t s) {
  const long Tv = (long)v * (v + 1) / 2;
  if (v <= 0) return hipSuccess;
  if (bounds_checking() && !range_ok(pm, 0, Tv - 1, sizeof(int), "pair rows")) return hipErrorInvalidValue;
  if (dry_run()) return hipSuccess;
  hipLaunchKernelGGL(pair_minus_rows_kernel, dim3((v + kThreads - 1) / kThreads), dim3(kThreads), 0, s, pm, v);
  return hipGetLastError();
}

hipError_t pack_full(double* V, const double* W, int a0, int a1, int v, hipStream_t s) {
  const long vv = (long)v * v;
  if (a1 <= a0) return hipSuccess;
  if (bounds_checking() && !(chk(V, vv * vv, "pack_full out") && chk(W, (long)(a1 - a0) * v * vv, "pack_full in")))
    return hipErrorInvalidValue;
  if (dry_run()) return hipSuccess;
  dim3 grid((unsigned)std::min<long>((vv + kThreads - 1) / kThreads, 64), (a1 - a0) * v);
  hipLaunchKernelGGL(pack_full_kernel, grid, dim3(kThreads), 0, s, V, W, a0, v);
  return hipGetLastError();
}

int update_partial_blocks() { return kRedBlocks; }

hipError_t diis_update(const UpdateArgs& u, hipStream_t s) {
  // Whether this call stores a pair is decided by the caller; the device state decides the
  // slot, which stored pairs are valid and the coefficients.
  UK p;
  p.t1 = u.t1;
  p.t2 = u.t2;
  p.r1 = u.r1;
  p.r2 = u.r2;
  p.eps = u.eps;
  p.hist_t = u.hist_t;
  p.hist_e = u.hist_e;
  p.partial = u.partial;
  p.st = u.st;
  p.o = u.no;
  p.v = u.nv;
  p.m = u.m;
  p.start = u.start;
  p.nstat = 3 + kMaxDiis;
  p.len = u.len;
  p.shift = u.shift;
  p.ss = u.nslot > 1 || u.tab ? u.ss : 0;
  p.tab = u.tab;
  const long ov = (long)u.no * u.nv;
  if (u.nslot < 1 || u.nslot > 65535 || (p.ss % 8)) return hipErrorInvalidValue;
  if (bounds_checking()) {
    // every slot the table can name (or every grid row), each checked where it lies
    const long nk = u.tab ? u.tab_max + 1 : u.nslot;
    for (long k = 0; k < (p.ss ? nk : 1); ++k) {
      const long o8 = k * p.ss / 8;  // slot offset in doubles
      auto at = [&](const void* q) { return reinterpret_cast<const char*>(q) + k * p.ss; };
      if (!(range_ok(at(u.t1), 0, ov - 1, 8, "update t1") && range_ok(at(u.t2), 0, u.len - ov - 1, 8, "update t2") &&
            range_ok(at(u.r1), 0, ov - 1, 8, "update r1") && range_ok(at(u.r2), 0, u.len - ov - 1, 8, "update r2") &&
            range_ok(at(u.e), 0, 0, 8, "update e") && range_ok(at(u.eps), 0, u.no + u.nv - 1, 8, "update eps") &&
            range_ok(at(u.hist_t), 0, (long)u.m * u.len - 1, 8, "update hist_t") &&
            range_ok(at(u.hist_e), 0, (long)u.m * u.len - 1, 8, "update hist_e") &&
            range_ok(at(u.partial), 0, (long)kRedBlocks * (3 + kMaxDiis) - 1, 8, "update partial") &&
            range_ok(at(u.st), 0, 0, sizeof(DiisState), "update state") &&
            range_ok(u.stats, 8 * (p.ss ? k : 0), 8 * (p.ss ? k : 0) + 7, 8, "update stats")))
        return hipErrorInvalidValue;
      (void)o8;
    }
  }
  if (u.m < 1 || u.m > kMaxDiis) return hipErrorInvalidValue;
  if (dry_run()) return hipSuccess;
  hipLaunchKernelGGL(update_stage1, dim3(kRedBlocks, u.nslot), dim3(kThreads), 0, s, p);
  hipLaunchKernelGGL(update_stage2, dim3(1, u.nslot), dim3(kThreads), 0, s, u.st, u.partial, kRedBlocks, 3 + kMaxDiis,
                     u.m, u.start, u.e, u.stats, u.shift, p.ss, u.tab);
  hipLaunchKernelGGL(update_stage3, dim3(grid_for(u.len), u.nslot), dim3(kThreads), 0, s, u.t1, u.t2, u.hist_t, u.st,
                     u.m, (long)u.no * u.nv, u.len, p.ss, u.tab);
  return hipGetLastError();
}

}  // namespace ascc
