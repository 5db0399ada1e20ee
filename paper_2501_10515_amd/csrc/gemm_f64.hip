// Strided, batched FP64 GEMM on the CDNA4 matrix cores.
//
// C_z(m,n) = alpha * sum_r sum_k A_{z,r}(m,k) B_{z,r}(k,n) + beta * C_z(m,n)
//
// Every contraction of the residual is expressed through this one kernel family: the
// operands are arbitrary strided 2-D views (a permuted slice of T2 or of an integral block
// is just another pair of strides), tiles are staged through LDS, and each wave64 owns a
// (BM/WM) x (BN/WN) block of the output.
//
// The inner product uses v_mfma_f64_4x4x4_f64 (four independent 4x4x4 products per wave64),
// which sustains about 1.6x the FP64 rate of the 16x16x4 form on gfx950 (measured with register
// operands: ~72-75 vs ~45-49 TFLOP/s).  Lane layout (gfx950, measured): lane l belongs to block
// q = (l%16)/4, supplies A_q(l%4, l/16) and B_q(l/16, l%4), and receives D_q(l/16, l%4); the
// CBSZ/ABID broadcast fields have no effect on this instruction, so operands are arranged in
// registers instead (see the main loop).
//
// The particle-particle ladder has its own entry point (gemm_f64_ladder): 256 x 128 tiles when
// the pair dimension fits them, and optionally the symmetric/antisymmetric vvvv combinations
// formed while staging from the stored full (ac|bd) matrix.
#include <algorithm>

#include "internal.h"

namespace ascc {
namespace {


struct GP {
  int M, N, K;
  const double* A;
  long sam, sak, sa1, sa2, sar;
  const double* B;
  long sbk, sbn, sb1, sb2, sbr;
  double* C;
  long scm, scn, sc1, sc2;
  double alpha, beta;
  int nb2, nred;
  int tiles_m, tiles_n;
  int split, it_per_split;  // split-K: slices of the (nred x K-tile) iteration space
  double* part;             // partial tiles [split][nb1*nb2][M][N] when split > 1
  const int* pm;            // pair-combined B (ladder): second row of pair n
};

// Workgroup-to-tile map.  Workgroups are dispatched to the 8 XCDs round-robin; each XCD gets
// one contiguous range of tiles, walked in groups of kGroupM M-tiles (M fastest inside a group)
// so that the workgroups resident on one XCD at a time cover a compact block of C and share
// both A and B panels in that XCD's L2.
constexpr int kGroupM = 8;
__device__ __forceinline__ void tile_of(int bid, int tiles_m, int tiles_n, int& tm, int& tn) {
  const int total = tiles_m * tiles_n;
  const int q = total >> 3, rem = total & 7;
  const int x = bid & 7, local = bid >> 3;
  const int t = x * q + min(x, rem) + local;
  const int per = kGroupM * tiles_n;
  const int g = t / per, first = g * kGroupM;
  const int gs = min(tiles_m - first, kGroupM);
  const int r = t - g * per;
  tm = first + r % gs;
  tn = r / gs;
}

#ifndef ASCC_GEMM_BK
#define ASCC_GEMM_BK 8  // K depth of one LDS stage of the 128x128 tile
#endif
#ifndef ASCC_GEMM_MINBLOCKS
#define ASCC_GEMM_MINBLOCKS 2  // workgroups per CU the 128x128 tile is register-budgeted for
#endif

// PM: B is pair-combined (ladder against the full (ac|bd) in pair order): for batch z2 = 0 (+)
// or 1 (-), B(k, n) = V[n][k] +- V[pm[n]][k] (rows of V at stride sbn).
template <int BM, int BN, int BK, int WM, int WN, bool AMF, bool BNF, bool PM = false>
__global__ __launch_bounds__(WM* WN * 64, (WM * WN >= 8) ? 1 : (WM * WN >= 4) ? ASCC_GEMM_MINBLOCKS : 4) void gemm_f64_kernel(GP p) {
  constexpr int NT = WM * WN * 64;
  constexpr int TM = BM / WM, TN = BN / WN;
  constexpr int RB = TM / 4, CP = TN / 16;
  constexpr int LA = BM * BK / NT, LB = BK * BN / NT;
  constexpr int PA = BM + 1, PB = BN + 1;  // +1 double: conflict-free transposing stores
  static_assert(RB >= 1 && CP >= 1 && LA >= 1 && LB >= 1 && TM % 4 == 0 && TN % 16 == 0, "tile config");
  static_assert(!PM || (!BNF && NT % BK == 0), "pair-combined B is staged k-fast");
  __shared__ double As[2][BK * PA];
  __shared__ double Bs[2][BK * PB];

  const int tid = threadIdx.x;
  const int lane = tid & 63, wave = tid >> 6;
  const int wm = wave / WN, wn = wave % WN;

  int tm, tn;
  const int ntiles = p.tiles_m * p.tiles_n;
  int bid = blockIdx.x, z2 = blockIdx.y;
  if constexpr (PM) {
    // Both halves of a tile read the same V rows: they are dispatched back to back to the same
    // XCD (workgroups b and b + 8 share an XCD), so the second one finds them in L2.
    const int x = bid & 7, local = bid >> 3;
    z2 = local & 1;
    bid = ((local >> 1) << 3) | x;
    if (bid >= ntiles) return;  // padding of the grid to whole groups of 8
  }
  const int slice = bid / ntiles;
  tile_of(bid - slice * ntiles, p.tiles_m, p.tiles_n, tm, tn);
  const int m0 = tm * BM, n0 = tn * BN;
  const int z1 = blockIdx.z;
  const double* Ab = p.A + z1 * p.sa1 + z2 * p.sa2;
  const double* Bb = p.B + z1 * p.sb1 + z2 * p.sb2;
  double* Cb = p.C + z1 * p.sc1 + z2 * p.sc2;

  // acc[x][y]: lane l holds C(4x + l/16, 16y + l%16) of the wave's tile (x: 4-row block,
  // y: 16-column panel)
  double acc[RB][CP];
#pragma unroll
  for (int x = 0; x < RB; ++x)
#pragma unroll
    for (int y = 0; y < CP; ++y) acc[x][y] = 0.0;

  const int nkt = (p.K + BK - 1) / BK;
  const int it_begin = slice * p.it_per_split;
  const int it_end = min(nkt * p.nred, it_begin + p.it_per_split);

  double ra[LA], rb[LB];
  // pair-combined B: the two V rows of each staged pair n are fixed for the whole K loop
  const double* pva[PM ? LB : 1];
  const double* pvb[PM ? LB : 1];
  if constexpr (PM) {
#pragma unroll
    for (int l = 0; l < LB; ++l) {
      const int gn = n0 + (tid + l * NT) / BK;
      pva[l] = gn < p.N ? Bb + (long)gn * p.sbn : nullptr;
      pvb[l] = gn < p.N ? Bb + (long)p.pm[gn] * p.sbn : nullptr;
    }
  }
  const bool minus = PM && z2 == 1;
  auto load = [&](int it) {
    const int r = it / nkt, k0 = (it % nkt) * BK;
    const double* Ar = Ab + r * p.sar;
    const double* Br = Bb + r * p.sbr;
#pragma unroll
    for (int l = 0; l < LA; ++l) {
      const int e = tid + l * NT;
      const int m = AMF ? (e % BM) : (e / BK);
      const int k = AMF ? (e / BM) : (e % BK);
      const int gm = m0 + m, gk = k0 + k;
      ra[l] = (gm < p.M && gk < p.K) ? Ar[gm * p.sam + gk * p.sak] : 0.0;
    }
    if constexpr (PM) {
      const int gk = k0 + tid % BK;  // the same k for every element this thread stages
#pragma unroll
      for (int l = 0; l < LB; ++l) {
        double x = 0.0;
        if (pva[l] && gk < p.K) {
          const double u = pva[l][gk], w = pvb[l][gk];
          x = minus ? u - w : u + w;
        }
        rb[l] = x;
      }
      (void)Br;
    } else {
#pragma unroll
      for (int l = 0; l < LB; ++l) {
        const int e = tid + l * NT;
        const int n = BNF ? (e % BN) : (e / BK);
        const int k = BNF ? (e / BN) : (e % BK);
        const int gn = n0 + n, gk = k0 + k;
        rb[l] = (gn < p.N && gk < p.K) ? Br[gk * p.sbk + gn * p.sbn] : 0.0;
      }
    }
  };
  auto store = [&](int buf) {
#pragma unroll
    for (int l = 0; l < LA; ++l) {
      const int e = tid + l * NT;
      const int m = AMF ? (e % BM) : (e / BK);
      const int k = AMF ? (e / BM) : (e % BK);
      As[buf][k * PA + m] = ra[l];
    }
#pragma unroll
    for (int l = 0; l < LB; ++l) {
      const int e = tid + l * NT;
      const int n = BNF ? (e % BN) : (e / BK);
      const int k = BNF ? (e / BN) : (e % BK);
      Bs[buf][k * PB + n] = rb[l];
    }
  };

  // Operands of v_mfma_f64_4x4x4 (block q = (l%16)/4 of lane l; A_q(l%4, l/16), B_q(l/16, l%4)):
  // the A register of 4-row block x carries the same four rows in all four blocks (each group of
  // 16 lanes reads 4 distinct LDS words), the B register of panel y gives block q the columns
  // 16y + 4q .. 16y + 4q + 3, so one instruction yields C(4x .. 4x+3, 16y .. 16y+15).
  const int fk = lane >> 4, fa = lane & 3, fb = lane & 15;
  if (it_begin < it_end) {
    load(it_begin);
    store(0);
  }
  __syncthreads();
  for (int it = it_begin; it < it_end; ++it) {
    const int cur = (it - it_begin) & 1;
    if (it + 1 < it_end) load(it + 1);
    const double* as = As[cur] + fk * PA + wm * TM + fa;
    const double* bs = Bs[cur] + fk * PB + wn * TN + fb;
#pragma unroll
    for (int kk = 0; kk < BK; kk += 4) {
      double b[CP];
#pragma unroll
      for (int y = 0; y < CP; ++y) b[y] = bs[kk * PB + 16 * y];
#pragma unroll
      for (int x = 0; x < RB; ++x) {
        const double a = as[kk * PA + 4 * x];
#pragma unroll
        for (int y = 0; y < CP; ++y) acc[x][y] = __builtin_amdgcn_mfma_f64_4x4x4f64(a, b[y], acc[x][y], 0, 0, 0);
      }
    }
    if (it + 1 < it_end) store(cur ^ 1);
    __syncthreads();
  }

  // epilogue
#pragma unroll
  for (int x = 0; x < RB; ++x)
#pragma unroll
    for (int y = 0; y < CP; ++y) {
      const int gm = m0 + wm * TM + 4 * x + fk;
      const int gn = n0 + wn * TN + 16 * y + fb;
      if (gm < p.M && gn < p.N) {
        const double v = p.alpha * acc[x][y];
        if (p.split > 1) {
          const long zl = (long)z1 * gridDim.y + z2;
          p.part[(((long)slice * gridDim.z * gridDim.y + zl) * p.M + gm) * p.N + gn] = v;
        } else {
          double* c = Cb + gm * p.scm + gn * p.scn;
          *c = (p.beta == 0.0) ? v : v + p.beta * *c;
        }
      }
    }
}

// C_z(m,n) = beta * C_z(m,n) + sum_s part[s][z][m][n], summed in slice order.
__global__ __launch_bounds__(256) void splitk_reduce(GP p, int nb1, long total) {
  for (long x = blockIdx.x * 256L + threadIdx.x; x < total; x += (long)gridDim.x * 256) {
    const long mn = (long)p.M * p.N;
    const long zl = x / mn, r = x % mn;
    const int gm = r / p.N, gn = r % p.N;
    const int z1 = zl / p.nb2, z2 = zl % p.nb2;
    double acc = 0.0;
    for (int sl = 0; sl < p.split; ++sl) acc += p.part[(long)sl * total + x];
    double* c = p.C + z1 * p.sc1 + z2 * p.sc2 + gm * p.scm + gn * p.scn;
    *c = (p.beta == 0.0) ? acc : acc + p.beta * *c;
  }
}

template <int BM, int BN, int BK, int WM, int WN>
hipError_t launch_cfg(const GP& p0, bool amf, bool bnf, int nb1, double* ws, long ws_elems, hipStream_t s) {
  GP p = p0;
  p.tiles_m = (p.M + BM - 1) / BM;
  p.tiles_n = (p.N + BN - 1) / BN;
  const long tiles = (long)p.tiles_m * p.tiles_n * p.nb2 * nb1;
  const int nit = ((p.K + BK - 1) / BK) * p.nred;
  p.split = 1;
  p.it_per_split = nit;
  p.part = nullptr;
  const long outs = (long)p.M * p.N * p.nb2 * nb1;
  if (ws && tiles < 192 && nit >= 16) {
    int sp = (int)std::min<long>({(512 + tiles - 1) / tiles, (long)nit / 8, 256L});
    if (ws_elems > 0) sp = (int)std::min<long>(sp, ws_elems / std::max<long>(outs, 1));
    if (sp > 1) {
      p.it_per_split = (nit + sp - 1) / sp;
      p.split = (nit + p.it_per_split - 1) / p.it_per_split;
      p.part = ws;
    }
  }
  dim3 grid(p.tiles_m * p.tiles_n * p.split, p.nb2, nb1);
  dim3 block(WM * WN * 64);
  if (amf && bnf)
    hipLaunchKernelGGL((gemm_f64_kernel<BM, BN, BK, WM, WN, true, true>), grid, block, 0, s, p);
  else if (amf)
    hipLaunchKernelGGL((gemm_f64_kernel<BM, BN, BK, WM, WN, true, false>), grid, block, 0, s, p);
  else if (bnf)
    hipLaunchKernelGGL((gemm_f64_kernel<BM, BN, BK, WM, WN, false, true>), grid, block, 0, s, p);
  else
    hipLaunchKernelGGL((gemm_f64_kernel<BM, BN, BK, WM, WN, false, false>), grid, block, 0, s, p);
  if (p.split > 1) {
    const long blocks = std::min<long>((outs + 255) / 256, 4096);
    hipLaunchKernelGGL(splitk_reduce, dim3((unsigned)blocks), dim3(256), 0, s, p, nb1, outs);
  }
  return hipGetLastError();
}

// Ladder: both halves (grid.y = 2), no split-K, A/B staged k-fast.
template <int BM, int WM>
hipError_t launch_ladder(GP p, bool pm, hipStream_t s) {
  p.tiles_m = (p.M + BM - 1) / BM;
  p.tiles_n = (p.N + 127) / 128;
  p.split = 1;
  p.it_per_split = (p.K + ASCC_GEMM_BK - 1) / ASCC_GEMM_BK;
  p.part = nullptr;
  const int tiles = p.tiles_m * p.tiles_n;
  // pair-combined: the two halves interleave in grid.x (see the kernel), padded to groups of 8
  dim3 grid(pm ? 2 * ((tiles + 7) / 8 * 8) : tiles, pm ? 1 : 2, 1), block(WM * 2 * 64);
  if (pm)
    hipLaunchKernelGGL((gemm_f64_kernel<BM, 128, ASCC_GEMM_BK, WM, 2, false, false, true>), grid, block, 0, s, p);
  else
    hipLaunchKernelGGL((gemm_f64_kernel<BM, 128, ASCC_GEMM_BK, WM, 2, false, false, false>), grid, block, 0, s, p);
  return hipGetLastError();
}

}  // namespace

Gemm gemm_rm(int M, int N, int K, double alpha, const double* A, long lda, bool ta, const double* B, long ldb,
             bool tb, double beta, double* C, long ldc) {
  Gemm g;
  g.M = M;
  g.N = N;
  g.K = K;
  g.alpha = alpha;
  g.beta = beta;
  g.A = A;
  if (!ta) {
    g.sam = lda;
    g.sak = 1;
  } else {
    g.sam = 1;
    g.sak = lda;
  }
  g.B = B;
  if (!tb) {
    g.sbk = ldb;
    g.sbn = 1;
  } else {
    g.sbk = 1;
    g.sbn = ldb;
  }
  g.C = C;
  g.scm = ldc;
  g.scn = 1;
  return g;
}

// Lowest and highest element offset of an affine index expression sum_t i_t * s_t, 0 <= i_t < e_t.
static void affine_range(const long* ext, const long* str, int n, long& lo, long& hi) {
  lo = hi = 0;
  for (int t = 0; t < n; ++t) {
    const long d = (ext[t] - 1) * str[t];
    if (d < 0) lo += d; else hi += d;
  }
}

static bool gemm_in_bounds(const Gemm& g) {
  long lo, hi;
  const long ea[5] = {g.M, g.K, g.nb1, g.nb2, g.nred}, sa[5] = {g.sam, g.sak, g.sa1, g.sa2, g.sar};
  affine_range(ea, sa, 5, lo, hi);
  if (!range_ok(g.A, lo, hi, sizeof(double), "gemm A")) return false;
  const long eb[5] = {g.K, g.N, g.nb1, g.nb2, g.nred}, sb[5] = {g.sbk, g.sbn, g.sb1, g.sb2, g.sbr};
  affine_range(eb, sb, 5, lo, hi);
  if (!range_ok(g.B, lo, hi, sizeof(double), "gemm B")) return false;
  const long ec[4] = {g.M, g.N, g.nb1, g.nb2}, sc[4] = {g.scm, g.scn, g.sc1, g.sc2};
  affine_range(ec, sc, 4, lo, hi);
  if (!range_ok(g.C, lo, hi, sizeof(double), "gemm C")) return false;
  return !g.ws || range_ok(g.ws, 0, g.ws_elems - 1, sizeof(double), "gemm split-K scratch");
}

hipError_t gemm_f64(const Gemm& g, hipStream_t s) {
  if (g.M <= 0 || g.N <= 0 || g.nb1 <= 0 || g.nb2 <= 0) return hipSuccess;
  if (bounds_checking() && !gemm_in_bounds(g)) return hipErrorInvalidValue;
  if (dry_run()) return hipSuccess;
  if (g.nb1 > 65535 || g.nb2 > 65535) return hipErrorInvalidValue;
  const int nbatch = g.nb1 * g.nb2;
  if (g.K <= 0 || g.nred <= 0) return hipErrorInvalidValue;  // callers never pass an empty contraction
  GP p;
  p.M = g.M;
  p.N = g.N;
  p.K = g.K;
  p.A = g.A;
  p.sam = g.sam;
  p.sak = g.sak;
  p.sa1 = g.sa1;
  p.sa2 = g.sa2;
  p.sar = g.sar;
  p.B = g.B;
  p.sbk = g.sbk;
  p.sbn = g.sbn;
  p.sb1 = g.sb1;
  p.sb2 = g.sb2;
  p.sbr = g.sbr;
  p.C = g.C;
  p.scm = g.scm;
  p.scn = g.scn;
  p.sc1 = g.sc1;
  p.sc2 = g.sc2;
  p.alpha = g.alpha;
  p.beta = g.beta;
  p.nb2 = g.nb2;
  p.nred = g.nred;
  p.pm = nullptr;
  // Global-load order: an operand whose m (n) stride is 1 is read m-fast (n-fast).
  const bool amf = (g.sam == 1 && g.sak != 1);
  const bool bnf = (g.sbn == 1) || (g.sbk != 1);
  const long tiles128 = (long)((g.M + 127) / 128) * ((g.N + 127) / 128) * nbatch;
  // 128 x 128 tiles when they fill the chip, or when a long K lets split-K make up the count
  const bool long_k = g.ws && (long)g.K * g.nred >= 8192 && tiles128 >= 64;
  if (g.M >= 96 && g.N >= 96 && (tiles128 >= 256 || long_k))
    return launch_cfg<128, 128, ASCC_GEMM_BK, 2, 2>(p, amf, bnf, g.nb1, g.ws, g.ws_elems, s);
  const long tiles64 = (long)((g.M + 63) / 64) * ((g.N + 63) / 64) * nbatch;
  if (g.M >= 48 && g.N >= 48 && tiles64 >= 128) return launch_cfg<64, 64, 16, 2, 2>(p, amf, bnf, g.nb1, g.ws, g.ws_elems, s);
  return launch_cfg<32, 32, 16, 1, 1>(p, amf, bnf, g.nb1, g.ws, g.ws_elems, s);
}

hipError_t gemm_f64_ladder(int M, int Tv, const double* A, const double* V, long ldv, long vrows, const int* pm,
                           double* C, hipStream_t s) {
  if (M <= 0 || Tv <= 0) return hipSuccess;
  const bool pmode = pm != nullptr;
  if (pmode && (ldv < Tv || vrows < Tv)) return hipErrorInvalidValue;
  const long half = (long)M * Tv;
  if (bounds_checking()) {
    const long vlast = pmode ? (vrows - 1) * ldv + Tv - 1 : 2L * Tv * Tv - 1;
    if (!(range_ok(A, 0, 2 * half - 1, sizeof(double), "ladder A") && range_ok(C, 0, 2 * half - 1, sizeof(double), "ladder C") &&
          range_ok(V, 0, vlast, sizeof(double), "ladder V") &&
          (!pmode || range_ok(pm, 0, Tv - 1, sizeof(int), "ladder pair rows"))))
      return hipErrorInvalidValue;
  }
  if (dry_run()) return hipSuccess;
  GP p{};
  p.M = M;
  p.N = Tv;
  p.K = Tv;
  p.A = A;
  p.sam = Tv;
  p.sak = 1;
  p.sa2 = half;
  p.B = V;
  p.sbk = 1;
  p.sbn = pmode ? ldv : Tv;
  p.sb2 = pmode ? 0 : (long)Tv * Tv;
  p.C = C;
  p.scm = Tv;
  p.scn = 1;
  p.sc2 = half;
  p.alpha = 1.0;
  p.beta = 0.0;
  p.nb2 = 2;
  p.nred = 1;
  p.pm = pm;
  // 256-row tiles read the vvvv operand once per 256 pair rows; take them unless their row
  // padding costs more than the 128-row tiles' second pass
  const long pad256 = (M + 255L) / 256 * 256, pad128 = (M + 127L) / 128 * 128;
  if (pad256 * 19 <= pad128 * 20) return launch_ladder<256, 4>(p, pmode, s);
  return launch_ladder<128, 2>(p, pmode, s);
}

}  // namespace ascc
