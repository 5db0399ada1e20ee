// Strided, batched FP64 GEMM on the CDNA4 matrix cores (v_mfma_f64_16x16x4_f64).
//
// C_z(m,n) = alpha * sum_r sum_k A_{z,r}(m,k) B_{z,r}(k,n) + beta * C_z(m,n)
//
// Every contraction of the residual is expressed through this one kernel family: the
// operands are arbitrary strided 2-D views (a permuted slice of T2 or of an integral block
// is just another pair of strides), tiles are staged through LDS, and each wave64 owns a
// (BM/WM) x (BN/WN) block of 16x16 MFMA accumulators.
//
// MFMA f64 16x16x4 lane layout (gfx950, measured): lane l supplies A(l%16, l/16) and
// B(l/16, l%16); accumulator register r of lane l holds C(l/16 + 4r, l%16).
#include "internal.h"

namespace ascc {
namespace {

typedef double d4 __attribute__((ext_vector_type(4)));

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
};

// Workgroup-to-tile map that gives each of the 8 XCDs (workgroups are dispatched to them
// round-robin) one contiguous range of tiles, M-tile fastest, so the workgroups that share a
// B panel run on the same XCD and hit the same L2.
__device__ __forceinline__ void tile_of(int bid, int tiles_m, int total, int& tm, int& tn) {
  const int q = total >> 3, rem = total & 7;
  const int x = bid & 7, local = bid >> 3;
  const int tile = x * q + min(x, rem) + local;
  tm = tile % tiles_m;
  tn = tile / tiles_m;
}

template <int BM, int BN, int BK, int WM, int WN, bool AMF, bool BNF>
__global__ __launch_bounds__(WM* WN * 64) void gemm_f64_kernel(GP p) {
  constexpr int NT = WM * WN * 64;
  constexpr int TM = BM / WM, TN = BN / WN;
  constexpr int FM = TM / 16, FN = TN / 16;
  constexpr int LA = BM * BK / NT, LB = BK * BN / NT;
  constexpr int PA = BM + 1, PB = BN + 1;  // +1 double: conflict-free transposing stores
  static_assert(FM >= 1 && FN >= 1 && LA >= 1 && LB >= 1, "tile config");
  __shared__ double As[BK * PA];
  __shared__ double Bs[BK * PB];

  const int tid = threadIdx.x;
  const int lane = tid & 63, wave = tid >> 6;
  const int wm = wave / WN, wn = wave % WN;

  int tm, tn;
  tile_of(blockIdx.x, p.tiles_m, p.tiles_m * p.tiles_n, tm, tn);
  const int m0 = tm * BM, n0 = tn * BN;
  const int z1 = blockIdx.z, z2 = blockIdx.y;
  const double* Ab = p.A + z1 * p.sa1 + z2 * p.sa2;
  const double* Bb = p.B + z1 * p.sb1 + z2 * p.sb2;
  double* Cb = p.C + z1 * p.sc1 + z2 * p.sc2;

  d4 acc[FM][FN];
#pragma unroll
  for (int i = 0; i < FM; ++i)
#pragma unroll
    for (int j = 0; j < FN; ++j) acc[i][j] = d4{0.0, 0.0, 0.0, 0.0};

  const int nkt = (p.K + BK - 1) / BK;
  const int niter = nkt * p.nred;

  double ra[LA], rb[LB];
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
#pragma unroll
    for (int l = 0; l < LB; ++l) {
      const int e = tid + l * NT;
      const int n = BNF ? (e % BN) : (e / BK);
      const int k = BNF ? (e / BN) : (e % BK);
      const int gn = n0 + n, gk = k0 + k;
      rb[l] = (gn < p.N && gk < p.K) ? Br[gk * p.sbk + gn * p.sbn] : 0.0;
    }
  };
  auto store = [&]() {
#pragma unroll
    for (int l = 0; l < LA; ++l) {
      const int e = tid + l * NT;
      const int m = AMF ? (e % BM) : (e / BK);
      const int k = AMF ? (e / BM) : (e % BK);
      As[k * PA + m] = ra[l];
    }
#pragma unroll
    for (int l = 0; l < LB; ++l) {
      const int e = tid + l * NT;
      const int n = BNF ? (e % BN) : (e / BK);
      const int k = BNF ? (e / BN) : (e % BK);
      Bs[k * PB + n] = rb[l];
    }
  };

  const int lr = lane & 15, lk = lane >> 4;
  if (niter > 0) load(0);
  for (int it = 0; it < niter; ++it) {
    __syncthreads();
    store();
    __syncthreads();
    if (it + 1 < niter) load(it + 1);
#pragma unroll
    for (int kk = 0; kk < BK; kk += 4) {
      double a[FM], b[FN];
#pragma unroll
      for (int i = 0; i < FM; ++i) a[i] = As[(kk + lk) * PA + wm * TM + i * 16 + lr];
#pragma unroll
      for (int j = 0; j < FN; ++j) b[j] = Bs[(kk + lk) * PB + wn * TN + j * 16 + lr];
#pragma unroll
      for (int i = 0; i < FM; ++i)
#pragma unroll
        for (int j = 0; j < FN; ++j) acc[i][j] = __builtin_amdgcn_mfma_f64_16x16x4f64(a[i], b[j], acc[i][j], 0, 0, 0);
    }
  }

  // epilogue: register r of lane l holds C(l/16 + 4r, l%16) of each 16x16 block
#pragma unroll
  for (int i = 0; i < FM; ++i)
#pragma unroll
    for (int j = 0; j < FN; ++j)
#pragma unroll
      for (int r = 0; r < 4; ++r) {
        const int gm = m0 + wm * TM + i * 16 + lk + 4 * r;
        const int gn = n0 + wn * TN + j * 16 + lr;
        if (gm < p.M && gn < p.N) {
          double* c = Cb + gm * p.scm + gn * p.scn;
          const double v = p.alpha * acc[i][j][r];
          *c = (p.beta == 0.0) ? v : v + p.beta * *c;
        }
      }
}

template <int BM, int BN, int BK, int WM, int WN>
hipError_t launch_cfg(const GP& p0, bool amf, bool bnf, int nb1, hipStream_t s) {
  GP p = p0;
  p.tiles_m = (p.M + BM - 1) / BM;
  p.tiles_n = (p.N + BN - 1) / BN;
  dim3 grid(p.tiles_m * p.tiles_n, p.nb2, nb1);
  dim3 block(WM * WN * 64);
  if (amf && bnf)
    hipLaunchKernelGGL((gemm_f64_kernel<BM, BN, BK, WM, WN, true, true>), grid, block, 0, s, p);
  else if (amf)
    hipLaunchKernelGGL((gemm_f64_kernel<BM, BN, BK, WM, WN, true, false>), grid, block, 0, s, p);
  else if (bnf)
    hipLaunchKernelGGL((gemm_f64_kernel<BM, BN, BK, WM, WN, false, true>), grid, block, 0, s, p);
  else
    hipLaunchKernelGGL((gemm_f64_kernel<BM, BN, BK, WM, WN, false, false>), grid, block, 0, s, p);
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
  return range_ok(g.C, lo, hi, sizeof(double), "gemm C");
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
  // Global-load order: an operand whose m (n) stride is 1 is read m-fast (n-fast).
  const bool amf = (g.sam == 1 && g.sak != 1);
  const bool bnf = (g.sbn == 1) || (g.sbk != 1);
  const long tiles128 = (long)((g.M + 127) / 128) * ((g.N + 127) / 128) * nbatch;
  if (g.M >= 96 && g.N >= 96 && tiles128 >= 256) return launch_cfg<128, 128, 16, 2, 2>(p, amf, bnf, g.nb1, s);
  const long tiles64 = (long)((g.M + 63) / 64) * ((g.N + 63) / 64) * nbatch;
  if (g.M >= 48 && g.N >= 48 && tiles64 >= 128) return launch_cfg<64, 64, 16, 2, 2>(p, amf, bnf, g.nb1, s);
  return launch_cfg<32, 32, 16, 1, 1>(p, amf, bnf, g.nb1, s);
}

}  // namespace ascc
