// Strided, batched FP64 GEMM on the CDNA4 matrix cores.
//
// C_z(m,n) = alpha * sum_r sum_k A_{z,r}(m,k) B_{z,r}(k,n) + beta * C_z(m,n)
//
// Every contraction of the residual is expressed through this one kernel family: the
// operands are arbitrary strided 2-D views (a permuted slice of T2 or of an integral block
// is just another pair of strides), tiles are staged through LDS, and each wave64 owns a
// (BM/WM) x (BN/WN) block of the output.
//
// The inner product uses v_mfma_f64_16x16x4_f64.  With register operands the 4x4x4 form issues
// more FP64 work per cycle on gfx950, but fed from LDS the 16x16x4 form wins (3-8% on the
// residual's shapes, measured): a 64 x 64 wave tile needs 16 instructions and 8 LDS reads per
// K-step of 4 instead of 64 and 20.  Lane layout (measured): lane l supplies A(l%16, l/16) and
// B(l/16, l%16); register r of the result holds D(l/16 + 4r, l%16).
//
// Tile configurations: 128 x 128 (4 waves, two workgroups per CU), 256 x 128 and 192 x 192
// (8 waves, one per CU), all with K staged 16 deep, chosen per call by how well whole rounds of 256 workgroups cover
// the output; 64 x 64 and 32 x 32 for small outputs; 128 x 128 with split-K when a long K meets
// too few tiles.  The particle-particle ladder has its own entry point (gemm_f64_ladder): 256-,
// 224-, 208- or 128-row tiles, whichever pads the pair dimension least, and optionally the
// symmetric/antisymmetric vvvv combinations formed while staging from the stored full (ac|bd).
#include <algorithm>
#include <cstdint>

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
  const int* tab1;          // batch level 1: operand block of grid index z1 (nullptr: z1 itself)
  int lower;                // symmetric C: tiles on and below the diagonal only (tiles_m == tiles_n)
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

// The lower-triangle tiles (tn <= tm) of a symmetric product, each XCD a contiguous range of them
// in row order (consecutive tiles share their A rows).
__device__ __forceinline__ void tile_of_lower(int bid, int tiles, int& tm, int& tn) {
  const int total = tiles * (tiles + 1) / 2;
  const int q = total >> 3, rem = total & 7;
  const int x = bid & 7, local = bid >> 3;
  const int t = x * q + min(x, rem) + local;
  int m = (int)((sqrtf(8.f * (float)t + 1.f) - 1.f) * 0.5f);
  while ((m + 1) * (m + 2) / 2 <= t) ++m;
  while (m * (m + 1) / 2 > t) --m;
  tm = m;
  tn = t - m * (m + 1) / 2;
}

// C_z(r, c) = C_z(c, r) for c > r: the strict upper triangle of a symmetric product copied from
// its lower one through a 32 x 32 LDS tile (coalesced reads and writes).  grid.x enumerates the
// 32 x 32 blocks on and above the diagonal, grid.y / grid.z the batch levels.
__global__ __launch_bounds__(256) void mirror_upper_kernel(GP p) {
  __shared__ double tile[32][33];
  const int nb = (p.M + 31) / 32;
  int by = (int)((sqrtf(8.f * (float)blockIdx.x + 1.f) - 1.f) * 0.5f);  // column block index
  while ((by + 1) * (by + 2) / 2 <= (int)blockIdx.x) ++by;
  while (by * (by + 1) / 2 > (int)blockIdx.x) --by;
  const int bx = (int)blockIdx.x - by * (by + 1) / 2;  // row block, bx <= by
  if (by >= nb) return;
  const int zs = p.tab1 ? p.tab1[blockIdx.z] : (int)blockIdx.z;
  double* C = p.C + zs * p.sc1 + (long)blockIdx.y * p.sc2;
  const int r0 = bx * 32, c0 = by * 32;  // destination rows r0.., columns c0.. (upper side)
  const int tx = threadIdx.x & 31, ty = threadIdx.x >> 5;
  for (int i = ty; i < 32; i += 8) {  // source C(c, r): rows c0 + i, columns r0 + tx
    const int c = c0 + i, r = r0 + tx;
    if (c < p.M && r < p.M) tile[i][tx] = C[(long)c * p.scm + (long)r * p.scn];
  }
  __syncthreads();
  for (int i = ty; i < 32; i += 8) {
    const int r = r0 + i, c = c0 + tx;
    if (r < p.M && c < p.M && c > r) C[(long)r * p.scm + (long)c * p.scn] = tile[tx][i];
  }
}

// PM: B is pair-combined (ladder against the full (ac|bd) in pair order): for batch z2 = 0 (+)
// or 1 (-), B(k, n) = V[n][k] +- V[pm[n]][k] (rows of V at stride sbn).
// MINB: workgroups per CU the register budget is sized for.
template <int BM, int BN, int BK, int WM, int WN, int MINB, bool AMF, bool BNF, bool PM = false>
__global__ __launch_bounds__(WM* WN * 64, MINB) void gemm_f64_kernel(GP p) {
  constexpr int NT = WM * WN * 64;
  constexpr int TM = BM / WM, TN = BN / WN;
  constexpr int RI = TM / 16, RJ = TN / 16;
  constexpr int LA = BM * BK / NT, LB = BK * BN / NT;
  constexpr int PA = BM + 1, PB = BN + 1;  // +1 double: conflict-free transposing stores
  static_assert(RI >= 1 && RJ >= 1 && LA >= 1 && LB >= 1 && TM % 16 == 0 && TN % 16 == 0, "tile config");
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
  const int zs = p.tab1 ? p.tab1[z1] : z1;  // operand block of batch level 1
  const double* Ab = p.A + zs * p.sa1 + z2 * p.sa2;
  const double* Bb = p.B + zs * p.sb1 + z2 * p.sb2;
  double* Cb = p.C + zs * p.sc1 + z2 * p.sc2;

  // acc[i][j]: register r of lane l holds C(16i + l/16 + 4r, 16j + l%16) of the wave's tile
  typedef double d4 __attribute__((ext_vector_type(4)));
  d4 acc[RI][RJ];
#pragma unroll
  for (int i = 0; i < RI; ++i)
#pragma unroll
    for (int j = 0; j < RJ; ++j) acc[i][j] = d4{0.0, 0.0, 0.0, 0.0};

  const int nkt = (p.K + BK - 1) / BK;
  const int it_begin = slice * p.it_per_split;
  const int it_end = min(nkt * p.nred, it_begin + p.it_per_split);

  double ra[LA], rb[LB];
  double rw[PM ? LB : 1];  // pair-combined B: second row, combined with rb only when staged to LDS
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
  (void)rw;
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
        const bool ok = pva[l] && gk < p.K;
        rb[l] = ok ? pva[l][gk] : 0.0;
        rw[l] = ok ? pvb[l][gk] : 0.0;
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
      // the combination waits for the loads here, after the MFMAs, not where they are issued
      if constexpr (PM)
        Bs[buf][k * PB + n] = minus ? rb[l] - rw[l] : rb[l] + rw[l];
      else
        Bs[buf][k * PB + n] = rb[l];
    }
  };

  const int lk = lane >> 4, l16 = lane & 15;
  if (it_begin < it_end) {
    load(it_begin);
    store(0);
  }
  __syncthreads();
  for (int it = it_begin; it < it_end; ++it) {
    const int cur = (it - it_begin) & 1;
    if (it + 1 < it_end) load(it + 1);
    const double* as = As[cur] + lk * PA + wm * TM + l16;
    const double* bs = Bs[cur] + lk * PB + wn * TN + l16;
#pragma unroll
    for (int kk = 0; kk < BK; kk += 4) {
      double a[RI], b[RJ];
#pragma unroll
      for (int i = 0; i < RI; ++i) a[i] = as[kk * PA + 16 * i];
#pragma unroll
      for (int j = 0; j < RJ; ++j) b[j] = bs[kk * PB + 16 * j];
#pragma unroll
      for (int i = 0; i < RI; ++i)
#pragma unroll
        for (int j = 0; j < RJ; ++j) acc[i][j] = __builtin_amdgcn_mfma_f64_16x16x4f64(a[i], b[j], acc[i][j], 0, 0, 0);
    }
    if (it + 1 < it_end) store(cur ^ 1);
    __syncthreads();
  }

  // epilogue
#pragma unroll
  for (int i = 0; i < RI; ++i)
#pragma unroll
    for (int j = 0; j < RJ; ++j)
#pragma unroll
      for (int r = 0; r < 4; ++r) {
        const int gm = m0 + wm * TM + 16 * i + lk + 4 * r;
        const int gn = n0 + wn * TN + 16 * j + l16;
        if (gm < p.M && gn < p.N) {
          const double v = p.alpha * acc[i][j][r];
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

// C_z(m,n) = beta * C_z(m,n) + sum_s part[s][z][m][n].  Each block takes 64 consecutive outputs; its
// four waves sum four contiguous slice ranges in slice order, and the four partial sums are added
// in wave order (a fixed order, so the result is deterministic).
__global__ __launch_bounds__(256) void splitk_reduce(GP p, int nb1, long total) {
  __shared__ double red[4][64];
  const int lane = threadIdx.x & 63, w = threadIdx.x >> 6;
  const long x = blockIdx.x * 64L + lane;
  const int s0 = (int)((long)p.split * w / 4), s1 = (int)((long)p.split * (w + 1) / 4);
  double acc = 0.0;
  if (x < total)
    for (int sl = s0; sl < s1; ++sl) acc += p.part[(long)sl * total + x];
  red[w][lane] = acc;
  __syncthreads();
  if (w != 0 || x >= total) return;
  const double sum = ((red[0][lane] + red[1][lane]) + red[2][lane]) + red[3][lane];
  const long mn = (long)p.M * p.N;
  const long zl = x / mn, r = x % mn;
  const int gm = r / p.N, gn = r % p.N;
  const int z1 = zl / p.nb2, z2 = zl % p.nb2;
  const int zs = p.tab1 ? p.tab1[z1] : z1;
  double* c = p.C + zs * p.sc1 + z2 * p.sc2 + gm * p.scm + gn * p.scn;
  *c = (p.beta == 0.0) ? sum : sum + p.beta * *c;
}

// grid of splitk_reduce for `outs` outputs
inline unsigned splitk_blocks(long outs) { return (unsigned)((outs + 63) / 64); }

// nb1d: the outer batch count the split-K decision is made for (1: as for one operand block, so a
// block's sums take the same order whatever the batch; nb1 otherwise).
template <int BM, int BN, int BK, int WM, int WN, int MINB>
hipError_t launch_cfg(const GP& p0, bool amf, bool bnf, int nb1, int nb1d, double* ws, long ws_elems, hipStream_t s) {
  GP p = p0;
  p.tiles_m = (p.M + BM - 1) / BM;
  p.tiles_n = (p.N + BN - 1) / BN;
  const long tiles = (long)p.tiles_m * p.tiles_n * p.nb2 * nb1d;
  const int nit = ((p.K + BK - 1) / BK) * p.nred;
  p.split = 1;
  p.it_per_split = nit;
  p.part = nullptr;
  const long outs = (long)p.M * p.N * p.nb2 * nb1;
  if (ws && tiles < 192 && nit >= 16) {
    // slices enough for one full round of resident workgroups (MINB per CU)
    int sp = (int)std::min<long>({(256L * MINB + tiles - 1) / tiles, (long)nit / 8, 256L});
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
    hipLaunchKernelGGL((gemm_f64_kernel<BM, BN, BK, WM, WN, MINB, true, true>), grid, block, 0, s, p);
  else if (amf)
    hipLaunchKernelGGL((gemm_f64_kernel<BM, BN, BK, WM, WN, MINB, true, false>), grid, block, 0, s, p);
  else if (bnf)
    hipLaunchKernelGGL((gemm_f64_kernel<BM, BN, BK, WM, WN, MINB, false, true>), grid, block, 0, s, p);
  else
    hipLaunchKernelGGL((gemm_f64_kernel<BM, BN, BK, WM, WN, MINB, false, false>), grid, block, 0, s, p);
  if (p.split > 1) hipLaunchKernelGGL(splitk_reduce, dim3(splitk_blocks(outs)), dim3(256), 0, s, p, nb1, outs);
  return hipGetLastError();
}

// ---------------------------------------------------------------------------------------
// Direct-to-LDS path for K-contiguous operands, A(m,k) = A[m*sam + k] and B(k,n) = B[n*sbn + k]:
// rows go from global memory straight into LDS with global_load_lds_dwordx4 (lane l of an
// instruction writes LDS bytes 16l .. 16l + 15), S stages in flight, one barrier per stage and no
// staging registers.  A stage holds KS K-values of every tile row: KS = 8 (64-byte rows, the 16-byte
// chunk c of row r at slot c ^ ((r >> 1) & 3)) or KS = 16 (whole 128-byte lines, chunk c of row r
// at slot c ^ (r & 7)); either swizzle makes the fragment reads conflict-free.  Each fragment read
// returns two K-values and feeds two MFMAs: lane group g = l / 16 supplies K = 2g to the first and
// 2g + 1 to the second, identically for A and B; a 16-deep stage is read as two 8-deep halves in
// order, so the MFMA sequence along K, and with it every result, is the same for both depths.  Rows
// past M or N and K-values past K are read from a 16-byte zero block instead, so every load
// instruction runs on all lanes and the per-wave vmcnt bookkeeping is exact.  PM: B is
// pair-combined as in gemm_f64_kernel, both rows of each pair staged and combined at the fragment
// read (two B rows per pair leave room for two 16-deep stages only: the next stage loads while the
// current one is computed; every wave has read the refilled slot before the barrier that precedes
// the refill, as with more stages).
typedef __attribute__((address_space(3))) void lds_void_t;
typedef __attribute__((address_space(1))) const void gbl_void_t;
__device__ __attribute__((aligned(16))) double kZero16[2];

// s_waitcnt vmcnt(N) (bits 3:0 and 15:14), no wait on the other counters
template <int N>
__device__ __forceinline__ void wait_vmcnt() {
  static_assert(N >= 0 && N < 64, "vmcnt range");
  __builtin_amdgcn_s_waitcnt(0xF70 | (N & 15) | ((N >> 4) << 14));
}

template <int BM, int BN, int WM, int WN, int S, bool PM, int KS>
__global__ __launch_bounds__(WM* WN * 64, 1) void gemm_f64_dma_kernel(GP p) {
  typedef double dd2 __attribute__((ext_vector_type(2)));
  typedef double d4 __attribute__((ext_vector_type(4)));
  constexpr int NW = WM * WN;
  constexpr int TM = BM / WM, TN = BN / WN, RI = TM / 16, RJ = TN / 16;
  constexpr int NB = PM ? 2 : 1;
  constexpr int CPR = KS / 2, RPI = 64 / CPR;  // 16-byte chunks per staged row, rows per load instruction
  constexpr int IA = BM / RPI, IB = BN / RPI, NI = IA + NB * IB;  // 1 KB load instructions per stage
  constexpr int NPW = (NI + NW - 1) / NW, NPWMIN = NI / NW;        // per wave
  constexpr int ROWS = BM + NB * BN;
  static_assert(TM % 16 == 0 && TN % 16 == 0 && S >= 2 && NPWMIN >= 1, "tile config");
  static_assert(KS == 8 || KS == 16, "stage depth");
  __shared__ __attribute__((aligned(1024))) double T[S][ROWS * KS];
  auto swz = [](int r) { return KS == 8 ? (r >> 1) & 3 : r & 7; };  // slot of chunk 0 of row r

  const int tid = threadIdx.x, lane = tid & 63;
  const int wave = __builtin_amdgcn_readfirstlane(tid >> 6);
  const int wm = wave / WN, wn = wave % WN;
  const int ntiles = p.tiles_m * p.tiles_n;
  int bid = blockIdx.x, z2 = blockIdx.y;
  if constexpr (PM) {  // the + and - halves of a tile back to back on one XCD (see gemm_f64_kernel)
    const int x = bid & 7, local = bid >> 3;
    z2 = local & 1;
    bid = ((local >> 1) << 3) | x;
    if (bid >= ntiles) return;
  }
  const int slice = PM ? 0 : bid / ntiles;  // split-K slice (never for PM)
  int tm, tn;
  if (!PM && p.lower)
    tile_of_lower(bid, p.tiles_m, tm, tn);
  else
    tile_of(bid - slice * ntiles, p.tiles_m, p.tiles_n, tm, tn);
  const int m0 = tm * BM, n0 = tn * BN;
  const int z1 = blockIdx.z;
  const int zs = p.tab1 ? p.tab1[z1] : z1;  // operand block of batch level 1
  const double* Ab = p.A + zs * p.sa1 + z2 * p.sa2;
  const double* Bb = p.B + zs * p.sb1 + z2 * p.sb2;
  double* Cb = p.C + zs * p.sc1 + z2 * p.sc2;

  // the source row (chunk included) of this lane in each instruction its wave issues
  const double* src[NPW];
  bool ok[NPW];
  int ck[NPW];
#pragma unroll
  for (int j = 0; j < NPW; ++j) {
    const int g = wave + NW * j;
    const int r = RPI * g + lane / CPR;
    const int c = (lane % CPR) ^ swz(r);
    const double* row = nullptr;
    if (g < IA) {
      const int gm = m0 + r;
      if (gm < p.M) row = Ab + (long)gm * p.sam;
    } else if (g < IA + IB) {
      const int gn = n0 + r - BM;
      if (gn < p.N) row = Bb + (long)gn * p.sbn;
    } else if (g < NI) {
      const int gn = n0 + r - BM - BN;
      if (gn < p.N) row = Bb + (long)p.pm[gn] * p.sbn;
    }
    ok[j] = row != nullptr;
    ck[j] = 2 * c;
    src[j] = ok[j] ? row + 2 * c : kZero16;
  }
  // stages [kt0, kt0 + nkt) of this slice
  const int kt0 = slice * p.it_per_split;
  const int nkt = min((p.K + KS - 1) / KS, kt0 + p.it_per_split) - kt0;
  auto issue = [&](int kt, int st) {
#pragma unroll
    for (int j = 0; j < NPW; ++j) {
      const int g = wave + NW * j;
      if (NPW * NW == NI || g < NI) {
        const double* a = (ok[j] && kt * KS + ck[j] < p.K) ? src[j] + kt * KS : kZero16;
        __builtin_amdgcn_global_load_lds((gbl_void_t*)a, (lds_void_t*)&T[st][g * 128], 16, 0, 0);
      }
    }
  };

  d4 acc[RI][RJ];
#pragma unroll
  for (int i = 0; i < RI; ++i)
#pragma unroll
    for (int j = 0; j < RJ; ++j) acc[i][j] = d4{0.0, 0.0, 0.0, 0.0};
  const bool minus = PM && z2 == 1;
  const int l16 = lane & 15, q = lane >> 4;
#pragma unroll
  for (int st = 0; st < S - 1; ++st)
    if (st < nkt) issue(kt0 + st, st);
  for (int kt = 0; kt < nkt; ++kt) {  // kt counts stages of this slice
    const int st = kt % S;
    // stage kt has landed once no more than the later stages' loads of this wave are in flight
    if (kt + S - 2 < nkt)
      wait_vmcnt<(S - 2) * NPWMIN>();
    else
      wait_vmcnt<0>();
    // every wave has waited for its own part of the stage; no memory fence is needed (and
    // __syncthreads would add one that drains all stages in flight)
    asm volatile("" ::: "memory");
    __builtin_amdgcn_s_barrier();
    asm volatile("" ::: "memory");
    const double* Ts = T[st];
#pragma unroll
    for (int kk = 0; kk < KS / 8; ++kk) {  // 8-deep halves of the stage, in K order
      dd2 fa[RI], fb[RJ];
#pragma unroll
      for (int i = 0; i < RI; ++i) {
        const int r = wm * TM + 16 * i + l16;
        fa[i] = *reinterpret_cast<const dd2*>(Ts + r * KS + 2 * ((q + 4 * kk) ^ swz(r)));
      }
#pragma unroll
      for (int j = 0; j < RJ; ++j) {
        const int r = BM + wn * TN + 16 * j + l16;
        fb[j] = *reinterpret_cast<const dd2*>(Ts + r * KS + 2 * ((q + 4 * kk) ^ swz(r)));
        if constexpr (PM) {
          const int rw = r + BN;  // (r + BN) has the same swizzle as r: BN is a multiple of 16
          const dd2 w = *reinterpret_cast<const dd2*>(Ts + rw * KS + 2 * ((q + 4 * kk) ^ swz(rw)));
          fb[j] = minus ? fb[j] - w : fb[j] + w;
        }
      }
      // the stage refilled now was last read in the previous iteration, before this barrier
      if (kk == 0 && kt + S - 1 < nkt) issue(kt0 + kt + S - 1, (kt + S - 1) % S);
#pragma unroll
      for (int h = 0; h < 2; ++h)
#pragma unroll
        for (int i = 0; i < RI; ++i)
#pragma unroll
          for (int j = 0; j < RJ; ++j)
            acc[i][j] = __builtin_amdgcn_mfma_f64_16x16x4f64(fa[i][h], fb[j][h], acc[i][j], 0, 0, 0);
    }
  }
#pragma unroll
  for (int i = 0; i < RI; ++i)
#pragma unroll
    for (int j = 0; j < RJ; ++j)
#pragma unroll
      for (int r = 0; r < 4; ++r) {
        const int gm = m0 + wm * TM + 16 * i + q + 4 * r;
        const int gn = n0 + wn * TN + 16 * j + l16;
        if (gm < p.M && gn < p.N) {
          const double v = p.alpha * acc[i][j][r];
          if (p.split > 1) {
            const long zl = (long)z1 * gridDim.y + z2;
            p.part[(((long)slice * gridDim.z * gridDim.y + zl) * p.M + gm) * p.N + gn] = v;
          } else {
            double* c = Cb + (long)gm * p.scm + (long)gn * p.scn;
            *c = (p.beta == 0.0) ? v : v + p.beta * *c;
          }
        }
      }
}

// K-contiguous operands with 16-byte aligned rows and an even K (the loads move K-value pairs).
bool dma_eligible(const GP& p) {
  auto al = [](const void* x) { return (reinterpret_cast<uintptr_t>(x) & 15) == 0; };
  return p.sak == 1 && p.sbk == 1 && p.nred == 1 && p.K % 2 == 0 && p.sam % 2 == 0 && p.sbn % 2 == 0 &&
         p.sa1 % 2 == 0 && p.sa2 % 2 == 0 && p.sb1 % 2 == 0 && p.sb2 % 2 == 0 && al(p.A) && al(p.B);
}

// split > 1 (never with pm): K cut into `split` slices whose partial tiles go to ws, then summed
// in a fixed order by splitk_reduce.
template <int BM, int BN, int WM, int WN, int S, int KS = 8>
hipError_t launch_dma(GP p, int nb1, bool pm, int split, double* ws, hipStream_t s) {
  static_assert(KS == 8 || KS == 16, "stage depth");
  p.tiles_m = (p.M + BM - 1) / BM;
  p.tiles_n = (p.N + BN - 1) / BN;
  const int nkt = (p.K + KS - 1) / KS;
  p.it_per_split = (nkt + split - 1) / split;
  p.split = (nkt + p.it_per_split - 1) / p.it_per_split;
  p.part = p.split > 1 ? ws : nullptr;
  const int tiles = p.lower ? p.tiles_m * (p.tiles_m + 1) / 2 : p.tiles_m * p.tiles_n;
  if (p.lower && (p.split > 1 || pm || BM != BN || p.tiles_m != p.tiles_n)) return hipErrorInvalidValue;
  if (pm) {  // both halves in grid.x, padded to whole groups of 8
    if constexpr ((long)S * (BM + 2 * BN) * KS * 8 <= 160 * 1024) {
      dim3 grid(2 * ((tiles + 7) / 8 * 8), 1, nb1);
      hipLaunchKernelGGL((gemm_f64_dma_kernel<BM, BN, WM, WN, S, true, KS>), grid, dim3(WM * WN * 64), 0, s, p);
      return hipGetLastError();
    } else {
      return hipErrorInvalidValue;  // two B rows per pair do not fit this many stages
    }
  }
  dim3 grid(tiles * p.split, p.nb2, nb1);
  hipLaunchKernelGGL((gemm_f64_dma_kernel<BM, BN, WM, WN, S, false, KS>), grid, dim3(WM * WN * 64), 0, s, p);
  if (p.split > 1) {
    const long outs = (long)p.M * p.N * p.nb2 * nb1;
    hipLaunchKernelGGL(splitk_reduce, dim3(splitk_blocks(outs)), dim3(256), 0, s, p, nb1, outs);
  }
  return hipGetLastError();
}

// Direct-to-LDS launch for a non-pair-combined contraction: the tile (192 x 192, 256 x 128 or
// 224 x 128) and split-K count with the least estimated time = whole rounds of 256 workgroups x
// tile area x K-stages per slice; split-K only with scratch, when the tiles cannot fill one round.
hipError_t launch_dma_auto(const GP& p, int nb1, int nb1d, double* ws, long ws_elems, hipStream_t s) {
  const long nbatch = (long)p.nb2 * nb1d, outs = (long)p.M * p.N * p.nb2 * nb1;
  const int nkt = (p.K + 7) / 8;
  int best = -1, best_split = 1;
  double best_cost = 0.0;
  const int bms[3] = {192, 256, 224}, bns[3] = {192, 128, 128};
  for (int c = 0; c < 3; ++c) {
    const long tiles = (long)((p.M + bms[c] - 1) / bms[c]) * ((p.N + bns[c] - 1) / bns[c]) * nbatch;
    int sp = 1;
    if (ws && tiles < 192 && nkt >= 32) {
      sp = (int)std::min<long>({256 / tiles, (long)nkt / 16, 256L, ws_elems / std::max<long>(outs, 1)});
      sp = std::max(sp, 1);
    }
    const double cost = (double)((tiles * sp + 255) / 256) * bms[c] * bns[c] * ((nkt + sp - 1) / sp);
    if (best < 0 || cost < best_cost) {
      best = c;
      best_cost = cost;
      best_split = sp;
    }
  }
  if (best == 0) return launch_dma<192, 192, 2, 4, 3, 16>(p, nb1, false, best_split, ws, s);
  if (best == 1) return launch_dma<256, 128, 4, 2, 3, 16>(p, nb1, false, best_split, ws, s);
  return launch_dma<224, 128, 2, 4, 3, 16>(p, nb1, false, best_split, ws, s);
}

// Ladder: BM x 128 tiles of 8 waves, both halves (grid.y = 2), no split-K, A/B staged k-fast.
template <int BM, int WM>
hipError_t launch_ladder(GP p, int nb1, bool pm, hipStream_t s) {
  constexpr int BK = 16, WN = 8 / WM;
  p.tiles_m = (p.M + BM - 1) / BM;
  p.tiles_n = (p.N + 127) / 128;
  p.split = 1;
  p.it_per_split = (p.K + BK - 1) / BK;
  p.part = nullptr;
  const int tiles = p.tiles_m * p.tiles_n;
  // pair-combined: the two halves interleave in grid.x (see the kernel), padded to groups of 8
  dim3 grid(pm ? 2 * ((tiles + 7) / 8 * 8) : tiles, pm ? 1 : 2, nb1), block(512);
  if (pm)
    hipLaunchKernelGGL((gemm_f64_kernel<BM, 128, BK, WM, WN, 1, false, false, true>), grid, block, 0, s, p);
  else
    hipLaunchKernelGGL((gemm_f64_kernel<BM, 128, BK, WM, WN, 1, false, false, false>), grid, block, 0, s, p);
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
  const long e1 = g.tab1 ? g.tab1_max + 1 : g.nb1;  // batch level 1 spans the table's entries
  const long ea[5] = {g.M, g.K, e1, g.nb2, g.nred}, sa[5] = {g.sam, g.sak, g.sa1, g.sa2, g.sar};
  affine_range(ea, sa, 5, lo, hi);
  if (!range_ok(g.A, lo, hi, sizeof(double), "gemm A")) return false;
  const long eb[5] = {g.K, g.N, e1, g.nb2, g.nred}, sb[5] = {g.sbk, g.sbn, g.sb1, g.sb2, g.sbr};
  affine_range(eb, sb, 5, lo, hi);
  if (!range_ok(g.B, lo, hi, sizeof(double), "gemm B")) return false;
  const long ec[4] = {g.M, g.N, e1, g.nb2}, sc[4] = {g.scm, g.scn, g.sc1, g.sc2};
  affine_range(ec, sc, 4, lo, hi);
  if (!range_ok(g.C, lo, hi, sizeof(double), "gemm C")) return false;
  return !g.ws || range_ok(g.ws, 0, g.ws_elems - 1, sizeof(double), "gemm split-K scratch");
}

hipError_t gemm_f64(const Gemm& g, hipStream_t s) {
  if (g.M <= 0 || g.N <= 0 || g.nb1 <= 0 || g.nb2 <= 0) return hipSuccess;
  if (bounds_checking() && !gemm_in_bounds(g)) return hipErrorInvalidValue;
  if (dry_run()) return hipSuccess;
  if (g.nb1 > 65535 || g.nb2 > 65535) return hipErrorInvalidValue;
  // tile and split-K choices: for the whole batch, or as for one block of the outer level
  const int nb1d = g.per_block ? 1 : g.nb1, nbatch = nb1d * g.nb2;
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
  p.tab1 = g.tab1;
  p.lower = 0;
  if (g.lower && g.M == g.N && g.beta == 0.0 && dma_eligible(p)) {
    // symmetric C: the 192 x 192 tiles on and below the diagonal, then the mirror of the strict
    // upper triangle (each mirrored value sums the same products in the same K order); other
    // symmetric products (odd K, unaligned rows) take the full product below
    p.lower = 1;
    hipError_t e = launch_dma<192, 192, 2, 4, 3, 16>(p, g.nb1, false, 1, nullptr, s);
    if (e != hipSuccess) return e;
    const long nbk = (g.M + 31) / 32;
    hipLaunchKernelGGL(mirror_upper_kernel, dim3((unsigned)(nbk * (nbk + 1) / 2), (unsigned)g.nb2, (unsigned)g.nb1),
                       dim3(256), 0, s, p);
    return hipGetLastError();
  }
  // Global-load order: an operand whose m (n) stride is 1 is read m-fast (n-fast).
  const bool amf = (g.sam == 1 && g.sak != 1);
  const bool bnf = (g.sbn == 1) || (g.sbk != 1);
  const long tiles128 = (long)((g.M + 127) / 128) * ((g.N + 127) / 128) * nbatch;
  if (g.M >= 96 && g.N >= 96 && tiles128 >= 256) {
    // Large outputs: among 128x128 (4 waves), 256x128 and 192x192 (8 waves) take the least
    // estimated time = whole rounds of 256 tiles x tile area / sustained rate (measured on full
    // rounds: 59.5, 60, 61.5 TFLOP/s), which prices both the padding of M and N and the partly
    // filled last round.
    auto est = [&](int bm, int bn, double rate) {
      const long t = (long)((g.M + bm - 1) / bm) * ((g.N + bn - 1) / bn) * nbatch;
      return (double)((t + 255) / 256) * bm * bn / rate;
    };
    const double e128 = est(128, 128, 59.5), e256 = est(256, 128, 60.0), e192 = est(192, 192, 61.5);
    // direct-to-LDS tiles sustain ~67-68 TFLOP/s on full rounds
    if (dma_eligible(p)) return launch_dma_auto(p, g.nb1, nb1d, g.ws, g.ws_elems, s);
    if (e192 < e128 && e192 <= e256) return launch_cfg<192, 192, 16, 2, 4, 1>(p, amf, bnf, g.nb1, nb1d, nullptr, 0, s);
    if (e256 < e128) return launch_cfg<256, 128, 16, 4, 2, 1>(p, amf, bnf, g.nb1, nb1d, nullptr, 0, s);
    return launch_cfg<128, 128, 16, 2, 2, 2>(p, amf, bnf, g.nb1, nb1d, g.ws, g.ws_elems, s);
  }
  // a long K lets split-K make up for too few 128 x 128 tiles (down to 16 of them: split into up
  // to 32 slices, a long K still leaves each slice enough iterations to hide its reduction)
  const bool long_k = g.ws && (long)g.K * g.nred >= 2048 && tiles128 >= 16;
  if (g.M >= 96 && g.N >= 96 && long_k) {
    if (dma_eligible(p)) return launch_dma_auto(p, g.nb1, nb1d, g.ws, g.ws_elems, s);
    return launch_cfg<128, 128, 16, 2, 2, 2>(p, amf, bnf, g.nb1, nb1d, g.ws, g.ws_elems, s);
  }
  const long tiles64 = (long)((g.M + 63) / 64) * ((g.N + 63) / 64) * nbatch;
  if (g.M >= 48 && g.N >= 48 && tiles64 >= 128)
    return launch_cfg<64, 64, 16, 2, 2, 2>(p, amf, bnf, g.nb1, nb1d, g.ws, g.ws_elems, s);
  // a narrow output over a long K: 64 x 64 tiles of four waves, split along K, keep more of each
  // CU busy (and more loads in flight) than single-wave 32 x 32 tiles
  if (g.ws && g.M >= 16 && g.N >= 16 && (long)g.K * g.nred >= 2048 && tiles64 < 192)
    return launch_cfg<64, 64, 16, 2, 2, 2>(p, amf, bnf, g.nb1, nb1d, g.ws, g.ws_elems, s);
  return launch_cfg<32, 32, 16, 1, 1, 3>(p, amf, bnf, g.nb1, nb1d, g.ws, g.ws_elems, s);
}

hipError_t gemm_f64_ladder(int M, int Tv, const double* A, const double* V, long ldv, long vrows, const int* pm,
                           double* C, hipStream_t s, const LadderBatch& lb) {
  if (M <= 0 || Tv <= 0) return hipSuccess;
  const bool pmode = pm != nullptr;
  if (pmode && (ldv < Tv || vrows < Tv)) return hipErrorInvalidValue;
  const long half = (long)M * Tv;
  if (bounds_checking()) {
    const long vlast = pmode ? (vrows - 1) * ldv + Tv - 1 : 2L * Tv * Tv - 1;
    const long e1 = lb.tab ? lb.tab_max : lb.n - 1;  // last operand block of batch level 1
    if (!(range_ok(A, 0, e1 * lb.sa + 2 * half - 1, sizeof(double), "ladder A") &&
          range_ok(C, 0, e1 * lb.sc + 2 * half - 1, sizeof(double), "ladder C") &&
          range_ok(V, 0, e1 * lb.sv + vlast, sizeof(double), "ladder V") &&
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
  p.sa1 = lb.sa;
  p.sb1 = lb.sv;
  p.sc1 = lb.sc;
  p.tab1 = lb.tab;
  // Row tiles of 256, 240, 224, 208 or 128 pair rows: the least padded M wins (each extra row is a full
  // row of wasted products); on a tie the taller tile, which reads the vvvv operand fewer times.
  // 208 rows (one wave column of 13 x 16 rows per wave) fit T(40) = 820 pairs in four tiles with
  // 1.5 % padding where 224 rows pad by 9 %.
  const long pad256 = (M + 255L) / 256 * 256, pad224 = (M + 223L) / 224 * 224, pad128 = (M + 127L) / 128 * 128;
  const long pad208 = (M + 207L) / 208 * 208, pad240 = (M + 239L) / 240 * 240;
  if (lb.n > 65535) return hipErrorInvalidValue;
  if (dma_eligible(p)) {
    // 240 rows (one wave column of 15 x 16 rows per wave) fit T(21) = 231 pairs with 4 % padding
    // where 256 rows pad by 11 %, and sixteen stacked T(30) = 465 states exactly
    const long best = std::min({pad256, pad240, pad224, pad208, pad128});
    const int t = pad256 == best ? 0 : pad240 == best ? 4 : pad224 == best ? 1 : pad208 == best ? 2 : 3;
    if (pmode) {  // two B rows per pair: two 16-deep stages
      if (t == 0) return launch_dma<256, 128, 4, 2, 2, 16>(p, lb.n, true, 1, nullptr, s);
      if (t == 4) return launch_dma<240, 128, 1, 8, 2, 16>(p, lb.n, true, 1, nullptr, s);
      if (t == 1) return launch_dma<224, 128, 2, 4, 2, 16>(p, lb.n, true, 1, nullptr, s);
      if (t == 2) return launch_dma<208, 128, 1, 8, 2, 16>(p, lb.n, true, 1, nullptr, s);
      return launch_dma<128, 128, 2, 4, 2, 16>(p, lb.n, true, 1, nullptr, s);
    }
    if (t == 0) return launch_dma<256, 128, 4, 2, 3, 16>(p, lb.n, false, 1, nullptr, s);
    if (t == 4) return launch_dma<240, 128, 1, 8, 3, 16>(p, lb.n, false, 1, nullptr, s);
    if (t == 1) return launch_dma<224, 128, 2, 4, 3, 16>(p, lb.n, false, 1, nullptr, s);
    if (t == 2) return launch_dma<208, 128, 1, 8, 3, 16>(p, lb.n, false, 1, nullptr, s);
    return launch_dma<128, 128, 2, 4, 3, 16>(p, lb.n, false, 1, nullptr, s);
  }
  if (pad256 <= pad224 && pad256 <= pad128) return launch_ladder<256, 4>(p, lb.n, pmode, s);
  if (pad224 <= pad128) return launch_ladder<224, 2>(p, lb.n, pmode, s);
  return launch_ladder<128, 2>(p, lb.n, pmode, s);
}

}  // namespace ascc
