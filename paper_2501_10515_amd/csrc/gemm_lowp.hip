// Low-precision contractions on the matrix cores, FP64 result:
//
//   C_z(m,n) = alpha * sum_k A_z[m][k] B_z[n][k] + beta * C_z(m,n)
//
// A and B are low-precision shadows of FP64 operands (row-major, K contiguous, zero-padded rows,
// rounded to nearest even by the conversion kernels); C is FP64 with general strides.  Two
// arithmetic policies:
//
//   FP32   : v_mfma_f32_16x16x4_f32 on FP32 shadows (256 x 256 direct-to-LDS tiles for large
//            products, 128 x 128 register-staged ones for small).
//   BF16X3 : the shadows are two bf16 planes, x = hi + lo with hi = RNE_bf16(x),
//            lo = RNE_bf16(x - hi); v_mfma_f32_16x16x32_bf16 forms lo*hi + hi*lo + hi*hi (the
//            lo*lo term, relative size 2^-16, is dropped).
//
// Both accumulate in FP32 inside a K chunk and add each chunk's partial sum into the FP64 C tile
// (which the workgroup owns for the whole K range), so accumulation across chunks is FP64.
//
// MFMA lane layouts (gfx950, measured): f32 16x16x4 -- lane l supplies A(l%16, l/16) and
// B(l/16, l%16); bf16 16x16x32 -- lane l supplies A(l%16, 8(l/16)+j) and B(8(l/16)+j, l%16),
// j = 0..7; both return register r of lane l as C(4(l/16)+r, l%16); bf16 32x32x16 -- lane l
// supplies A(l%32, 8(l/32)+j) and B(8(l/32)+j, l%32) and returns register q as
// C(8(q/4) + 4(l/32) + q%4, l%32).
#include <algorithm>
#include <cstdint>
#include <cstdlib>

#include "internal.h"

namespace ascc {
namespace {

typedef float f4 __attribute__((ext_vector_type(4)));
typedef __bf16 bf8 __attribute__((ext_vector_type(8)));

struct LP {
  int M, N, K;
  const float* A;
  long lda, sa2;
  const float* B;
  long ldb, sb2;
  double* C;
  long scm, scn, sc2;
  double alpha, beta;
  int tiles_m, tiles_n;
  int chunk;    // K-tiles per FP32 accumulation chunk
  int ktps;     // K-tiles per split-K slice (blockIdx.z); the whole K when not split
  long cslice;  // C offset between slices (partial tiles of a split launch), 0 otherwise
  // batch: blockIdx.y = z1 * nb + z; z1 selects operand block tab1[z1] (or z1) at strides
  // sa1, sb1, sc1 (partial tiles of a split launch: block z1 itself)
  int nb, part;
  const int* tab1;
  long sa1, sb1, sc1;
};

// The eight-wave split-BF16x3 kernel adds a later FP32 chunk's partial sum into the FP64 result with
// a non-returning FP64 atomic add, performed at L2: the old value is never read into registers
// (2.8 % of the o40 v360 split-BF16x3 step; the FP32 kernels' 16 x 16 output layout, four rows per
// instruction, made the same change twice as slow there, so they keep the load-add-store).  Each
// element has one writer (the lane that owns it) and its chunks arrive in order, so the sums are
// those of a load-add-store; the first chunk's plain stores are waited for before any add follows.
__device__ __forceinline__ void add_to(double* p, double v) { unsafeAtomicAdd(p, v); }

// Round-to-nearest-even FP32 -> bf16 bits (finite inputs; NaN stays NaN).
__device__ __forceinline__ unsigned short bf16_rne(float f) {
  const uint32_t u = __float_as_uint(f);
  if ((u & 0x7f800000u) == 0x7f800000u) return (unsigned short)((u >> 16) | ((u & 0xffffu) ? 0x40u : 0u));
  const uint32_t r = u + 0x7fffu + ((u >> 16) & 1u);
  return (unsigned short)(r >> 16);
}
__device__ __forceinline__ float bf16_to_f(unsigned short h) { return __uint_as_float(((uint32_t)h) << 16); }

// ASCC_NO_TAIL_TILES=1 (read once per process) keeps a last row tile of at most 64 rows in the
// full-tile launch instead of the tail launch; both give the same rows bit for bit.
bool tail_tiles_enabled() {
  static const bool on = [] {
    const char* e = std::getenv("ASCC_NO_TAIL_TILES");
    return !(e && e[0] == '1');
  }();
  return on;
}

// Same, walked in groups of 8 M-tiles (M fastest inside a group): the workgroups resident on one
// XCD at a time cover a compact block of C and share A and B slices in its L2.
__device__ __forceinline__ void tile_of_grouped(int bid, int tiles_m, int tiles_n, int& tm, int& tn) {
  constexpr int GM = 8;
  const int total = tiles_m * tiles_n;
  const int q = total >> 3, rem = total & 7;
  const int x = bid & 7, local = bid >> 3;
  const int t = x * q + min(x, rem) + local;
  const int per = GM * tiles_n;
  const int g = t / per, first = g * GM;
  const int gs = min(tiles_m - first, GM);
  const int r = t - g * per;
  tm = first + r % gs;
  tn = r / gs;
}

__device__ __forceinline__ void tile_of_lp(int bid, int tiles_m, int total, int& tm, int& tn) {
  const int q = total >> 3, rem = total & 7;
  const int x = bid & 7, local = bid >> 3;
  const int tile = x * q + min(x, rem) + local;
  tm = tile % tiles_m;
  tn = tile / tiles_m;
}

constexpr int BM = 128, BN = 128, NT = 256;

// FP32 policy: 128 x 128 tiles, four 64 x 64 waves, v_mfma_f32_16x16x4_f32.
__global__ __launch_bounds__(NT, 1) void gemm_lowp_kernel(LP p) {
  // K depth per LDS stage and row pitch of the staged tiles (elements)
  constexpr int BK = 32;
  constexpr int PITCH = BK + 4;
  // per stage each thread moves 4 float4 of A and 4 of B (128 x 32 floats each)
  constexpr int LQ = BM * BK / 4 / NT;
  static_assert(LQ == 4, "tile config");
  __shared__ __attribute__((aligned(16))) float As[2][BM * PITCH];
  __shared__ __attribute__((aligned(16))) float Bs[2][BN * PITCH];

  const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
  const int wm = wave >> 1, wn = wave & 1;  // 2 x 2 waves of 64 x 64
  int tm, tn;
  tile_of_lp(blockIdx.x, p.tiles_m, p.tiles_m * p.tiles_n, tm, tn);
  const int m0 = tm * BM, n0 = tn * BN;
  const int z = blockIdx.y % p.nb, z1 = blockIdx.y / p.nb;
  const int zs = __builtin_amdgcn_readfirstlane(p.tab1 ? p.tab1[z1] : z1);  // uniform: scalar buffer descriptors
  const float* Ab = p.A + z * p.sa2 + zs * p.sa1;
  const float* Bb = p.B + z * p.sb2 + zs * p.sb1;
  double* Cb = p.C + z * p.sc2 + (p.part ? z1 : zs) * p.sc1 + blockIdx.z * p.cslice;

  f4 acc[4][4];
#pragma unroll
  for (int i = 0; i < 4; ++i)
#pragma unroll
    for (int j = 0; j < 4; ++j) acc[i][j] = f4{0.f, 0.f, 0.f, 0.f};

  // K-tiles [kt0, nkt) of this split-K slice
  const int kt0 = blockIdx.z * p.ktps, nkt = min((p.K + BK - 1) / BK, kt0 + p.ktps);
  f4 ra[LQ], rb[LQ];
  // chunk c = tid + NT*l of the tile: row c/8, k offset 4*(c%8)
  auto load = [&](int kt) {
    const int k0 = kt * BK;
#pragma unroll
    for (int l = 0; l < LQ; ++l) {
      const int c = tid + l * NT;
      const int r = c >> 3, kq = (c & 7) * 4;
      const int gk = k0 + kq;
      const int gm = m0 + r, gn = n0 + r;
      f4 va = f4{0.f, 0.f, 0.f, 0.f}, vb = va;
      if (gm < p.M) {
        const float* src = Ab + gm * p.lda + gk;
        if (gk + 3 < p.K && ((reinterpret_cast<uintptr_t>(src) & 15) == 0)) {
          va = *reinterpret_cast<const f4*>(src);
        } else {
#pragma unroll
          for (int t = 0; t < 4; ++t)
            if (gk + t < p.K) va[t] = src[t];
        }
      }
      if (gn < p.N) {
        const float* src = Bb + gn * p.ldb + gk;
        if (gk + 3 < p.K && ((reinterpret_cast<uintptr_t>(src) & 15) == 0)) {
          vb = *reinterpret_cast<const f4*>(src);
        } else {
#pragma unroll
          for (int t = 0; t < 4; ++t)
            if (gk + t < p.K) vb[t] = src[t];
        }
      }
      ra[l] = va;
      rb[l] = vb;
    }
  };
  auto store = [&](int buf) {
#pragma unroll
    for (int l = 0; l < LQ; ++l) {
      const int c = tid + l * NT;
      const int r = c >> 3, kq = (c & 7) * 4;
      *reinterpret_cast<f4*>(&As[buf][r * PITCH + kq]) = ra[l];
      *reinterpret_cast<f4*>(&Bs[buf][r * PITCH + kq]) = rb[l];
    }
  };

  auto flush = [&](bool first) {
#pragma unroll
    for (int i = 0; i < 4; ++i)
#pragma unroll
      for (int j = 0; j < 4; ++j)
#pragma unroll
        for (int r = 0; r < 4; ++r) {
          const int gm = m0 + wm * 64 + i * 16 + 4 * (lane >> 4) + r;
          const int gn = n0 + wn * 64 + j * 16 + (lane & 15);
          if (gm < p.M && gn < p.N) {
            double* c = Cb + gm * p.scm + gn * p.scn;
            const double v = p.alpha * (double)acc[i][j][r];
            if (first)
              *c = (p.beta == 0.0) ? v : v + p.beta * *c;
            else
              *c += v;
          }
          acc[i][j][r] = 0.f;
        }
  };

  const int lr = lane & 15, lg = lane >> 4;
  if (kt0 < nkt) {
    load(kt0);
    store(0);
  }
  __syncthreads();
  for (int kc = kt0; kc < nkt; kc += p.chunk) {
  const int kend = min(nkt, kc + p.chunk);
  for (int kt = kc; kt < kend; ++kt) {
    const int cur = (kt - kt0) & 1;
    if (kt + 1 < nkt) load(kt + 1);
    const float* as = As[cur];
    const float* bs = Bs[cur];
#pragma unroll
    for (int kk = 0; kk < BK; kk += 4) {
      float xa[4], xb[4];
#pragma unroll
      for (int i = 0; i < 4; ++i) xa[i] = as[(wm * 64 + i * 16 + lr) * PITCH + kk + lg];
#pragma unroll
      for (int j = 0; j < 4; ++j) xb[j] = bs[(wn * 64 + j * 16 + lr) * PITCH + kk + lg];
#pragma unroll
      for (int i = 0; i < 4; ++i)
#pragma unroll
        for (int j = 0; j < 4; ++j) acc[i][j] = __builtin_amdgcn_mfma_f32_16x16x4f32(xa[i], xb[j], acc[i][j], 0, 0, 0);
    }
    if (kt + 1 < nkt) store(cur ^ 1);
    __syncthreads();
  }
  flush(kc == kt0);
  }
  if (kt0 >= nkt) flush(true);
}

// Row-padded conversions: out row r holds in row r (cols values) then zeros up to ldo.
__global__ __launch_bounds__(256) void cvt_f32_2d_kernel(float* __restrict__ out, long ldo, const double* __restrict__ in,
                                                         long ldi, long rows, long cols) {
  const long total = rows * ldo;
  for (long x = blockIdx.x * 256L + threadIdx.x; x < total; x += (long)gridDim.x * 256) {
    const long r = x / ldo, c = x - r * ldo;
    out[x] = (c < cols) ? (float)in[r * ldi + c] : 0.f;
  }
}

// Interleaved split of a row-padded matrix: row r of the output holds, for each K-block kb of 32,
// hi[32] at r * 2ldo + 64kb and lo[32] right after it (ldo a multiple of 32; padding zeroed).
__global__ __launch_bounds__(256) void split_bf16_2d_kernel(unsigned short* __restrict__ out, long ldo,
                                                            const double* __restrict__ in, long ldi, long rows,
                                                            long cols) {
  const long total = rows * ldo;
  for (long x = blockIdx.x * 256L + threadIdx.x; x < total; x += (long)gridDim.x * 256) {
    const long r = x / ldo, c = x - r * ldo;
    unsigned short h = 0, l = 0;
    if (c < cols) {
      const double d = in[r * ldi + c];
      h = bf16_rne((float)d);
      l = bf16_rne((float)(d - (double)bf16_to_f(h)));
    }
    const long o = r * 2 * ldo + (c >> 5) * 64 + (c & 31);
    out[o] = h;
    out[o + 32] = l;
  }
}

// The same two conversions, eight columns per thread (one K-block of 32 never splits a group):
// 16-byte loads of the FP64 source (16-byte aligned rows: `in` aligned, ldi even) and 16-byte
// stores, one index division per eight elements; each element is converted exactly as above.
__global__ __launch_bounds__(256) void cvt_f32_2d_v8_kernel(float* __restrict__ out, long ldo,
                                                            const double* __restrict__ in, long ldi, long rows,
                                                            long cols) {
  const long per = ldo >> 3, total = rows * per;
  for (long x = blockIdx.x * 256L + threadIdx.x; x < total; x += (long)gridDim.x * 256) {
    const long r = x / per, c = (x - r * per) << 3;
    const double* src = in + r * ldi + c;
    double d[8];
    if (c + 8 <= cols) {
#pragma unroll
      for (int j = 0; j < 4; ++j) {
        const double2 v = reinterpret_cast<const double2*>(src)[j];
        d[2 * j] = v.x;
        d[2 * j + 1] = v.y;
      }
    } else {
#pragma unroll
      for (int j = 0; j < 8; ++j) d[j] = (c + j < cols) ? src[j] : 0.0;
    }
    float4* o = reinterpret_cast<float4*>(out + r * ldo + c);
    o[0] = make_float4((float)d[0], (float)d[1], (float)d[2], (float)d[3]);
    o[1] = make_float4((float)d[4], (float)d[5], (float)d[6], (float)d[7]);
  }
}

__global__ __launch_bounds__(256) void split_bf16_2d_v8_kernel(unsigned short* __restrict__ out, long ldo,
                                                               const double* __restrict__ in, long ldi, long rows,
                                                               long cols) {
  const long per = ldo >> 3, total = rows * per;
  for (long x = blockIdx.x * 256L + threadIdx.x; x < total; x += (long)gridDim.x * 256) {
    const long r = x / per, c = (x - r * per) << 3;
    const double* src = in + r * ldi + c;
    double d[8];
    if (c + 8 <= cols) {
#pragma unroll
      for (int j = 0; j < 4; ++j) {
        const double2 v = reinterpret_cast<const double2*>(src)[j];
        d[2 * j] = v.x;
        d[2 * j + 1] = v.y;
      }
    } else {
#pragma unroll
      for (int j = 0; j < 8; ++j) d[j] = (c + j < cols) ? src[j] : 0.0;
    }
    uint32_t hw[4], lw[4];
#pragma unroll
    for (int j = 0; j < 4; ++j) {
      const unsigned short h0 = bf16_rne((float)d[2 * j]), h1 = bf16_rne((float)d[2 * j + 1]);
      const unsigned short l0 = bf16_rne((float)(d[2 * j] - (double)bf16_to_f(h0)));
      const unsigned short l1 = bf16_rne((float)(d[2 * j + 1] - (double)bf16_to_f(h1)));
      hw[j] = (uint32_t)h0 | ((uint32_t)h1 << 16);
      lw[j] = (uint32_t)l0 | ((uint32_t)l1 << 16);
    }
    unsigned short* o = out + r * 2 * ldo + (c >> 5) * 64 + (c & 31);
    *reinterpret_cast<uint4*>(o) = make_uint4(hw[0], hw[1], hw[2], hw[3]);
    *reinterpret_cast<uint4*>(o + 32) = make_uint4(lw[0], lw[1], lw[2], lw[3]);
  }
}

// Transposing low-precision shadow: out row r (< rows) holds in[c][r] for c < cols, zero padding
// up to ldo (a multiple of 32), laid out as to_lowp_2d lays out its rows.  32 x 32 tiles through
// LDS, so both the reads (along r) and the writes (along c) are coalesced.
template <bool BF>
__global__ __launch_bounds__(256) void lowp_t_kernel(void* __restrict__ outp, long ldo, const double* __restrict__ in,
                                                     long ldi, long rows, long cols) {
  __shared__ double tile[32][33];
  const long r0 = (long)blockIdx.x * 32, c0 = (long)blockIdx.y * 32;
  const int tx = threadIdx.x & 31, ty = threadIdx.x >> 5;  // 32 x 8
#pragma unroll
  for (int k = 0; k < 4; ++k) {
    const int cy = ty + 8 * k;
    const long r = r0 + tx, c = c0 + cy;
    tile[cy][tx] = (r < rows && c < cols) ? in[c * ldi + r] : 0.0;
  }
  __syncthreads();
#pragma unroll
  for (int k = 0; k < 4; ++k) {
    const int ry = ty + 8 * k;
    const long r = r0 + ry, c = c0 + tx;
    if (r >= rows) continue;
    const double d = tile[tx][ry];
    if (BF) {
      unsigned short* out = reinterpret_cast<unsigned short*>(outp);
      const unsigned short h = bf16_rne((float)d);
      const long o = r * 2 * ldo + (c >> 5) * 64 + (c & 31);
      out[o] = h;
      out[o + 32] = bf16_rne((float)(d - (double)bf16_to_f(h)));
    } else {
      reinterpret_cast<float*>(outp)[r * ldo + c] = (float)d;
    }
  }
}

// Low-precision shadow of the vvvv halves formed from the full (ac|bd) matrix in pair order (rows
// at stride ldv): row r = h*Tv + n (h = 0: +, 1: -), column k < Tv, zero padding up to ldo; in FP64
// x = V[n][k] +- V[pm[n]][k], then rounded and laid out as to_lowp_2d does (FP32, or interleaved bf16).
template <bool BF>
__global__ __launch_bounds__(256) void lowp_pm_kernel(unsigned short* __restrict__ bo, float* __restrict__ out,
                                                      long ldo, const double* __restrict__ V, long ldv,
                                                      const int* __restrict__ pm, long Tv) {
  const long total = 2 * Tv * ldo;
  for (long x = blockIdx.x * 256L + threadIdx.x; x < total; x += (long)gridDim.x * 256) {
    const long r = x / ldo, c = x - r * ldo;
    double d = 0.0;
    if (c < Tv) {
      const bool minus = r >= Tv;
      const long n = minus ? r - Tv : r;
      const double u = V[n * ldv + c], w = V[(long)pm[n] * ldv + c];
      d = minus ? u - w : u + w;
    }
    if (BF) {
      const unsigned short h = bf16_rne((float)d);
      const long o = r * 2 * ldo + (c >> 5) * 64 + (c & 31);
      bo[o] = h;
      bo[o + 32] = bf16_rne((float)(d - (double)bf16_to_f(h)));
    } else {
      out[x] = (float)d;
    }
  }
}



// ---------------------------------------------------------------------------------------
// Split-BF16x3 on pre-split operands: each row of A and B holds, per K-block of 32, the 32 hi
// values then the 32 lo values (bf16; row stride lda/ldb a multiple of 64, zero padding), so one
// K-step of a row is one 128-byte line, every staging load is one 16-byte chunk and no
// conversion happens in the kernel.
//
// LDS tiles hold 32 K-values per row (64 bytes) with no padding; the 16-byte chunk c of row r is
// stored at slot c ^ ((r >> 1) & 3).  Measured on gfx950 (bank-conflict counters), this makes both
// the fragment reads of v_mfma_f32_16x16x32_bf16 (row = lane % 16, chunk = lane / 16) and the
// four-lanes-per-row staging stores conflict-free; padded 80-byte rows conflict 2-way on both.
//
// Two kernels: 256 x 128 tiles of eight 64 x 64 waves with register-staged loads (small
// contractions: fewer than 128 tiles of 256 x 256, or 64 with split-K scratch), and 256 x 256 tiles
// of eight 128 x 64 waves whose operands are loaded straight into LDS by buffer_load ... lds,
// double-buffered (the rest, K split into slices to fill a round when the tiles are too few: half
// the LDS traffic per MFMA and no staging registers).
__device__ __forceinline__ int lds_slot(int r, int c) { return r * 32 + ((c ^ ((r >> 1) & 3)) << 3); }

struct LPB {
  int M, N, K;
  const unsigned short* A;
  long lda, sa2;
  const unsigned short* B;
  long ldb, sb2;
  double* C;
  long scm, scn, sc2;
  double alpha, beta;
  int tiles_m, tiles_n;
  int chunk;
  int ktps;
  long cslice;
  int nb, part;  // batch levels as in LP
  const int* tab1;
  long sa1, sb1, sc1;
};

constexpr int BM2 = 256, BN2 = 128, BK2 = 32, NT2 = 512;
typedef unsigned int u4 __attribute__((ext_vector_type(4)));

__global__ __launch_bounds__(NT2, 1) void gemm_bf16x3_kernel(LPB p) {
  __shared__ __attribute__((aligned(16))) unsigned short As[2][2][BM2 * BK2];
  __shared__ __attribute__((aligned(16))) unsigned short Bs[2][2][BN2 * BK2];
  const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
  const int wm = wave >> 1, wn = wave & 1;  // 4 x 2 waves of 64 x 64
  int tm, tn;
  tile_of_lp(blockIdx.x, p.tiles_m, p.tiles_m * p.tiles_n, tm, tn);
  const int m0 = tm * BM2, n0 = tn * BN2;
  const int z = blockIdx.y % p.nb, z1 = blockIdx.y / p.nb;
  const int zs = __builtin_amdgcn_readfirstlane(p.tab1 ? p.tab1[z1] : z1);  // uniform: scalar buffer descriptors
  const unsigned short* Ab = p.A + z * p.sa2 + zs * p.sa1;
  const unsigned short* Bb = p.B + z * p.sb2 + zs * p.sb1;
  double* Cb = p.C + z * p.sc2 + (p.part ? z1 : zs) * p.sc1 + blockIdx.z * p.cslice;

  f4 acc[4][4];
#pragma unroll
  for (int i = 0; i < 4; ++i)
#pragma unroll
    for (int j = 0; j < 4; ++j) acc[i][j] = f4{0.f, 0.f, 0.f, 0.f};

  const int kt0 = blockIdx.z * p.ktps, nkt = min((p.K + BK2 - 1) / BK2, kt0 + p.ktps);
  u4 ra[4], rb[2];
  // Workgroup-uniform bases (scalar registers) plus 32-bit per-lane element offsets keep the
  // address arithmetic out of the vector register budget.
  const unsigned short* Arow = Ab + (long)m0 * p.lda;
  const unsigned short* Brow = Bb + (long)n0 * p.ldb;
  const int lda = (int)p.lda, ldb = (int)p.ldb, kpad = lda / 2;  // lda == ldb for these operands
  // A: 256 rows x 4 chunks x 2 planes = 2048 chunks (4 per thread); B: 1024 chunks (2 per thread)
  auto load = [&](int kt) {
    const int k0 = kt * BK2;
#pragma unroll
    for (int l = 0; l < 4; ++l) {
      const int c = tid + l * NT2;
      const int plane = c >> 10, rem = c & 1023, row = rem >> 2, kc = (rem & 3) * 8;
      const int gk = k0 + kc;
      u4 v = u4{0u, 0u, 0u, 0u};
      if (m0 + row < p.M && gk < kpad)
        v = *reinterpret_cast<const u4*>(Arow + (unsigned)(row * lda + 2 * k0 + plane * 32 + kc));
      ra[l] = v;
    }
#pragma unroll
    for (int l = 0; l < 2; ++l) {
      const int c = tid + l * NT2;
      const int plane = c >> 9, rem = c & 511, row = rem >> 2, kc = (rem & 3) * 8;
      const int gk = k0 + kc;
      u4 v = u4{0u, 0u, 0u, 0u};
      if (n0 + row < p.N && gk < kpad)
        v = *reinterpret_cast<const u4*>(Brow + (unsigned)(row * ldb + 2 * k0 + plane * 32 + kc));
      rb[l] = v;
    }
  };
  auto store = [&](int buf) {
#pragma unroll
    for (int l = 0; l < 4; ++l) {
      const int c = tid + l * NT2;
      const int plane = c >> 10, rem = c & 1023, row = rem >> 2, kc = (rem & 3) * 8;
      *reinterpret_cast<u4*>(&As[buf][plane][lds_slot(row, kc >> 3)]) = ra[l];
    }
#pragma unroll
    for (int l = 0; l < 2; ++l) {
      const int c = tid + l * NT2;
      const int plane = c >> 9, rem = c & 511, row = rem >> 2, kc = (rem & 3) * 8;
      *reinterpret_cast<u4*>(&Bs[buf][plane][lds_slot(row, kc >> 3)]) = rb[l];
    }
  };
  double* Cw = Cb + (long)(m0 + wm * 64) * p.scm + (long)(n0 + wn * 64) * p.scn;  // wave-uniform
  const int scm = (int)p.scm, scn = (int)p.scn;
  auto flush = [&](bool first) {
    int lx = lane;  // opaque to the compiler: the addresses below are not hoisted out of the K loop
    asm volatile("" : "+v"(lx));
#pragma unroll
    for (int i = 0; i < 4; ++i)
#pragma unroll
      for (int j = 0; j < 4; ++j)
#pragma unroll
        for (int r = 0; r < 4; ++r) {
          const int lm = i * 16 + 4 * (lx >> 4) + r, ln = j * 16 + (lx & 15);
          if (m0 + wm * 64 + lm < p.M && n0 + wn * 64 + ln < p.N) {
            double* c = Cw + (lm * scm + ln * scn);
            const double v = p.alpha * (double)acc[i][j][r];
            if (first)
              *c = (p.beta == 0.0) ? v : v + p.beta * *c;
            else
              *c += v;
          }
          acc[i][j][r] = 0.f;
        }
  };

  const int lr = lane & 15, lg = lane >> 4;
  if (kt0 < nkt) {
    load(kt0);
    store(0);
  }
  __syncthreads();
  for (int kc = kt0; kc < nkt; kc += p.chunk) {
    const int kend = min(nkt, kc + p.chunk);
    for (int kt = kc; kt < kend; ++kt) {
      const int cur = (kt - kt0) & 1;
      if (kt + 1 < nkt) load(kt + 1);
      // all A fragments stay in registers; B fragments are loaded one 16-column panel at a time
      bf8 xa[4][2];
#pragma unroll
      for (int i = 0; i < 4; ++i) {
        const int off = lds_slot(wm * 64 + i * 16 + lr, lg);
        xa[i][0] = *reinterpret_cast<const bf8*>(&As[cur][0][off]);
        xa[i][1] = *reinterpret_cast<const bf8*>(&As[cur][1][off]);
      }
#pragma unroll
      for (int j = 0; j < 4; ++j) {
        const int off = lds_slot(wn * 64 + j * 16 + lr, lg);
        const bf8 bh = *reinterpret_cast<const bf8*>(&Bs[cur][0][off]);
        const bf8 bl = *reinterpret_cast<const bf8*>(&Bs[cur][1][off]);
#pragma unroll
        for (int i = 0; i < 4; ++i) {
          acc[i][j] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(xa[i][1], bh, acc[i][j], 0, 0, 0);
          acc[i][j] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(xa[i][0], bl, acc[i][j], 0, 0, 0);
          acc[i][j] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(xa[i][0], bh, acc[i][j], 0, 0, 0);
        }
      }
      if (kt + 1 < nkt) store(cur ^ 1);
      __syncthreads();
    }
    flush(kc == kt0);
  }
  if (kt0 >= nkt) flush(true);
}

// Buffer descriptor of a wave-uniform range (base, bytes), built from scalar registers: every
// component goes through readfirstlane, so the buffer loads take it straight from SGPRs (left to
// itself the compiler kept parts of it in VGPRs and wrapped each load in a waterfall loop).
__device__ __forceinline__ __amdgpu_buffer_rsrc_t uniform_rsrc(const void* base, int bytes) {
  const uintptr_t b = reinterpret_cast<uintptr_t>(base);
  const uint32_t lo = __builtin_amdgcn_readfirstlane((uint32_t)b);
  const uint32_t hi = __builtin_amdgcn_readfirstlane((uint32_t)(b >> 32));
  void* ub = reinterpret_cast<void*>(((uintptr_t)hi << 32) | lo);
  return __builtin_amdgcn_make_buffer_rsrc(ub, (short)0, __builtin_amdgcn_readfirstlane(bytes), 0x00020000);
}

// 256 x 256 tiles, eight waves of 128 x 64 (two per SIMD, so one wave's fragment reads and barrier
// wait overlap the other's MFMAs), v_mfma_f32_32x32x16_bf16 (4 x 2 fragments of 32 x 32 per wave).
// Each wave stages 64 rows of one operand per K-step as whole 128-byte lines (a row's K-block holds
// hi 32 | lo 32) with eight buffer_load_dwordx4 ... lds (lane l of an instruction writes LDS bytes
// 16l .. 16l + 15, so lanes pick the global chunk that belongs at their swizzled slot; staged as two
// 64-byte planes, each line was fetched by two waves and the step took 3-4 % longer); rows past M
// or N and K-blocks past the padded row read as zero through the buffer range check.  Per K-step:
// wait for this wave's part of the stage, barrier, issue the next stage into the other buffer, then
// two K = 16 halves of fragment reads and 24 MFMAs.  The buffer refilled after a step's barrier was
// read in the step before, whose fragments every wave consumed before reaching that barrier, so one
// barrier per step suffices.  Measured at o40 v360 (ring products 14400^3, ladder 820 x 64980 x 64980, W/Z 1600 x
// 16000 x 129600): 0.49 / 0.41 / 0.40 of the split-BF16x3 peak, against 0.37 / 0.31 / 0.29 with four
// waves of 128 x 128 (one per SIMD); with eight waves the kernel is bound by the rate at which the
// operand stages reach LDS (a copy of it without MFMAs takes as long), not by the matrix cores.
typedef __attribute__((address_space(3))) void lds_void_t;
typedef __attribute__((address_space(3))) char lds_char_t;
typedef float f16v __attribute__((ext_vector_type(16)));
constexpr int BM3 = 256, BN3 = 256, NT3 = 512;

__global__ __launch_bounds__(NT3, 1) void gemm_bf16x3_dma_kernel(LPB p) {
  // [stage][operand][row][64 bf16]: a row's whole K-block (hi 32 | lo 32, one 128-byte line), its
  // eight 16-byte chunks c at slots c ^ ((row >> 1) & 7)
  __shared__ __attribute__((aligned(1024))) unsigned short T[2][2][256 * 64];
  const int tid = threadIdx.x, lane = tid & 63;
  const int wave = __builtin_amdgcn_readfirstlane(tid >> 6);
  const int wm = wave >> 2, wn = wave & 3;  // this wave's 128 x 64 block of the tile
  int tm, tn;
  tile_of_grouped(blockIdx.x, p.tiles_m, p.tiles_n, tm, tn);
  const int m0 = tm * BM3, n0 = tn * BN3;
  const int z = blockIdx.y % p.nb, z1 = blockIdx.y / p.nb;
  const int zs = __builtin_amdgcn_readfirstlane(p.tab1 ? p.tab1[z1] : z1);  // uniform: scalar buffer descriptors
  const int lop = wave >> 2, lq = wave & 3;  // staging: operand (A, B), rows 64 lq .. 64 lq + 63
  const bool isA = lop == 0;
  const unsigned short* base = isA ? p.A + z * p.sa2 + zs * p.sa1 + (long)m0 * p.lda
                                   : p.B + z * p.sb2 + zs * p.sb1 + (long)n0 * p.ldb;
  const int ld = isA ? (int)p.lda : (int)p.ldb;  // row stride (bf16): K-blocks of [hi 32 | lo 32]
  const int rows = min(256, isA ? p.M - m0 : p.N - n0);
  const __amdgpu_buffer_rsrc_t rs = uniform_rsrc(base, rows * ld * 2);
  // lane l of a load writes row l / 8 of an 8-row group, slot l % 8; the chunk that belongs there
  // differs by 4 between even and odd groups (the swizzle's (row >> 1) & 4 term)
  const int r8 = lane >> 3, c0 = (lane & 7) ^ (r8 >> 1);
  const unsigned off_even = (unsigned)(((64 * lq + r8) * ld + c0 * 8) * 2);
  const unsigned off_odd = (unsigned)(((64 * lq + r8) * ld + (c0 ^ 4) * 8) * 2);
  auto issue = [&](int kt, int stage) {
    unsigned oe = off_even, oo = off_odd;
    asm volatile("" : "+v"(oe), "+v"(oo));  // two offset registers across the loop, not one per load
    lds_char_t* dst = (lds_char_t*)(lds_void_t*)&T[stage][lop][64 * lq * 64];
#pragma unroll
    for (int g = 0; g < 8; ++g) {
      const unsigned uni = (unsigned)((8 * g * ld + kt * 64) * 2);  // wave-uniform
      const unsigned off = kt * 64 < ld ? ((g & 1) ? oo : oe) + uni : 0x80000000u;
      __builtin_amdgcn_raw_ptr_buffer_load_lds(rs, (lds_void_t*)(dst + g * 1024), 16, off, 0, 0, 0);
    }
  };
  double* Cb = p.C + z * p.sc2 + (p.part ? z1 : zs) * p.sc1 + blockIdx.z * p.cslice;
  f16v acc[4][2];
#pragma unroll
  for (int i = 0; i < 4; ++i)
#pragma unroll
    for (int j = 0; j < 2; ++j)
#pragma unroll
      for (int q = 0; q < 16; ++q) acc[i][j][q] = 0.f;
  // 32 x 32 fragment: register q of lane l holds C(8 (q / 4) + 4 (l / 32) + q % 4, l % 32)
  auto flush = [&](bool first) {
    // addresses formed here, from a lane index the compiler cannot see through: hoisted out of the
    // K loop they would hold registers across it (and spill)
    int ln = lane;
    asm volatile("" : "+v"(ln));
#pragma unroll
    for (int i = 0; i < 4; ++i)
#pragma unroll
      for (int j = 0; j < 2; ++j)
#pragma unroll
        for (int q = 0; q < 16; ++q) {
          const int gm = m0 + wm * 128 + i * 32 + 8 * (q >> 2) + 4 * (ln >> 5) + (q & 3);
          const int gn = n0 + wn * 64 + j * 32 + (ln & 31);
          if (gm < p.M && gn < p.N) {
            double* cp = Cb + (long)gm * p.scm + (long)gn * p.scn;
            const double v = p.alpha * (double)acc[i][j][q];
            if (first)
              *cp = (p.beta == 0.0) ? v : v + p.beta * *cp;
            else
              add_to(cp, v);
          }
          acc[i][j][q] = 0.f;
        }
    if (first) __builtin_amdgcn_s_waitcnt(0xF70);  // the stores have reached L2
  };
  const int kt0 = blockIdx.z * p.ktps, nkt = min((p.K + 31) / 32, kt0 + p.ktps);
  const int fr = lane & 31, fc = lane >> 5;  // fragment row, K-chunk within a K = 16 half
  const int sw = (fr >> 1) & 7;                // the slot swizzle of every row this lane reads
  if (kt0 < nkt) issue(kt0, 0);
  for (int kc = kt0; kc < nkt; kc += p.chunk) {
    const int kend = min(nkt, kc + p.chunk);
    for (int kt = kc; kt < kend; ++kt) {
      const int cur = (kt - kt0) & 1;
      __builtin_amdgcn_s_waitcnt(0xF70);  // vmcnt(0): this wave's part of stage kt has landed
      asm volatile("" ::: "memory");
      __builtin_amdgcn_s_barrier();  // every wave's has, and every wave has read stage cur ^ 1
      asm volatile("" ::: "memory");  // (its fragments fed the MFMAs of the previous step)
      if (kt + 1 < nkt) issue(kt + 1, cur ^ 1);
#pragma unroll
      for (int sub = 0; sub < 2; ++sub) {
        // hi chunk q = 2 sub + fc at slot q ^ sw, lo chunk 4 + q at (q ^ sw) ^ 4 (sw depends on fr only)
        const int hs = ((2 * sub + fc) ^ sw) * 8, ls = hs ^ 32;
        bf8 xa[4][2], xb[2][2];
#pragma unroll
        for (int i = 0; i < 4; ++i) {
          const int row = (wm * 128 + i * 32 + fr) * 64;
          xa[i][0] = *reinterpret_cast<const bf8*>(&T[cur][0][row + hs]);
          xa[i][1] = *reinterpret_cast<const bf8*>(&T[cur][0][row + ls]);
        }
#pragma unroll
        for (int j = 0; j < 2; ++j) {
          const int row = (wn * 64 + j * 32 + fr) * 64;
          xb[j][0] = *reinterpret_cast<const bf8*>(&T[cur][1][row + hs]);
          xb[j][1] = *reinterpret_cast<const bf8*>(&T[cur][1][row + ls]);
        }
#pragma unroll
        for (int j = 0; j < 2; ++j)
#pragma unroll
          for (int i = 0; i < 4; ++i) {
            acc[i][j] = __builtin_amdgcn_mfma_f32_32x32x16_bf16(xa[i][1], xb[j][0], acc[i][j], 0, 0, 0);
            acc[i][j] = __builtin_amdgcn_mfma_f32_32x32x16_bf16(xa[i][0], xb[j][1], acc[i][j], 0, 0, 0);
            acc[i][j] = __builtin_amdgcn_mfma_f32_32x32x16_bf16(xa[i][0], xb[j][0], acc[i][j], 0, 0, 0);
          }
      }
    }
    flush(kc == kt0);
  }
  if (kt0 >= nkt) flush(true);
}


// The last rows of M (at most 64, the part of a 256-row tile that would be padding) against 256-column
// tiles of B: eight waves of 64 x 32 (both 32-row fragments of one 32-column block each).  A stage
// holds 64 A rows and 256 B rows in the layout of the eight-wave kernel (40 KB of loads instead of
// 64 KB: each wave issues one A and four B loads), and every output element sees the MFMA sequence
// and chunk flushes of that kernel, so the rows it computes are bit for bit the same.
__global__ __launch_bounds__(NT3, 1) void gemm_bf16x3_dma_tail_kernel(LPB p) {
  __shared__ __attribute__((aligned(1024))) unsigned short T[2][2][256 * 64];  // A uses rows 0..63
  const int tid = threadIdx.x, lane = tid & 63;
  const int wave = __builtin_amdgcn_readfirstlane(tid >> 6);
  int tm, tn;
  tile_of_grouped(blockIdx.x, 1, p.tiles_n, tm, tn);
  const int n0 = tn * BN3;
  const int z = blockIdx.y % p.nb, z1 = blockIdx.y / p.nb;
  const int zs = __builtin_amdgcn_readfirstlane(p.tab1 ? p.tab1[z1] : z1);
  const unsigned short* abase = p.A + z * p.sa2 + zs * p.sa1;
  const unsigned short* bbase = p.B + z * p.sb2 + zs * p.sb1 + (long)n0 * p.ldb;
  const int arows = min(64, p.M), brows = min(256, p.N - n0);
  const __amdgpu_buffer_rsrc_t ra = uniform_rsrc(abase, arows * (int)p.lda * 2);
  const __amdgpu_buffer_rsrc_t rb = uniform_rsrc(bbase, brows * (int)p.ldb * 2);
  // whole 128-byte lines in the layout of the eight-wave kernel: a stage is 8 groups of 8 A rows and
  // 32 of 8 B rows; wave w loads A group w and B groups w, w + 8, w + 16, w + 24, all of the parity
  // of w, so one chunk choice per lane serves every load of the wave
  const int r8 = lane >> 3, c = (lane & 7) ^ (r8 >> 1) ^ ((wave & 1) << 2);
  const unsigned a_off = (unsigned)((r8 * (int)p.lda + c * 8) * 2), b_off = (unsigned)((r8 * (int)p.ldb + c * 8) * 2);
  auto issue = [&](int kt, int stage) {
    unsigned ao = a_off, bo = b_off;
    asm volatile("" : "+v"(ao), "+v"(bo));
    const bool have = kt * 64 < (int)p.lda;  // the K-block exists (lda == ldb)
    {
      const unsigned uni = (unsigned)((8 * wave * (int)p.lda + kt * 64) * 2);
      lds_char_t* dst = (lds_char_t*)(lds_void_t*)&T[stage][0][8 * wave * 64];
      __builtin_amdgcn_raw_ptr_buffer_load_lds(ra, (lds_void_t*)dst, 16, have ? ao + uni : 0x80000000u, 0, 0, 0);
    }
#pragma unroll
    for (int j = 0; j < 4; ++j) {
      const int gb = wave + 8 * j;
      const unsigned uni = (unsigned)((8 * gb * (int)p.ldb + kt * 64) * 2);
      lds_char_t* dst = (lds_char_t*)(lds_void_t*)&T[stage][1][8 * gb * 64];
      __builtin_amdgcn_raw_ptr_buffer_load_lds(rb, (lds_void_t*)dst, 16, have ? bo + uni : 0x80000000u, 0, 0, 0);
    }
  };
  double* Cb = p.C + z * p.sc2 + (p.part ? z1 : zs) * p.sc1 + blockIdx.z * p.cslice;
  f16v acc[2];
#pragma unroll
  for (int i = 0; i < 2; ++i)
#pragma unroll
    for (int q = 0; q < 16; ++q) acc[i][q] = 0.f;
  auto flush = [&](bool first) {
#pragma unroll
    for (int i = 0; i < 2; ++i)
#pragma unroll
      for (int q = 0; q < 16; ++q) {
        const int gm = i * 32 + 8 * (q >> 2) + 4 * (lane >> 5) + (q & 3);
        const int gn = n0 + wave * 32 + (lane & 31);
        if (gm < p.M && gn < p.N) {
          double* cp = Cb + (long)gm * p.scm + (long)gn * p.scn;
          const double v = p.alpha * (double)acc[i][q];
          if (first)
            *cp = (p.beta == 0.0) ? v : v + p.beta * *cp;
          else
            add_to(cp, v);
        }
        acc[i][q] = 0.f;
      }
    if (first) __builtin_amdgcn_s_waitcnt(0xF70);  // the stores have reached L2
  };
  const int kt0 = blockIdx.z * p.ktps, nkt = min((p.K + 31) / 32, kt0 + p.ktps);
  const int fr = lane & 31, fc = lane >> 5;
  const int sw = (fr >> 1) & 7;  // the slot swizzle of every row this lane reads
  if (kt0 < nkt) issue(kt0, 0);
  for (int kc = kt0; kc < nkt; kc += p.chunk) {
    const int kend = min(nkt, kc + p.chunk);
    for (int kt = kc; kt < kend; ++kt) {
      const int cur = (kt - kt0) & 1;
      __builtin_amdgcn_s_waitcnt(0xF70);  // vmcnt(0): this wave's part of stage kt has landed
      asm volatile("" ::: "memory");
      __builtin_amdgcn_s_barrier();  // every wave's has, and every wave has read stage cur ^ 1
      asm volatile("" ::: "memory");
      if (kt + 1 < nkt) issue(kt + 1, cur ^ 1);
#pragma unroll
      for (int sub = 0; sub < 2; ++sub) {
        const int hs = ((2 * sub + fc) ^ sw) * 8, ls = hs ^ 32;  // hi and lo chunk slots
        bf8 xa[2][2], xb[2];
#pragma unroll
        for (int i = 0; i < 2; ++i) {
          const int row = (i * 32 + fr) * 64;
          xa[i][0] = *reinterpret_cast<const bf8*>(&T[cur][0][row + hs]);
          xa[i][1] = *reinterpret_cast<const bf8*>(&T[cur][0][row + ls]);
        }
        const int rowb = (wave * 32 + fr) * 64;
        xb[0] = *reinterpret_cast<const bf8*>(&T[cur][1][rowb + hs]);
        xb[1] = *reinterpret_cast<const bf8*>(&T[cur][1][rowb + ls]);
#pragma unroll
        for (int i = 0; i < 2; ++i) {
          acc[i] = __builtin_amdgcn_mfma_f32_32x32x16_bf16(xa[i][1], xb[0], acc[i], 0, 0, 0);
          acc[i] = __builtin_amdgcn_mfma_f32_32x32x16_bf16(xa[i][0], xb[1], acc[i], 0, 0, 0);
          acc[i] = __builtin_amdgcn_mfma_f32_32x32x16_bf16(xa[i][0], xb[0], acc[i], 0, 0, 0);
        }
      }
    }
    flush(kc == kt0);
  }
  if (kt0 >= nkt) flush(true);
}


// FP32, direct to LDS: 256 x 256 tiles, eight waves of 128 x 64 (two per SIMD), v_mfma_f32_16x16x4_f32.
// A stage holds 16 K-values of every tile row (64 bytes; the 16-byte chunk c of row r at slot
// c ^ ((r >> 1) & 3), the 64-byte-row layout of the FP64 direct-to-LDS kernel), four stages (three in flight),
// one barrier per stage after a per-wave vmcnt wait.  Each wave loads 64 rows of one operand per
// stage (four 1 KB buffer_load ... lds; rows past M or N read as zero through the buffer range
// check, the K padding of the shadows is zero).  Each fragment read returns four K-values of a row
// and feeds four MFMAs: lane group g = l / 16 supplies K = 4g + t to MFMA t, identically for A and B.
// FP32 accumulation within K chunks, FP64 across them; split-K slices as in the other kernels.
constexpr int BM4 = 256, BN4 = 256, NT4 = 512, S4 = 4;

__global__ __launch_bounds__(NT4, 1) void gemm_f32_dma_kernel(LP p) {
  __shared__ __attribute__((aligned(1024))) float T[S4][(BM4 + BN4) * 16];
  const int tid = threadIdx.x, lane = tid & 63;
  const int wave = __builtin_amdgcn_readfirstlane(tid >> 6);
  const int wm = wave >> 2, wn = wave & 3;  // this wave's 128 x 64 block of the tile
  int tm, tn;
  tile_of_grouped(blockIdx.x, p.tiles_m, p.tiles_n, tm, tn);
  const int m0 = tm * BM4, n0 = tn * BN4;
  const int z = blockIdx.y % p.nb, z1 = blockIdx.y / p.nb;
  const int zs = __builtin_amdgcn_readfirstlane(p.tab1 ? p.tab1[z1] : z1);  // uniform: scalar buffer descriptors
  // staging: waves 0-3 load rows 64 w .. 64 w + 63 of the A tile, waves 4-7 the same of the B tile
  const bool isA = wave < 4;
  const int r0 = 64 * (wave & 3);
  const float* base = isA ? p.A + z * p.sa2 + zs * p.sa1 + (long)(m0 + r0) * p.lda
                          : p.B + z * p.sb2 + zs * p.sb1 + (long)(n0 + r0) * p.ldb;
  const int ld = isA ? (int)p.lda : (int)p.ldb;  // row stride (floats), a multiple of 32 covering K
  const int rows = max(0, min(64, (isA ? p.M - m0 : p.N - n0) - r0));
  const __amdgpu_buffer_rsrc_t rs = uniform_rsrc(base, rows * ld * 4);
  const int lr = lane >> 2, c = (lane & 3) ^ ((lr >> 1) & 3);  // row in a 16-row block, chunk loaded
  const int lrow0 = (isA ? 0 : BM4) + r0;                         // first LDS row of this wave's rows
  auto issue = [&](int ks, int stage) {
    lds_char_t* dst = (lds_char_t*)(lds_void_t*)&T[stage][lrow0 * 16];
#pragma unroll
    for (int g = 0; g < 4; ++g) {
      const unsigned off = (unsigned)(((g * 16 + lr) * ld + ks * 16 + c * 4) * 4);
      __builtin_amdgcn_raw_ptr_buffer_load_lds(rs, (lds_void_t*)(dst + g * 1024), 16, off, 0, 0, 0);
    }
  };
  double* Cb = p.C + z * p.sc2 + (p.part ? z1 : zs) * p.sc1 + blockIdx.z * p.cslice;
  f4 acc[8][4];
#pragma unroll
  for (int i = 0; i < 8; ++i)
#pragma unroll
    for (int j = 0; j < 4; ++j) acc[i][j] = f4{0.f, 0.f, 0.f, 0.f};
  auto flush = [&](bool first) {
    // addresses formed here from an opaque lane index (hoisted, they would spill)
    int ln = lane;
    asm volatile("" : "+v"(ln));
#pragma unroll
    for (int i = 0; i < 8; ++i)
#pragma unroll
      for (int j = 0; j < 4; ++j)
#pragma unroll
        for (int r = 0; r < 4; ++r) {
          const int gm = m0 + wm * 128 + i * 16 + 4 * (ln >> 4) + r;
          const int gn = n0 + wn * 64 + j * 16 + (ln & 15);
          if (gm < p.M && gn < p.N) {
            double* cp = Cb + (long)gm * p.scm + (long)gn * p.scn;
            const double v = p.alpha * (double)acc[i][j][r];
            if (first)
              *cp = (p.beta == 0.0) ? v : v + p.beta * *cp;
            else
              *cp += v;
          }
          acc[i][j][r] = 0.f;
        }
  };
  // stages of 16 K-values [ks0, nks) of this split-K slice (ktps and chunk count 32-wide K-tiles)
  const int ks0 = blockIdx.z * 2 * p.ktps, nks = min((p.K + 15) / 16, ks0 + 2 * p.ktps);
  const int chunk = 2 * p.chunk;
  const int l16 = lane & 15, q = lane >> 4;
#pragma unroll
  for (int st = 0; st < S4 - 1; ++st)
    if (ks0 + st < nks) issue(ks0 + st, st);
  for (int kc = ks0; kc < nks; kc += chunk) {
    const int kend = min(nks, kc + chunk);
    for (int ks = kc; ks < kend; ++ks) {
      const int st = (ks - ks0) % S4;
      // stage ks has landed once no more than the later stages' loads (four per stage) of this
      // wave are in flight
      const int ahead = min(S4 - 2, nks - 1 - ks);
      if (ahead >= 2)
        __builtin_amdgcn_s_waitcnt(0xF78);  // vmcnt(8)
      else if (ahead == 1)
        __builtin_amdgcn_s_waitcnt(0xF74);  // vmcnt(4)
      else
        __builtin_amdgcn_s_waitcnt(0xF70);  // vmcnt(0)
      __builtin_amdgcn_s_barrier();
      const float* Ts = T[st];
      f4 fa[8], fb[4];
#pragma unroll
      for (int i = 0; i < 8; ++i) {
        const int r = wm * 128 + i * 16 + l16;
        fa[i] = *reinterpret_cast<const f4*>(Ts + r * 16 + 4 * (q ^ ((r >> 1) & 3)));
      }
#pragma unroll
      for (int j = 0; j < 4; ++j) {
        const int r = BM4 + wn * 64 + j * 16 + l16;
        fb[j] = *reinterpret_cast<const f4*>(Ts + r * 16 + 4 * (q ^ ((r >> 1) & 3)));
      }
      // the stage refilled now was last read in the previous iteration, before this barrier
      if (ks + S4 - 1 < nks) issue(ks + S4 - 1, (ks - ks0 + S4 - 1) % S4);
#pragma unroll
      for (int t = 0; t < 4; ++t)
#pragma unroll
        for (int i = 0; i < 8; ++i)
#pragma unroll
          for (int j = 0; j < 4; ++j)
            acc[i][j] = __builtin_amdgcn_mfma_f32_16x16x4f32(fa[i][t], fb[j][t], acc[i][j], 0, 0, 0);
    }
    flush(kc == ks0);
  }
  if (ks0 >= nks) flush(true);
}

// The last rows of M (at most 64) for the FP32 kernel above: 64 x 256 tiles, eight waves of 64 x 32
// (four 16-row by two 16-column fragments each), stages of 64 A rows and 256 B rows (20 KB; each
// wave loads two 16-row blocks of B, waves 0-3 also one of A), four stages.  Every output element
// sees the MFMA sequence and chunk flushes of that kernel, so its rows are bit for bit the same.
__global__ __launch_bounds__(NT4, 1) void gemm_f32_dma_tail_kernel(LP p) {
  __shared__ __attribute__((aligned(1024))) float T[S4][(64 + BN4) * 16];
  const int tid = threadIdx.x, lane = tid & 63;
  const int wave = __builtin_amdgcn_readfirstlane(tid >> 6);
  int tm, tn;
  tile_of_grouped(blockIdx.x, 1, p.tiles_n, tm, tn);
  const int n0 = tn * BN4;
  const int z = blockIdx.y % p.nb, z1 = blockIdx.y / p.nb;
  const int zs = __builtin_amdgcn_readfirstlane(p.tab1 ? p.tab1[z1] : z1);
  const float* abase = p.A + z * p.sa2 + zs * p.sa1;
  const float* bbase = p.B + z * p.sb2 + zs * p.sb1 + (long)n0 * p.ldb;
  const __amdgpu_buffer_rsrc_t ra = uniform_rsrc(abase, min(64, p.M) * (int)p.lda * 4);
  const __amdgpu_buffer_rsrc_t rb = uniform_rsrc(bbase, min(256, p.N - n0) * (int)p.ldb * 4);
  const int lr = lane >> 2, c = (lane & 3) ^ ((lr >> 1) & 3);  // row in a 16-row block, chunk loaded
  const bool loadsA = wave < 4;                                   // three loads per stage, else two
  auto issue = [&](int ks, int stage) {
#pragma unroll
    for (int g = 0; g < 2; ++g) {
      const int blk = 2 * wave + g;
      const unsigned off = (unsigned)(((blk * 16 + lr) * (int)p.ldb + ks * 16 + c * 4) * 4);
      lds_char_t* dst = (lds_char_t*)(lds_void_t*)&T[stage][(64 + blk * 16) * 16];
      __builtin_amdgcn_raw_ptr_buffer_load_lds(rb, (lds_void_t*)dst, 16, off, 0, 0, 0);
    }
    if (loadsA) {
      const unsigned off = (unsigned)(((wave * 16 + lr) * (int)p.lda + ks * 16 + c * 4) * 4);
      lds_char_t* dst = (lds_char_t*)(lds_void_t*)&T[stage][(wave * 16) * 16];
      __builtin_amdgcn_raw_ptr_buffer_load_lds(ra, (lds_void_t*)dst, 16, off, 0, 0, 0);
    }
  };
  double* Cb = p.C + z * p.sc2 + (p.part ? z1 : zs) * p.sc1 + blockIdx.z * p.cslice;
  f4 acc[4][2];
#pragma unroll
  for (int i = 0; i < 4; ++i)
#pragma unroll
    for (int j = 0; j < 2; ++j) acc[i][j] = f4{0.f, 0.f, 0.f, 0.f};
  auto flush = [&](bool first) {
#pragma unroll
    for (int i = 0; i < 4; ++i)
#pragma unroll
      for (int j = 0; j < 2; ++j)
#pragma unroll
        for (int r = 0; r < 4; ++r) {
          const int gm = i * 16 + 4 * (lane >> 4) + r;
          const int gn = n0 + wave * 32 + j * 16 + (lane & 15);
          if (gm < p.M && gn < p.N) {
            double* cp = Cb + (long)gm * p.scm + (long)gn * p.scn;
            const double v = p.alpha * (double)acc[i][j][r];
            if (first)
              *cp = (p.beta == 0.0) ? v : v + p.beta * *cp;
            else
              *cp += v;
          }
          acc[i][j][r] = 0.f;
        }
  };
  const int ks0 = blockIdx.z * 2 * p.ktps, nks = min((p.K + 15) / 16, ks0 + 2 * p.ktps);
  const int chunk = 2 * p.chunk;
  const int l16 = lane & 15, q = lane >> 4;
#pragma unroll
  for (int st = 0; st < S4 - 1; ++st)
    if (ks0 + st < nks) issue(ks0 + st, st);
  for (int kc = ks0; kc < nks; kc += chunk) {
    const int kend = min(nks, kc + chunk);
    for (int ks = kc; ks < kend; ++ks) {
      const int st = (ks - ks0) % S4;
      // stage ks has landed once no more than the later stages' loads of this wave are in flight
      const int ahead = min(S4 - 2, nks - 1 - ks);
      if (loadsA) {
        if (ahead >= 2)
          __builtin_amdgcn_s_waitcnt(0xF76);  // vmcnt(6)
        else if (ahead == 1)
          __builtin_amdgcn_s_waitcnt(0xF73);  // vmcnt(3)
        else
          __builtin_amdgcn_s_waitcnt(0xF70);  // vmcnt(0)
      } else {
        if (ahead >= 2)
          __builtin_amdgcn_s_waitcnt(0xF74);  // vmcnt(4)
        else if (ahead == 1)
          __builtin_amdgcn_s_waitcnt(0xF72);  // vmcnt(2)
        else
          __builtin_amdgcn_s_waitcnt(0xF70);  // vmcnt(0)
      }
      asm volatile("" ::: "memory");
      __builtin_amdgcn_s_barrier();
      asm volatile("" ::: "memory");
      const float* Ts = T[st];
      f4 fa[4], fb[2];
#pragma unroll
      for (int i = 0; i < 4; ++i) {
        const int r = i * 16 + l16;
        fa[i] = *reinterpret_cast<const f4*>(Ts + r * 16 + 4 * (q ^ ((r >> 1) & 3)));
      }
#pragma unroll
      for (int j = 0; j < 2; ++j) {
        const int r = 64 + wave * 32 + j * 16 + l16;
        fb[j] = *reinterpret_cast<const f4*>(Ts + r * 16 + 4 * (q ^ ((r >> 1) & 3)));
      }
      // the stage refilled now was last read in the previous iteration, before this barrier
      if (ks + S4 - 1 < nks) issue(ks + S4 - 1, (ks - ks0 + S4 - 1) % S4);
#pragma unroll
      for (int t = 0; t < 4; ++t)
#pragma unroll
        for (int i = 0; i < 4; ++i)
#pragma unroll
          for (int j = 0; j < 2; ++j)
            acc[i][j] = __builtin_amdgcn_mfma_f32_16x16x4f32(fa[i][t], fb[j][t], acc[i][j], 0, 0, 0);
    }
    flush(kc == ks0);
  }
  if (ks0 >= nks) flush(true);
}

// C_z(m,n) = beta * C_z(m,n) + sum_s part[s][z][m][n], summed in slice order.
__global__ __launch_bounds__(256) void lowp_splitk_reduce(double* C, long scm, long scn, long sc2, long sc1, int nb,
                                                          const int* tab1, double beta, const double* part, int M,
                                                          int N, long total, int split) {
  for (long x = blockIdx.x * 256L + threadIdx.x; x < total; x += (long)gridDim.x * 256) {
    const long mn = (long)M * N;
    const long za = x / mn, r = x % mn;
    const int z = (int)(za % nb), z1 = (int)(za / nb);
    const int zs = tab1 ? tab1[z1] : z1;
    const int m = (int)(r / N), n = (int)(r % N);
    double acc = 0.0;
    for (int sl = 0; sl < split; ++sl) acc += part[(long)sl * total + x];
    double* c = C + z * sc2 + zs * sc1 + m * scm + n * scn;
    *c = (beta == 0.0) ? acc : acc + beta * *c;
  }
}

// Split-K plan for a launch of `tiles` workgroups (one per CU) over nkt K-tiles of 32: slices of
// at least 16 K-tiles, enough of them for one round of 256 workgroups, as the scratch allows.
struct SplitPlan {
  int split = 1, ktps = 0;
};
SplitPlan plan_split(const GemmLP& g, long tiles, int nkt) {
  SplitPlan sp;
  sp.ktps = nkt;
  const long outs = (long)g.M * g.N * g.nb * g.nb1;
  if (!g.ws || tiles >= 192 || nkt < 32) return sp;
  long n = std::min<long>({(256 + tiles - 1) / tiles, (long)nkt / 16, g.ws_elems / std::max<long>(outs, 1)});
  if (n < 2) return sp;
  sp.ktps = (int)((nkt + n - 1) / n);
  sp.split = (nkt + sp.ktps - 1) / sp.ktps;
  return sp;
}

}  // namespace



hipError_t to_lowp_2d(int prec, float* out, long ldo, const double* in, long ldi, long rows, long cols,
                      hipStream_t s) {
  const long total = rows * ldo;
  if (total <= 0) return hipSuccess;
  if (bounds_checking() && !(range_ok(out, 0, total - 1, 4, "lowp shadow") &&
                             range_ok(in, 0, (rows - 1) * ldi + cols - 1, 8, "lowp source")))
    return hipErrorInvalidValue;
  if (dry_run()) return hipSuccess;
  // eight columns per thread where the rows allow 16-byte accesses (ldo is a multiple of 32)
  const bool v8 = (reinterpret_cast<uintptr_t>(in) & 15) == 0 && (reinterpret_cast<uintptr_t>(out) & 15) == 0 &&
                  (ldi & 1) == 0 && (ldo & 31) == 0;
  long g = ((v8 ? total / 8 : total) + 255) / 256;
  if (g > 8192) g = 8192;
  if (prec == kPrecBF16x3) {
    if (v8)
      hipLaunchKernelGGL(split_bf16_2d_v8_kernel, dim3((unsigned)g), dim3(256), 0, s,
                         reinterpret_cast<unsigned short*>(out), ldo, in, ldi, rows, cols);
    else
      hipLaunchKernelGGL(split_bf16_2d_kernel, dim3((unsigned)g), dim3(256), 0, s,
                         reinterpret_cast<unsigned short*>(out), ldo, in, ldi, rows, cols);
  } else {
    if (v8)
      hipLaunchKernelGGL(cvt_f32_2d_v8_kernel, dim3((unsigned)g), dim3(256), 0, s, out, ldo, in, ldi, rows, cols);
    else
      hipLaunchKernelGGL(cvt_f32_2d_kernel, dim3((unsigned)g), dim3(256), 0, s, out, ldo, in, ldi, rows, cols);
  }
  return hipGetLastError();
}

hipError_t gemm_lowp(const GemmLP& g, hipStream_t s) {
  if (g.M <= 0 || g.N <= 0 || g.nb <= 0 || g.nb1 <= 0) return hipSuccess;
  if (g.K <= 0 || (long)g.nb * g.nb1 > 65535 || (g.prec != kPrecFP32 && g.prec != kPrecBF16x3))
    return hipErrorInvalidValue;
  const bool bf = (g.prec == kPrecBF16x3);
  // bf16: interleaved rows; the row strides are equal multiples of 64 and cover K
  if (bf && (((g.lda | g.ldb | g.sa2 | g.sb2 | g.sa1 | g.sb1) & 63) || g.lda != g.ldb || g.lda / 2 < g.K))
    return hipErrorInvalidValue;
  const long nz1 = g.tab1 ? g.tab1_max + 1 : g.nb1;  // operand blocks of the outer batch level
  if (bounds_checking()) {
    // bf16: every staged chunk stays inside its padded row
    const long la = (long)(g.M - 1) * g.lda + (bf ? g.lda - 1 : g.K - 1) + (long)(g.nb - 1) * g.sa2 + (nz1 - 1) * g.sa1;
    const long lb = (long)(g.N - 1) * g.ldb + (bf ? g.ldb - 1 : g.K - 1) + (long)(g.nb - 1) * g.sb2 + (nz1 - 1) * g.sb1;
    long lo = 0, hi = 0;
    const long dc[4] = {(long)(g.M - 1) * g.scm, (long)(g.N - 1) * g.scn, (long)(g.nb - 1) * g.sc2, (nz1 - 1) * g.sc1};
    for (long d : dc) {
      if (d < 0) lo += d; else hi += d;
    }
    const size_t el = bf ? 2 : 4;
    if (!(range_ok(g.A, 0, la, el, "lowp A") && range_ok(g.B, 0, lb, el, "lowp B") && range_ok(g.C, lo, hi, 8, "lowp C") &&
          (!g.ws || range_ok(g.ws, 0, g.ws_elems - 1, 8, "lowp split-K scratch"))))
      return hipErrorInvalidValue;
  }
  if (dry_run()) return hipSuccess;
  // 8192 of K per FP32 chunk in both modes (2048 for FP32 measured 15 % slower at o40 v360 for no
  // change in the refined solves; the flush of the FP64 tile is the cost)
  const int chunk = g.chunk_ktiles > 0 ? g.chunk_ktiles : 256;
  const int nbz = g.nb * g.nb1;                       // grid.y
  const int nbd = g.per_block ? g.nb : nbz;            // the batch the kernel and split choices see
  // the batch and output fields shared by both parameter blocks
  auto common = [&](auto& p) {
    p.M = g.M;
    p.N = g.N;
    p.K = g.K;
    p.lda = g.lda;
    p.sa2 = g.sa2;
    p.ldb = g.ldb;
    p.sb2 = g.sb2;
    p.C = g.C;
    p.scm = g.scm;
    p.scn = g.scn;
    p.sc2 = g.sc2;
    p.alpha = g.alpha;
    p.beta = g.beta;
    p.chunk = chunk;
    p.cslice = 0;
    p.nb = g.nb;
    p.part = 0;
    p.tab1 = g.tab1;
    p.sa1 = g.sa1;
    p.sb1 = g.sb1;
    p.sc1 = g.sc1;
  };
  // split launches write partial tiles [split][nb1][nb][M][N] into the scratch
  auto to_partials = [&](auto& p) {
    p.C = g.ws;
    p.scm = g.N;
    p.scn = 1;
    p.sc2 = (long)g.M * g.N;
    p.sc1 = (long)g.M * g.N * g.nb;
    p.cslice = (long)g.M * g.N * nbz;
    p.beta = 0.0;
    p.part = 1;
  };
  auto reduce = [&](int split) {
    const long total = (long)g.M * g.N * nbz;
    hipLaunchKernelGGL(lowp_splitk_reduce, dim3((unsigned)std::min<long>((total + 255) / 256, 4096)), dim3(256), 0, s,
                       g.C, g.scm, g.scn, g.sc2, g.sc1, g.nb, g.tab1, g.beta, g.ws, g.M, g.N, total, split);
  };
  if (bf) {
    LPB p;
    common(p);
    p.A = reinterpret_cast<const unsigned short*>(g.A);
    p.B = reinterpret_cast<const unsigned short*>(g.B);
    const int nkt = (g.K + 31) / 32;
    // buffer descriptors cover one tile's rows: 256 * ld bf16 must stay below 2^31 bytes
    const int mdec = g.m_dec > 0 ? g.m_dec : g.M;
    const long t3 = (long)((mdec + BM3 - 1) / BM3) * ((g.N + BN3 - 1) / BN3) * nbd;
    const bool dma_ok = 512L * g.lda < (1L << 31);
    // from 128 tiles on (half a round) the eight-wave kernel beats the register-staged one even
    // with the round partly idle; from 64 tiles with scratch, K is cut into slices so that the
    // tiles of all slices fill one round (partial tiles summed in slice order)
    int dsplit = 0;
    if (dma_ok && t3 >= 128) {
      dsplit = 1;
    } else if (dma_ok && g.ws && t3 >= 64) {
      const long outs = (long)g.M * g.N * g.nb * g.nb1;
      const long n = std::min<long>({256 / t3, (long)nkt / 16, g.ws_elems / std::max<long>(outs, 1)});
      if (n >= 2) dsplit = (int)n;
    }
    if (dsplit > 0) {
      p.tiles_m = (g.M + BM3 - 1) / BM3;
      p.tiles_n = (g.N + BN3 - 1) / BN3;
      p.ktps = (nkt + dsplit - 1) / dsplit;
      const int split = (nkt + p.ktps - 1) / p.ktps;
      const int mtail = g.M % BM3;
      if (tail_tiles_enabled() && split == 1 && mtail > 0 && mtail <= 64 && g.M > BM3) {
        // the last, mostly padding, row tile as 64-row tail tiles of 40 KB stages (about 5/8 of a
        // full workgroup's time) after the full row tiles, when that takes fewer rounds of 256
        const long full = (long)(g.M / BM3) * p.tiles_n * nbz, tail = (long)p.tiles_n * nbz;
        const double r_all = (double)((full + tail + 255) / 256);
        const double r_split = (double)((full + 255) / 256) + 0.625 * (double)((tail + 255) / 256);
        if (r_split < r_all) {
          LPB pt = p;
          p.M = g.M - mtail;
          p.tiles_m = p.M / BM3;
          pt.A += (long)p.M * g.lda;
          pt.C += (long)p.M * g.scm;
          pt.M = mtail;
          pt.tiles_m = 1;
          hipLaunchKernelGGL(gemm_bf16x3_dma_kernel, dim3(p.tiles_m * p.tiles_n, nbz, 1), dim3(NT3), 0, s, p);
          hipLaunchKernelGGL(gemm_bf16x3_dma_tail_kernel, dim3(pt.tiles_n, nbz, 1), dim3(NT3), 0, s, pt);
          return hipGetLastError();
        }
      }
      if (split > 1) to_partials(p);
      hipLaunchKernelGGL(gemm_bf16x3_dma_kernel, dim3(p.tiles_m * p.tiles_n, nbz, split), dim3(NT3), 0, s, p);
      if (split > 1) reduce(split);
      return hipGetLastError();
    }
    p.tiles_m = (g.M + BM2 - 1) / BM2;
    p.tiles_n = (g.N + BN2 - 1) / BN2;
    const SplitPlan sp = plan_split(g, (long)p.tiles_m * p.tiles_n * nbd, nkt);
    p.ktps = sp.ktps;
    if (sp.split > 1) to_partials(p);
    hipLaunchKernelGGL(gemm_bf16x3_kernel, dim3(p.tiles_m * p.tiles_n, nbz, sp.split), dim3(NT2), 0, s, p);
    if (sp.split > 1) reduce(sp.split);
    return hipGetLastError();
  }
  LP p;
  common(p);
  p.A = g.A;
  p.B = g.B;
  {
    // the direct-to-LDS kernel for the same sizes as the split-BF16x3 one (16-byte aligned rows,
    // zero-padded to whole K stages of 16)
    const int mdec = g.m_dec > 0 ? g.m_dec : g.M;
    const long t4 = (long)((mdec + BM4 - 1) / BM4) * ((g.N + BN4 - 1) / BN4) * nbd;
    const int nkt = (g.K + 31) / 32;
    const long k16 = (g.K + 15L) / 16 * 16;
    auto al16 = [](const void* x) { return (reinterpret_cast<uintptr_t>(x) & 15) == 0; };
    const bool dma_ok = al16(g.A) && al16(g.B) && ((g.lda | g.ldb | g.sa2 | g.sb2 | g.sa1 | g.sb1) & 3) == 0 &&
                        g.lda >= k16 && g.ldb >= k16 && 256L * std::max(g.lda, g.ldb) < (1L << 31);
    int dsplit = 0;
    if (dma_ok && t4 >= 128) {
      dsplit = 1;
    } else if (dma_ok && g.ws && t4 >= 64) {
      const long outs = (long)g.M * g.N * g.nb * g.nb1;
      const long n = std::min<long>({256 / t4, (long)nkt / 16, g.ws_elems / std::max<long>(outs, 1)});
      if (n >= 2) dsplit = (int)n;
    }
    if (dsplit > 0) {
      p.tiles_m = (g.M + BM4 - 1) / BM4;
      p.tiles_n = (g.N + BN4 - 1) / BN4;
      p.ktps = (nkt + dsplit - 1) / dsplit;
      const int split = (nkt + p.ktps - 1) / p.ktps;
      const int mtail = g.M % BM4;
      // (the tail kernel's B range spans 256 rows of one buffer descriptor)
      if (tail_tiles_enabled() && split == 1 && mtail > 0 && mtail <= 64 && g.M > BM4 && 1024L * g.ldb < (1L << 31)) {
        // the last row tile as 64-row tail tiles, as for split-BF16x3 (20 KB stages: about 5/8 of
        // a full workgroup's time)
        const long full = (long)(g.M / BM4) * p.tiles_n * nbz, tail = (long)p.tiles_n * nbz;
        const double r_all = (double)((full + tail + 255) / 256);
        const double r_split = (double)((full + 255) / 256) + 0.625 * (double)((tail + 255) / 256);
        if (r_split < r_all) {
          LP pt = p;
          p.M = g.M - mtail;
          p.tiles_m = p.M / BM4;
          pt.A += (long)p.M * g.lda;
          pt.C += (long)p.M * g.scm;
          pt.M = mtail;
          pt.tiles_m = 1;
          hipLaunchKernelGGL(gemm_f32_dma_kernel, dim3(p.tiles_m * p.tiles_n, nbz, 1), dim3(NT4), 0, s, p);
          hipLaunchKernelGGL(gemm_f32_dma_tail_kernel, dim3(pt.tiles_n, nbz, 1), dim3(NT4), 0, s, pt);
          return hipGetLastError();
        }
      }
      if (split > 1) to_partials(p);
      hipLaunchKernelGGL(gemm_f32_dma_kernel, dim3(p.tiles_m * p.tiles_n, nbz, split), dim3(NT4), 0, s, p);
      if (split > 1) reduce(split);
      return hipGetLastError();
    }
  }
  p.tiles_m = (g.M + BM - 1) / BM;
  p.tiles_n = (g.N + BN - 1) / BN;
  const SplitPlan sp = plan_split(g, (long)p.tiles_m * p.tiles_n * nbd, (g.K + 31) / 32);
  p.ktps = sp.ktps;
  if (sp.split > 1) to_partials(p);
  hipLaunchKernelGGL(gemm_lowp_kernel, dim3(p.tiles_m * p.tiles_n, nbz, sp.split), dim3(NT), 0, s, p);
  if (sp.split > 1) reduce(sp.split);
  return hipGetLastError();
}

hipError_t to_lowp_pm(int prec, float* out, long ldo, const double* V, long ldv, long vrows, const int* pm, long Tv,
                      hipStream_t s) {
  const long total = 2 * Tv * ldo;
  if (total <= 0) return hipSuccess;
  if (ldo < Tv || ldv < Tv || vrows < Tv) return hipErrorInvalidValue;
  if (bounds_checking() && !(range_ok(out, 0, total - 1, 4, "vvvv shadow") &&
                             range_ok(V, 0, (vrows - 1) * ldv + Tv - 1, 8, "full vvvv") &&
                             range_ok(pm, 0, Tv - 1, 4, "pair rows")))
    return hipErrorInvalidValue;
  if (dry_run()) return hipSuccess;
  long g = (total + 255) / 256;
  if (g > 8192) g = 8192;
  if (prec == kPrecBF16x3)
    hipLaunchKernelGGL(lowp_pm_kernel<true>, dim3((unsigned)g), dim3(256), 0, s,
                       reinterpret_cast<unsigned short*>(out), nullptr, ldo, V, ldv, pm, Tv);
  else
    hipLaunchKernelGGL(lowp_pm_kernel<false>, dim3((unsigned)g), dim3(256), 0, s, nullptr, out, ldo, V, ldv, pm, Tv);
  return hipGetLastError();
}

hipError_t to_lowp_t(int prec, float* out, long ldo, const double* in, long ldi, long rows, long cols, hipStream_t s) {
  if (rows <= 0 || cols <= 0) return hipSuccess;
  if ((ldo & 31) || ldo < cols || ldi < rows || (rows + 31) / 32 > 0x7fffffffL || ldo / 32 > 65535)
    return hipErrorInvalidValue;
  if (bounds_checking() && !(range_ok(out, 0, rows * ldo - 1, 4, "transposed shadow") &&
                             range_ok(in, 0, (cols - 1) * ldi + rows - 1, 8, "transposed shadow source")))
    return hipErrorInvalidValue;
  if (dry_run()) return hipSuccess;
  const dim3 grid((unsigned)((rows + 31) / 32), (unsigned)(ldo / 32));
  if (prec == kPrecBF16x3)
    hipLaunchKernelGGL(lowp_t_kernel<true>, grid, dim3(256), 0, s, (void*)out, ldo, in, ldi, rows, cols);
  else
    hipLaunchKernelGGL(lowp_t_kernel<false>, grid, dim3(256), 0, s, (void*)out, ldo, in, ldi, rows, cols);
  return hipGetLastError();
}

}  // namespace ascc
