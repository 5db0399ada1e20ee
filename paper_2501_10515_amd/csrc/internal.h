// Internal declarations shared by the libascc translation units (not part of the C ABI).
#pragma once

#include <hip/hip_runtime.h>

#include <cstddef>
#include <cstdint>
#include <string>

struct ascc_ints;
struct ascc_diis;
struct ascc_opts;
struct ascc_result;

namespace ascc {

// Status used inside the library; converted to the ASCC_E_* codes at the ABI boundary.
struct Error {
  int code;
  std::string msg;
};

void set_error(const std::string& msg);

// Optional host-side bounds checking of every strided launch (environment variable
// ASCC_CHECK_BOUNDS=1): device buffers are registered with their sizes, and each GEMM /
// permute launch first verifies that the lowest and highest element it can touch lie in one
// registered buffer.  A violation is reported as an error instead of being launched.
bool bounds_checking();
// Dry run (environment variable ASCC_DRY_RUN=1, implies bounds checking): device
// allocations return unbacked addresses and no kernel, copy or synchronisation is issued,
// so the complete host-side launch sequence -- every stride and extent -- can be validated
// on a machine without a GPU.
bool dry_run();
void register_buffer(const void* p, size_t bytes);
void unregister_buffer(const void* p);
// true if [base + lo, base + hi] (in elements of `elem` bytes) lies inside a registered buffer
bool range_ok(const void* base, long lo, long hi, size_t elem, const char* what);

// ---------------------------------------------------------------------------------------
// Strided batched FP64 GEMM on the matrix cores:
//   C_z(m,n) = alpha * sum_{r < nred} sum_k A_{z,r}(m,k) B_{z,r}(k,n) + beta * C_z(m,n)
// Every operand is a general strided 2-D view, e.g. A(m,k) = A[m*sam + k*sak].  The batch
// index z runs over nb1 x nb2 (z1 outer, z2 inner) with one stride per level; the reduction
// index r (nred >= 1) adds products of further (A, B) pairs into the same C.
// beta == 0 never reads C.
struct Gemm {
  int M = 0, N = 0, K = 0;
  const double* A = nullptr;
  long sam = 0, sak = 0, sa1 = 0, sa2 = 0, sar = 0;
  const double* B = nullptr;
  long sbk = 0, sbn = 0, sb1 = 0, sb2 = 0, sbr = 0;
  double* C = nullptr;
  long scm = 0, scn = 0, sc1 = 0, sc2 = 0;
  double alpha = 1.0, beta = 0.0;
  int nb1 = 1, nb2 = 1, nred = 1;
  // Optional scratch for split-K: when the output has too few tiles to fill the chip, the
  // (reduction x K) iteration space is cut into slices whose partial tiles land here and
  // are then summed in a fixed order (deterministic).  nullptr disables splitting.
  double* ws = nullptr;
  long ws_elems = 0;
  // Optional table of batch level 1: grid index z1 takes operand block tab1[z1] (device array of
  // nb1 entries, each at most tab1_max); nullptr: block z1.
  const int* tab1 = nullptr;
  int tab1_max = 0;
  // tile and split-K choices as for one block of batch level 1 (the same summation order for
  // each block whatever nb1 is, as long as the split-K scratch holds the partials of every block)
  bool per_block = false;
  // C = A B with B(k, n) = A(n, k) is symmetric: when M == N, beta == 0 and the rows qualify for
  // the direct-to-LDS kernel, only the tiles on and below the diagonal are computed and the strict
  // upper triangle is copied from the lower one (otherwise the full product)
  bool lower = false;
};

// Batch level of the particle-particle ladder: n operand blocks (A, V and C offset by sa, sv, sc
// elements per block; the pair-row table, which depends on v only, is shared), block z taken from
// tab[z] when tab is given (entries at most tab_max).
struct LadderBatch {
  int n = 1;
  const int* tab = nullptr;
  int tab_max = 0;
  long sa = 0, sv = 0, sc = 0;
};

// Convenience constructors for row-major matrices:
//   A is M x K with leading dimension lda (ta = false) or stored K x M (ta = true), etc.
Gemm gemm_rm(int M, int N, int K, double alpha, const double* A, long lda, bool ta, const double* B, long ldb,
             bool tb, double beta, double* C, long ldc);

hipError_t gemm_f64(const Gemm& g, hipStream_t s);

// Particle-particle ladder over pair indices, both halves h = 0 (+), 1 (-) in one launch:
//   C[h][m][n] = sum_k A[h][m][k] * Vh(n, k),   m < M;  n, k < Tv
// A and C are row-major [2][M][Tv].  pm == nullptr: Vh is stored, row-major [2][Tv][Tv] (V).
// Otherwise V is the full (ac|bd) matrix in pair order (see pack_full), [vrows = v^2][ldv], and
// Vh(n, k) = V[n][k] +- V[pm[n]][k] = (ac|bd) +- (ad|bc) for n = (a <= b), k = (c <= d) (on the
// diagonal k = (c,c) this is twice the packed V+, so A carries half the diagonal t+).
// No split-K, so every output is summed in the same order whatever M is.
hipError_t gemm_f64_ladder(int M, int Tv, const double* A, const double* V, long ldv, long vrows, const int* pm,
                           double* C, hipStream_t s, const LadderBatch& lb = LadderBatch());

// Low-precision contraction with FP64 result (gemm_lowp.hip):
//   C_z(m,n) = alpha * sum_k A_z[m*lda + k] * B_z[n*ldb + k] + beta * C_z(m,n)
// A, B are FP32 (K contiguous); prec selects FP32 MFMA or split-BF16x3 MFMA; FP32 accumulation
// inside chunks of chunk_ktiles K-tiles (32 wide; 0 = the default of the precision: 64 for FP32,
// 256 for split-BF16x3), FP64 accumulation across chunks.
constexpr int kPrecFP64 = 0, kPrecFP32 = 1, kPrecBF16x3 = 2;
struct GemmLP {
  int M = 0, N = 0, K = 0, nb = 1;
  const float* A = nullptr;
  long lda = 0, sa2 = 0;
  const float* B = nullptr;
  long ldb = 0, sb2 = 0;
  double* C = nullptr;
  long scm = 0, scn = 1, sc2 = 0;
  double alpha = 1.0, beta = 0.0;
  int prec = kPrecFP32;
  int chunk_ktiles = 0;
  // BF16X3: A and B are interleaved splits (see to_lowp_2d); lda, ldb, sa2, sb2 count bf16
  // elements (lda == ldb, multiples of 64, lda / 2 >= K)
  // Optional split-K scratch: an output with too few tiles to fill the chip has its K range cut
  // into slices (each at least 512 of K, each FP32 chunk starting at its slice's start) whose
  // FP64 partial tiles land here and are then summed in slice order (deterministic).
  double* ws = nullptr;
  long ws_elems = 0;
  // Optional outer batch level over operand blocks: nb1 blocks at strides sa1, sb1 (in the units of
  // lda) and sc1 (FP64 elements); block z1 taken from tab1[z1] when tab1 is given (entries at most
  // tab1_max).
  int nb1 = 1;
  long sa1 = 0, sb1 = 0, sc1 = 0;
  const int* tab1 = nullptr;
  int tab1_max = 0;
  bool per_block = false;  // kernel and split-K choices as for one outer block (see Gemm)
  // rows that decide the kernel (0: M): operands stacking the rows of several states pass one
  // state's rows, so that every state's rows are summed exactly as when it is alone
  int m_dec = 0;
};
hipError_t gemm_lowp(const GemmLP& g, hipStream_t s);
// Low-precision shadow of a row-major FP64 matrix with the leading dimension padded to ldo
// (a multiple of 32; padding zeroed).  FP32: one float per element, row stride ldo.  BF16X3: the
// same bytes as bf16, row stride 2 ldo, each K-block of 32 stored as hi[32] then lo[32] with
// hi = RNE_bf16(x), lo = RNE_bf16(x - hi).
hipError_t to_lowp_2d(int prec, float* out, long ldo, const double* in, long ldi, long rows, long cols, hipStream_t s);
// Transposed shadow: out row r (r < rows) = column r of in ([cols][ldi] FP64), padded to ldo.
hipError_t to_lowp_t(int prec, float* out, long ldo, const double* in, long ldi, long rows, long cols, hipStream_t s);
// Packed vvvv halves [2][Tv][ldo] (zero padded) in low precision, formed from the full (ac|bd)
// matrix in pair order [vrows][ldv] as gemm_f64_ladder forms them (V[n][k] +- V[pm[n]][k]).
hipError_t to_lowp_pm(int prec, float* out, long ldo, const double* V, long ldv, long vrows, const int* pm, long Tv,
                      hipStream_t s);
inline long lowp_ld(long k) { return (k + 31) / 32 * 32; }

// Hand-over test of a low-precision bulk phase: the residual norm has reached the rounding floor
// of the contractions when it has not set a new minimum (by 1%) for kPatience iterations.  Eight,
// not fewer: the excited-state (ASCC) iteration has plateaus of several iterations well above the
// floor, and a low-precision iteration costs less than half an FP64 one, so waiting longer is
// cheap while an early hand-over leaves most of the work to FP64.
struct LowpStall {
  static constexpr int kPatience = 8;
  double best = 0.0;
  int since = 0;
  bool stalled(double rnorm) {
    if (since == 0 && best == 0.0) best = rnorm;
    if (rnorm < 0.99 * best) {
      best = rnorm;
      since = 0;
    } else {
      ++since;
    }
    return since >= kPatience;
  }
};

// ---------------------------------------------------------------------------------------
// Element-wise kernels (elementwise.hip).

// out[i0,i1,i2,i3] = c0*out + sum_t coef[t] * in_t[i0*s_t0 + i1*s_t1 + i2*s_t2 + i3*s_t3]
// for up to four strided inputs (an input with coef 0 is not read; c0 == 0 never reads out).
struct Perm4In {
  const double* p = nullptr;
  long s[4] = {0, 0, 0, 0};
  double coef = 0.0;
};
hipError_t permute4(double* out, const int dims[4], double c0, const Perm4In* in, int nin, hipStream_t s);
// Same with an explicitly strided output view.
hipError_t permute4_strided(double* out, const long ostr[4], const int dims[4], double c0, const Perm4In* in,
                            int nin, hipStream_t s);

// Assembly of the doubles residual from the ring, ladder and E-term pieces (formula at the kernel).
hipError_t assemble_r2(double* r2, const double* g1, const double* rl, const double* em, const double* p1,
                       const double* p2, int no, int nv, hipStream_t s);

// Pair packing of the particle-particle ladder (p(i,j) = row-major index of i <= j).
// Full (ac|bd) storage in pair order R(a,b) (a <= b: p(a,b); a > b: T(v) + strict index of (b,a)):
// pm[n] = R(b,a) for pair n = (a <= b); pack_full scatters W[a - a0][b][c][d] = (ac|bd), a0 <= a < a1,
// to V[R(a,b)][R(c,d)].
hipError_t pair_minus_rows(int* pm, int v, hipStream_t s);
hipError_t pack_full(double* V, const double* W, int a0, int a1, int v, hipStream_t s);
// t+ rows -> tplus[T(o)][T(v)], t- rows -> tminus[T(o)][T(v)] (and back for R+-)
hipError_t pack_tpm(double* tplus, double* tminus, const double* t2, int o, int v, double dscale, hipStream_t s);
hipError_t unpack_rpm(double* RL, const double* Rplus, const double* Rminus, int o, int v, hipStream_t s);
hipError_t pack_vvvv(double* Vp, const double* W, int a0, int a1, int v, hipStream_t s);  // rows a0 <= a < a1

// r1[i][a] += Fhat[no+a][i]
hipError_t add_fvo(double* r1, const double* fhat, int no, int nv, hipStream_t s);

// T1 dressing of nb stacked n x n matrices S (n = o + v) given Tc[z][x][i] = sum_a S[z][x][o+a] t1[i][a]:
//   D[p][q] = b(p, q) - [p >= o] sum_{i<o} t1[i][p-o] b(i, q),  b(x, q) = S[x][q] + [q < o] Tc[x][q].
hipError_t dress_apply(double* D, const double* S, const double* Tc, const double* t1, int o, int v, int nb,
                       hipStream_t s);

// x -> (1 + c E_hp) x (1 - c E_hp) in place on nb stacked n x n matrices (E_hp: one at row h, column p).
hipError_t onebody_transform(double* X, long nb, int n, int h, int p, double c, hipStream_t s);
// A cross index set: over the n = no * nv indices r = i * nv + a, the members with i == h or
// a == pa (m = no + nv - 1 of them), listed compactly as (h, 0 .. nv-1), then (i, pa) for i != h
// ascending.  With (no, nv, h, pa) = (o, v, hole, particle) it is the set of (i, a) rows of an
// ov x ov matrix that touch a primary orbital; (o, o, h, h) and (v, v, pa, pa) are the pair
// indices ij and ab that do.
struct Cross {
  int no = 1, nv = 1, h = 0, pa = 0;
  __host__ __device__ long n() const { return (long)no * nv; }
  __host__ __device__ long m() const { return (long)no + nv - 1; }
};
//   cross_gather_rows: dst[k][c] = src[row k of X][c], c < ncols (zero_diag: the corner entry
//                      at row and column h*nv + pa written as 0).
//   cross_gather_cols: dst[r][k] = src[r][col k of X] for k < m, 0 for m <= k < ldd; zero_rows:
//                      rows r that are members of *zero_rows written as 0.
//   cross_scatter_add_rows / _cols / _block: the inverse placements, dst += alpha * src.
//   cross_rows_without_corner: dst[k][c] = Y[row k][c] - [row k == hp] T[hp][hp] K[hp][c] for
//                      square X.n() x X.n() operands (the cross rows of T' K, T' = T minus its
//                      corner entry, from Y = T K).
//   em_cross_column:   EM[ij][a][b] += tc[ij][v + a - [a > pa]] * A[b][pa] for a != pa.
// mixed_doubles: dst = src on the mixed doubles (index set holds h or pa, not all primary), else 0.
hipError_t cross_gather_rows(double* dst, long ldd, const double* src, long lds, long src_rows, long ncols,
                             const Cross& X, bool zero_diag, hipStream_t s);
hipError_t cross_gather_cols(double* dst, long ldd, const double* src, long lds, long nrows, const Cross& X,
                             const Cross* zero_rows, hipStream_t s);
hipError_t cross_scatter_add_rows(double* dst, long ldd, long dst_rows, const double* src, long lds, long ncols,
                                  double alpha, const Cross& X, hipStream_t s);
hipError_t cross_scatter_add_cols(double* dst, long ldd, long nrows, const double* src, long lds, double alpha,
                                  const Cross& X, hipStream_t s);
hipError_t cross_scatter_add_block(double* dst, long ldd, const double* src, long lds, double alpha, const Cross& X,
                                   hipStream_t s);
hipError_t cross_rows_without_corner(double* dst, long ldd, const double* Y, const double* T, const double* K,
                                     const Cross& X, hipStream_t s);
hipError_t em_cross_column(double* em, const double* tc, long ldt, const double* A, int o, int v, int pa,
                           hipStream_t s);
hipError_t mixed_doubles(double* dst, const double* src, int o, int v, int h, int pa, hipStream_t s);
// e0[0] = sum_{i<o} (h[i * hs] + f[i * fs]) (hlen, flen: elements of h and f, for the bounds check).
hipError_t reference_energy(double* e0, const double* h, long hs, long hlen, const double* f, long fs, long flen,
                            int o, hipStream_t s);
// t1 = 0, t2 = 0 except t1[h][a] = s1 and t2[h][h][a][a] = s2.
hipError_t initial_guess(double* t1, double* t2, int no, int nv, int h, int a, double s1, double s2, hipStream_t s);

// J[Q] = sum_k Bh[Q][k][k]
hipError_t diag_trace(double* J, const double* Bh, int naux, int n, int no, hipStream_t s);

// Deterministic two-stage energy reduction:
//   e = sum_{ijab} (t2 + t1_ia t1_jb) L[ijab] + 2 sum_ia f_ia t1_ia
hipError_t energy(double* e, double* partial, const double* t1, const double* t2, const double* Lijab,
                  const double* fov, int no, int nv, hipStream_t s);

// DIIS device state (one per amplitude set), kept in device memory.
constexpr int kMaxDiis = 16;
struct DiisState {
  int nvec;     // stored pairs
  int head;     // slot that receives the next pair
  int calls;    // update calls so far
  int flags;    // last call's flags
  double e_prev;
  int has_prev;
  int pad_;
  double Bm[kMaxDiis * kMaxDiis];  // error-vector overlaps, indexed by slot
  double coef[kMaxDiis];           // extrapolation coefficients by slot (0 for unused)
  int slot_age[kMaxDiis];          // insertion counter of each slot (-1 empty)
  int counter;
  int pad2_;
};

struct UpdateArgs {
  double* t1;
  double* t2;
  const double* r1;
  const double* r2;
  const double* e;
  const double* eps;  // diagonal of the Fock matrix [n]
  double* hist_t;     // [m][len]
  double* hist_e;     // [m][len]
  double* partial;    // [nblk][2 + m] reduction scratch
  DiisState* st;
  double* stats;
  int no, nv, m;
  int start;  // calls before this (device-side count) store no pair in the history
  long len;   // no*nv + no*no*nv*nv
  double shift;
  // Batched update of nslot amplitude sets: every pointer above except stats names slot 0 of a
  // layout repeated at a byte stride ss (slot k at + k ss, k = tab[z] for grid row z when tab is
  // given, entries at most tab_max); stats is [slot][8].
  int nslot = 1;
  long ss = 0;
  const int* tab = nullptr;
  int tab_max = 0;
};
hipError_t diis_update(const UpdateArgs& u, hipStream_t s);
int update_partial_blocks();

// The solve loop of ascc_solve with its DIIS state and work arrays carved from [ws, ws + ws_bytes)
// (ws == nullptr: allocated, as ascc_solve does), and the bytes that carving needs.
size_t solve_workspace_bytes(long o, long v, int diis_size);
int solve_impl(ascc_ints* I, const ascc_opts* opts, double* t1, double* t2, ascc_result* res, void* stream, char* ws,
               size_t ws_bytes);
// An unbacked, never dereferenced device address range for a dry run.
uintptr_t dry_run_address(size_t bytes);
// One iteration (residual, then the Jacobi/DIIS update) of n slots that repeat one layout at a
// byte stride: I, D and the amplitude / residual / energy pointers are those of the base slot,
// whose layout spans [region, region + stride); slot z of the batch is the base slot + htab[z]
// (dtab: the same table in device memory, read by the batched contractions and the update).
// stats receives one row of 8 statistics per slot, row htab[z] for slot z (see ascc_update).
int iterate_slots(ascc_ints* I, ::ascc_diis* D, int n, const int* dtab, const int* htab, const char* region,
                  long stride, double* t1, double* t2, double* r1, double* r2, double* e, double* stats,
                  hipStream_t s);

}  // namespace ascc
