// The C ABI of libascc (include/ascc.h): integral assembly, the closed-shell CCSD-form
// residual, the Jacobi/DIIS update and the solve loop, all on one HIP stream.
//
// Residual algorithm (FP64).  With T1-dressed factors B^_Q = X B_Q Y^T (X = 1 - t1 in the
// virtual-occupied block, Y = 1 + t1^T in the occupied-virtual block) and the dressed Fock
// matrix F^ = X h Y^T + sum_k (2 g^_pqkk - g^_pkkq), the closed-shell residual is
//   R_ij^ab = g^_aibj + sum_cd t_ij^cd g^_acbd + sum_kl t_kl^ab (g^_kilj + sum_cd t_ij^cd g_kcld)
//             + P_ij^ab [C + D + E]_aibj
// (the projections of the paper's Eq. (eqn:amp) for T = T1 + T2, Sec. II.A-B, in spin-adapted
// form, Supporting Information S1).  The particle-particle ladder is evaluated against the
// UNdressed (ac|bd), which is formed once per integral set, and the dressing is moved onto
// the amplitudes side:
//   sum_cd t_ij^cd g^_acbd = sum_cd t_ij^cd (ac|bd) - P_ij^ab sum_k t_k^a W'_ij[k,b]
//   W_ij[k,b] = sum_cd (kc|bd) t_ij^cd,  Z_ij[k,l] = sum_cd (kc|ld) t_ij^cd,
//   W'_ij[k,b] = W_ij[k,b] - 1/2 sum_l Z_ij[k,l] t_l^b
// so no v^4 array is ever re-dressed.  Ring terms use permuted views of t2 in the
// [o][v][o][v] layout:
//   Tx[iajb] = t_ij^ba, U[iajb] = u_ij^ab = 2 t_ij^ab - t_ij^ba,
//   Y1 = Tx K, Y2 = U L  (K[iajb] = (ib|ja), L = 2(ia|jb) - (ib|ja)),
//   Xc[iakc] = g^_kiac - Y1/2,  Zd[iakc] = 2 g^_aikc - g^_kiac + Y2/2,
//   P1 = Tx Xc^T, P2 = U Zd^T,
// and the N^5 terms go through N_Q[k,a] = sum_lc u_kl^ac B_Q,lc.
#include <algorithm>
#include <cmath>
#include <cstdio>
#include <cstdlib>
#include <cstring>
#include <map>
#include <mutex>
#include <string>
#include <vector>

#include "../../include/ascc.h"
#include "internal.h"

namespace ascc {

static thread_local std::string g_last_error;
void set_error(const std::string& msg) { g_last_error = msg; }

static std::mutex g_buf_mu;
static std::map<uintptr_t, size_t> g_bufs;
// set while a slot batch is issued: its launches span the slots, so an access may lie in an
// enclosing buffer (a server slab, a batch region) rather than in the base slot's own array
static thread_local bool g_enclosing_ok = false;

bool dry_run() {
  static const bool on = [] {
    const char* e = std::getenv("ASCC_DRY_RUN");
    return e && e[0] == '1';
  }();
  return on;
}

bool bounds_checking() {
  static const bool on = [] {
    const char* e = std::getenv("ASCC_CHECK_BOUNDS");
    return (e && e[0] == '1') || dry_run();
  }();
  return on;
}

void register_buffer(const void* p, size_t bytes) {
  if (!bounds_checking() || !p) return;
  std::lock_guard<std::mutex> lk(g_buf_mu);
  g_bufs[(uintptr_t)p] = bytes;
}

void unregister_buffer(const void* p) {
  if (!bounds_checking() || !p) return;
  std::lock_guard<std::mutex> lk(g_buf_mu);
  g_bufs.erase((uintptr_t)p);
}

bool range_ok(const void* base, long lo, long hi, size_t elem, const char* what) {
  if (!bounds_checking()) return true;
  std::lock_guard<std::mutex> lk(g_buf_mu);
  const uintptr_t b = (uintptr_t)base;
  auto it = g_bufs.upper_bound(b);
  if (it == g_bufs.begin()) {
    set_error(std::string(what) + ": pointer is not inside a registered buffer");
    return false;
  }
  // the innermost buffer that starts at or below base is tried first; an access that spans the
  // slots of a batch is accepted if an enclosing buffer (a server slab, a batch region) holds it
  long long first = 0, last = 0;
  size_t size0 = 0;
  for (auto jt = std::prev(it);; --jt) {
    const long long f = (long long)b + (long long)lo * (long long)elem - (long long)jt->first;
    const long long l = (long long)b + ((long long)hi + 1) * (long long)elem - (long long)jt->first;
    if (jt == std::prev(it)) {
      first = f;
      last = l;
      size0 = jt->second;
    }
    if (f >= 0 && l <= (long long)jt->second) return true;
    if (!g_enclosing_ok || jt == g_bufs.begin()) break;
  }
  char msg[256];
  std::snprintf(msg, sizeof msg, "%s: elements [%ld, %ld] fall outside their %zu-byte buffer (byte range %lld..%lld)",
                what, lo, hi, size0, first, last);
  set_error(msg);
  return false;
}

// Runtime calls that are skipped in a dry run (and bounds-checked when checking is on).
hipError_t d_copy(void* dst, const void* src, size_t bytes, hipMemcpyKind kind, hipStream_t s) {
  if (bytes == 0) return hipSuccess;
  if (bounds_checking()) {
    const bool dst_dev = (kind == hipMemcpyDeviceToDevice || kind == hipMemcpyHostToDevice);
    const bool src_dev = (kind == hipMemcpyDeviceToDevice || kind == hipMemcpyDeviceToHost);
    if ((dst_dev && !range_ok(dst, 0, (long)bytes - 1, 1, "copy destination")) ||
        (src_dev && !range_ok(src, 0, (long)bytes - 1, 1, "copy source")))
      return hipErrorInvalidValue;
  }
  if (dry_run()) return hipSuccess;
  return hipMemcpyAsync(dst, src, bytes, kind, s);
}
hipError_t d_sync(hipStream_t s) { return dry_run() ? hipSuccess : hipStreamSynchronize(s); }

// Registers caller buffers for the bounds checker for the duration of one ABI call.
struct ScopedBuffers {
  std::vector<const void*> ps;
  void add(const void* p, size_t bytes) {
    if (!bounds_checking() || !p) return;
    {
      std::lock_guard<std::mutex> lk(g_buf_mu);
      if (g_bufs.count((uintptr_t)p)) return;  // a library buffer, or already registered
    }
    register_buffer(p, bytes);
    ps.push_back(p);
  }
  ~ScopedBuffers() {
    for (const void* p : ps) unregister_buffer(p);
  }
};

constexpr size_t kAlign = 256;

// Where a handle's device arrays come from: carved from a caller workspace (base != nullptr,
// no runtime allocation at all) or allocated with hipMalloc.
struct Pool {
  char* base = nullptr;
  size_t size = 0, off = 0;
  std::vector<void*> owned;   // hipMalloc'd blocks
  std::vector<void*> carved;  // carved arrays (for the bounds checker)
  size_t total = 0;
};

// A scratch pool for build-time temporaries: the untouched rest of a carved workspace, or
// separate hipMalloc blocks.  Released with free_all once the temporaries are no longer used.
Pool sub_pool(const Pool& P) {
  Pool t;
  if (P.base) {
    const size_t o = (P.off + kAlign - 1) / kAlign * kAlign;
    t.base = P.base + std::min(o, P.size);
    t.size = P.size - std::min(o, P.size);
  }
  return t;
}

}  // namespace ascc

using namespace ascc;

struct ascc_ints {
  int no, nv, naux, n, precision, vvvv_mode, device;
  long ov, oo, vv, ovov, oovv;
  Pool pool;
  // constant integrals
  double* B;      // [Q][n][n]
  double* h;      // [n][n] core Hamiltonian
  double* eps;    // [n] Fock diagonal
  double* fov;    // [o][v] reference Fock, occupied-virtual block
  double* e0;     // [1] reference energy <phi_0|H|phi_0> = sum_i (h_ii + f_ii)
  double* Bov;    // [Q][o][v]
  double* BovT;   // [o][v][Q]: the same, K = Q contiguous
  double* KL;     // [2][ov][ov]: (ib|ja), 2(ia|jb) - (ib|ja)
  double* Lijab;  // [o][o][v][v]: 2(ia|jb) - (ib|ja)
  double* Gwz;    // [ov + o^2][v][v]: (kc|bd) at [k*v+b][c][d], (kc|ld) at [ov + k*o+l][c][d]
  double* V;      // FULL: [v^2][v^2], (ac|bd) at [R(a,b)][R(c,d)] (pair order: a <= b first, see pack_full)
                  // PACKED: [2][T(v)][T(v)], (ac|bd) +- (ad|bc) at [p(a,b)][p(c,d)], a <= b, c <= d
  double* pairtab;  // FULL: int32 [T(v)]: row R(b,a) of V for pair p(a,b), a <= b
  double *Tp, *Rp;  // ladder operands [2][T(o)][T(v)]: t+- (pack_tpm) and R+- (unpack_rpm)
  // residual work arrays
  double* Bc;                    // [Q][n][o] T1 correction of the first o columns of B
  double* Bh;                    // [Q][n][n]
  double* hc;                    // [n][o]
  double* Fh;                    // [n][n]
  double *J;                     // [Q]
  double *BvoTt, *Boo, *Bvv;     // [o][v][Q] (B^_ai at [i][a][Q]), [Q][o][o], [Q][v][v]
  double *G1, *G2, *G3, *G4;     // ovov, [k][i][a][c], ovov, [k][i][l][j]
  double *TU, *Y, *XZ, *P;       // each [2][ov][ov]
  double *Nq;                    // [Q][o][v]
  double *WZ;                    // [o^2][ov + o^2]
  double *chi;                   // [o^2][o^2]
  double *RL, *EM;               // [o^2][v^2]
  double *Abc, *Bkj, *Fvvp, *Foop, *Fovh;  // small
  double *partial;               // reduction scratch
  double *splitk;                // split-K partial tiles of small-output contractions
  // FP32 shadows of the large-contraction operands (only for a low-precision integral set)
  float *Vf, *GwzTf, *KLf;       // constant: vvvv, [ov+o^2][v^2] (kc|bd)|(kc|ld), K|L
  float *Tpf, *t2f, *TUf, *XZf;  // per residual: ladder rows, t2 rows, Tx|U, Xc|Zd
  // per residual, K = naux or o^2 contiguous: B^_ai as [ia][Q], B^_ki [ki][Q], B^_ac [ac][Q],
  // B^_kc [kc][Q], B^_kc as [Q][kc], t2 as [ab][ij], chi [ij][kl]
  float *BvoTtf, *BooTf, *BvvTf, *BovTf, *Bovf, *t2Tf, *chif;
  int cur_prec = 0;              // arithmetic of the large contractions in the next residual
  // multi-state batches (ascc_batch_reserve): stacked ladder operands and per-state RL
  int max_states = 0;
  double *Tp_all = nullptr, *Rp_all = nullptr, *RL_all = nullptr;
  float* Tpf_all = nullptr;
  int group = 1;             // states per batched pass of the other terms (ascc_batch_reserve_ws)
  char* group_base = nullptr;  // `group` work blocks of group_block bytes
  size_t group_block = 0;
  Pool batch;
  // partial linearisation (ascc_set_plascc): primaries and the slab buffers of the removal
  int pl_hole = -1, pl_pa = -1;
  double *plA, *plC, *plKr, *plKpp, *plYp, *plYpp, *plS, *plZ, *plZt, *plW;  // ov-cross slabs (rings)
  double *plN, *plBp, *plNw;                                                 // N^M and its slabs
  double *plTa, *plTc, *plGc, *plZo, *plZh, *plRc, *plEc;                    // oo / vv-cross slabs
  Pool pl;
  // optional per-phase timing with HIP events (ascc_timing_enable)
  bool timing = false;
  std::vector<std::pair<int, std::pair<hipEvent_t, hipEvent_t>>> marks;  // (phase, (start, end))
  std::vector<hipEvent_t> event_pool;
};

struct ascc_diis {
  int no, nv, m, start, calls;
  long len;
  double *hist_t, *hist_e, *partial;
  DiisState* st;
  Pool pool;
};

namespace {

const char* const kPhaseNames[] = {"dress",  "amp_views", "df_ints", "wz",      "pp_pack",  "pp_ladder",
                                   "pp_unpack", "hh_ladder", "ring_y", "ring_xz", "ring_p", "n5_terms",
                                   "assemble", "energy",    "update",  "plascc"};
constexpr int kNumPhases = sizeof(kPhaseNames) / sizeof(kPhaseNames[0]);
enum Phase { PH_DRESS, PH_AMP, PH_DF, PH_WZ, PH_PACK, PH_LADDER, PH_UNPACK, PH_HH, PH_RING_Y, PH_RING_XZ, PH_RING_P,
             PH_N5, PH_ASSEMBLE, PH_ENERGY, PH_UPDATE, PH_PLASCC };

hipEvent_t take_event(ascc_ints* I) {
  if (!I->event_pool.empty()) {
    hipEvent_t e = I->event_pool.back();
    I->event_pool.pop_back();
    return e;
  }
  hipEvent_t e = nullptr;
  if (hipEventCreate(&e) != hipSuccess) return nullptr;
  return e;
}

// Records the start of `phase` on `s` (no-op unless timing is on); close it with phase_end.
void phase_begin(ascc_ints* I, int phase, hipStream_t s) {
  if (!I->timing || dry_run()) return;
  hipEvent_t a = take_event(I), b = take_event(I);
  if (!a || !b) return;
  (void)hipEventRecord(a, s);
  I->marks.push_back({phase, {a, b}});
}
void phase_end(ascc_ints* I, hipStream_t s) {
  if (!I->timing || dry_run() || I->marks.empty()) return;
  (void)hipEventRecord(I->marks.back().second.second, s);
}

#define HIPCHK(expr)                                                                         \
  do {                                                                                       \
    hipError_t e_ = (expr);                                                                  \
    if (e_ != hipSuccess) {                                                                  \
      set_error(std::string(#expr) + ": " + hipGetErrorString(e_));                          \
      return ASCC_E_HIP;                                                                     \
    }                                                                                        \
  } while (0)

int fail(int code, const std::string& msg) {
  set_error(msg);
  return code;
}

// Unbacked, never dereferenced addresses handed out in a dry run.
uintptr_t fake_alloc(size_t bytes) {
  static uintptr_t next = (uintptr_t)1 << 44;
  static std::mutex mu;
  std::lock_guard<std::mutex> lk(mu);
  const uintptr_t p = next;
  next += (bytes + 4095) / 4096 * 4096 + 4096;
  return p;
}

// Pair-row tables of a FULL integral set (see gemm_f64_ladder).
inline int* pair_minus(const ascc_ints* I) { return reinterpret_cast<int*>(I->pairtab); }

constexpr long kSplitKElems = 1L << 23;  // 64 MiB of split-K partials
inline long pad_even(long x) { return x + (x & 1); }  // compact slab widths, even for the direct-to-LDS path

// Every device array of an integral set with its element count, in allocation order; the
// same list gives ascc_workspace_bytes its exact answer.
std::vector<std::pair<double* ascc_ints::*, long>> ints_plan(long o, long v, long Q, int mode) {
  const long n = o + v, nn = n * n, ov = o * v, oo = o * o, vv = v * v, ovov = ov * ov;
  const long To = o * (o + 1) / 2, Tv = v * (v + 1) / 2;
  const bool full = (mode == ASCC_VVVV_FULL);
  return {
      {&ascc_ints::B, Q * nn},        {&ascc_ints::h, nn},           {&ascc_ints::eps, n},
      {&ascc_ints::fov, ov},          {&ascc_ints::e0, 1},
      {&ascc_ints::Bov, Q * ov},      {&ascc_ints::KL, 2 * ovov},
      {&ascc_ints::Lijab, oo * vv},   {&ascc_ints::Gwz, vv * (ov + oo)},
      {&ascc_ints::BovT, ov * Q},
      {&ascc_ints::V, full ? vv * vv : 2 * Tv * Tv},
      {&ascc_ints::pairtab, full ? Tv : 0},
      {&ascc_ints::Tp, 2 * To * Tv},  {&ascc_ints::Rp, 2 * To * Tv},
      {&ascc_ints::Bc, Q * n * o},    {&ascc_ints::Bh, Q * nn},      {&ascc_ints::hc, n * o},
      {&ascc_ints::Fh, nn},           {&ascc_ints::J, Q},            {&ascc_ints::BvoTt, Q * ov},
      {&ascc_ints::Boo, Q * oo},      {&ascc_ints::Bvv, Q * vv},     {&ascc_ints::G1, ovov},
      {&ascc_ints::G2, oo * vv},      {&ascc_ints::G3, ovov},        {&ascc_ints::G4, oo * oo},
      {&ascc_ints::TU, 2 * ovov},     {&ascc_ints::Y, 2 * ovov},     {&ascc_ints::XZ, 2 * ovov},
      {&ascc_ints::P, 2 * ovov},      {&ascc_ints::Nq, Q * ov},      {&ascc_ints::WZ, oo * (ov + oo)},
      {&ascc_ints::chi, oo * oo},     {&ascc_ints::RL, oo * vv},     {&ascc_ints::EM, oo * vv},
      {&ascc_ints::Abc, vv},          {&ascc_ints::Bkj, oo},         {&ascc_ints::Fvvp, vv},
      {&ascc_ints::Foop, oo},         {&ascc_ints::Fovh, ov},        {&ascc_ints::partial, 8192},
      {&ascc_ints::splitk, kSplitKElems},
  };
}

// FP32 shadows allocated for a low-precision integral set.
std::vector<std::pair<float* ascc_ints::*, long>> lowp_plan(long o, long v, long Q, int mode) {
  const long ov = o * v, oo = o * o, vv = v * v;
  const long To = o * (o + 1) / 2, Tv = v * (v + 1) / 2;
  (void)mode;  // both storage modes keep the packed halves in low precision
  // rows x padded leading dimension (lowp_ld); one float = one bf16 hi + one bf16 lo for BF16X3
  const long lvv = lowp_ld(vv), lTv = lowp_ld(Tv), lov = lowp_ld(ov), lQ = lowp_ld(Q), loo = lowp_ld(oo);
  return {
      {&ascc_ints::Vf, 2 * Tv * lTv},  {&ascc_ints::GwzTf, (ov + oo) * lvv},
      {&ascc_ints::KLf, 2 * ov * lov}, {&ascc_ints::Tpf, 2 * To * lTv},
      {&ascc_ints::t2f, oo * lvv},     {&ascc_ints::TUf, 2 * ov * lov},
      {&ascc_ints::XZf, 2 * ov * lov}, {&ascc_ints::BvoTtf, ov * lQ},
      {&ascc_ints::BooTf, oo * lQ},    {&ascc_ints::BvvTf, vv * lQ},
      {&ascc_ints::BovTf, ov * lQ},    {&ascc_ints::Bovf, Q * lov},
      {&ascc_ints::t2Tf, vv * loo},    {&ascc_ints::chif, oo * loo},
  };
}

// Bytes of the (kc|bd) temporary and of one chunk of the packed-vvvv build (freed after the build).
long build_temp_elems(long o, long v, int mode, long* chunk_a) {
  const long vvv = v * v * v;
  long ac = std::max<long>(1, std::min<long>(v, (256L << 20) / std::max<long>(vvv, 1)));  // about 2 GB
  // a packed set needs the (ac|bd) slabs with b >= a only and computes those with b >= the chunk's
  // first a: chunks of at most v/16 values of a keep that within about 3 % of the a <= b triangle
  if (mode == ASCC_VVVV_PACKED) ac = std::min<long>(ac, std::max<long>(1, (v + 15) / 16));
  if (chunk_a) *chunk_a = ac;
  const long wtmp = o * v * v * v;
  return std::max(wtmp, ac * vvv);
}


size_t align_up(size_t x) { return (x + kAlign - 1) / kAlign * kAlign; }

// Bytes a DIIS state carves from a workspace.
size_t diis_footprint(long o, long v, int m) {
  const long len = o * v + o * o * v * v;
  size_t off = 0;
  off = align_up(off) + sizeof(double) * m * len;
  off = align_up(off) + sizeof(double) * m * len;
  off = align_up(off) + sizeof(double) * update_partial_blocks() * (3 + kMaxDiis);
  off = align_up(off) + sizeof(DiisState);
  return align_up(off);
}

template <class T>
int dalloc(Pool& P, T** out, size_t count) {
  const size_t bytes = std::max<size_t>(count, 1) * sizeof(T);
  if (P.base) {
    const size_t o = (P.off + kAlign - 1) / kAlign * kAlign;
    if (o + bytes > P.size) {
      set_error("workspace too small: needs at least " + std::to_string(o + bytes) + " bytes");
      return ASCC_E_NOMEM;
    }
    *out = reinterpret_cast<T*>(P.base + o);
    P.off = o + bytes;
    P.total += bytes;
    P.carved.push_back(*out);
    register_buffer(*out, bytes);
    return ASCC_OK;
  }
  void* q = nullptr;
  hipError_t e = dry_run() ? (q = (void*)fake_alloc(bytes), hipSuccess) : hipMalloc(&q, bytes);
  if (e != hipSuccess) {
    (void)hipGetLastError();
    set_error("hipMalloc of " + std::to_string(bytes) + " bytes failed: " + hipGetErrorString(e));
    return ASCC_E_NOMEM;
  }
  P.owned.push_back(q);
  P.total += bytes;
  *out = static_cast<T*>(q);
  register_buffer(q, bytes);
  return ASCC_OK;
}

void free_all(Pool& P) {
  if (!P.owned.empty() && !dry_run()) (void)hipDeviceSynchronize();
  for (void* p : P.owned) {
    unregister_buffer(p);
    if (!dry_run()) (void)hipFree(p);
  }
  for (void* p : P.carved) unregister_buffer(p);
  P.owned.clear();
  P.carved.clear();
  P.off = 0;
  P.total = 0;
}

inline Perm4In pin(const double* p, long s0, long s1, long s2, long s3, double coef) {
  Perm4In x;
  x.p = p;
  x.s[0] = s0;
  x.s[1] = s1;
  x.s[2] = s2;
  x.s[3] = s3;
  x.coef = coef;
  return x;
}

// ---- slot batches ----------------------------------------------------------------------
// A batched residual evaluates n slots -- amplitude sets whose arrays repeat one layout at fixed
// byte strides -- in one pass: each contraction is one launch with an outer batch level over the
// slots, and each element-wise step is issued once per slot.  The arrays the residual touches are
// registered as address ranges of the base slot with their slot stride (0 for arrays the slots
// share); slot z of a launch is table entry z (relative to the base slot).
struct SlotRange {
  uintptr_t lo, hi;
  long stride;  // bytes
};
struct SlotBatch {
  int n = 1;
  const int* dtab = nullptr;  // device table of the n slots (nullptr: 0 .. n-1)
  const int* htab = nullptr;  // its host copy
  int tab_max = 0;
  std::vector<SlotRange> ranges;
  bool bad = false;  // a pointer outside every registered range was met
};
thread_local SlotBatch* g_sb = nullptr;
thread_local int g_slot = 0;  // the slot an element-wise step is being issued for

inline int nslots() { return g_sb ? g_sb->n : 1; }
long slot_stride(const void* p) {
  const uintptr_t x = reinterpret_cast<uintptr_t>(p);
  for (const SlotRange& r : g_sb->ranges)
    if (x >= r.lo && x < r.hi) return r.stride;
  g_sb->bad = true;
  return 0;
}
// p (an array of the base slot) in the slot of the element-wise step being issued
template <class T>
T* S(T* p) {
  if (!g_sb || !p) return p;
  if (g_slot < 0 || g_slot >= g_sb->n) {
    g_sb->bad = true;
    return p;
  }
  const long k = g_sb->htab ? g_sb->htab[g_slot] : g_slot;
  return reinterpret_cast<T*>(reinterpret_cast<uintptr_t>(p) + k * slot_stride(p));
}
#define EACH_SLOT for (g_slot = 0; g_slot < nslots(); ++g_slot)

// FP64 contraction with the integral set's split-K scratch (shared by the slots of a batch).
inline hipError_t mm(const ascc_ints* I, Gemm g, hipStream_t s) {
  g.ws = I->splitk;
  g.ws_elems = kSplitKElems;
  if (nslots() > 1) {
    if (g.nb1 != 1) return hipErrorInvalidValue;
    const long a = slot_stride(g.A), b = slot_stride(g.B), c = slot_stride(g.C);
    if (g_sb->bad || (a | b | c) % 8) return hipErrorInvalidValue;
    g.nb1 = g_sb->n;
    g.sa1 = a / 8;
    g.sb1 = b / 8;
    g.sc1 = c / 8;
    g.tab1 = g_sb->dtab;
    g.tab1_max = g_sb->tab_max;
    g.per_block = true;  // each slot sums in the order it would alone
  }
  return gemm_f64(g, s);
}

// Low-precision contraction, one launch over the slots of a batch.
inline hipError_t glp(GemmLP g, hipStream_t s) {
  if (nslots() > 1) {
    const long el = g.prec == kPrecBF16x3 ? 2 : 4;  // operand strides count bf16 or FP32 elements
    const long a = slot_stride(g.A), b = slot_stride(g.B), c = slot_stride(g.C);
    if (g_sb->bad || a % el || b % el || c % 8) return hipErrorInvalidValue;
    g.nb1 = g_sb->n;
    g.sa1 = a / el;
    g.sb1 = b / el;
    g.sc1 = c / 8;
    g.tab1 = g_sb->dtab;
    g.tab1_max = g_sb->tab_max;
    g.per_block = true;
  }
  return gemm_lowp(g, s);
}

// T1 dressing of `nb` stacked n x n matrices, dst = X src Y^T with X = 1 - F, Y^T = 1 + F and
// F[o + a][i] = t1[i][a]: one GEMM for the correction of the first o columns, tc = src[:, o:n] t1^T,
// then one streaming pass (dress_apply) that forms dst from src and tc.
int dress(const ascc_ints* I, const double* src, double* tc, double* dst, const double* t1, int o, int v, int nb,
          hipStream_t s) {
  const long n = o + v, nn = n * n;
  Gemm g;
  g.M = (int)n;
  g.N = o;
  g.K = v;
  g.A = src + o;
  g.sam = n;
  g.sak = 1;
  g.sa2 = nn;
  g.B = t1;
  g.sbk = 1;
  g.sbn = v;
  g.C = tc;
  g.scm = o;
  g.scn = 1;
  g.sc2 = n * o;
  g.nb2 = nb;
  HIPCHK(mm(I, g, s));
  EACH_SLOT HIPCHK(dress_apply(S(dst), S(src), S(tc), S(t1), o, v, nb, s));
  return ASCC_OK;
}

// F += sign * (2 sum_Q J_Q B_Q - sum_Q B_Q[:,0:o] B_Q[0:o,:]),  J_Q = sum_k B_Q[k][k]
int add_two_electron_fock(const ascc_ints* I, double* F, const double* Bq, double* J, int o, int v, int Q, double sign,
                          hipStream_t s) {
  const long n = o + v, nn = n * n;
  EACH_SLOT HIPCHK(diag_trace(S(J), S(Bq), Q, n, o, s));
  {
    Gemm g;
    g.M = 1;
    g.N = nn;
    g.K = Q;
    g.A = J;
    g.sam = 0;
    g.sak = 1;
    g.B = Bq;
    g.sbk = nn;
    g.sbn = 1;
    g.C = F;
    g.scm = 0;
    g.scn = 1;
    g.alpha = 2.0 * sign;
    g.beta = 1.0;
    HIPCHK(mm(I, g, s));
  }
  {
    Gemm g;
    g.M = n;
    g.N = n;
    g.K = o;
    g.A = Bq;
    g.sam = n;
    g.sak = 1;
    g.sar = nn;
    g.B = Bq;
    g.sbk = n;
    g.sbn = 1;
    g.sbr = nn;
    g.C = F;
    g.scm = n;
    g.scn = 1;
    g.alpha = -sign;
    g.beta = 1.0;
    g.nred = Q;
    HIPCHK(mm(I, g, s));
  }
  return ASCC_OK;
}


// C_z[m][n] = sum_k A_z[m][k] B_z[n][k] in the handle's current low precision (FP64 result).
GemmLP lp_nt(const ascc_ints* I, long M, long N, long K, int nb, const float* A, long lda, long sa2, const float* B,
             long ldb, long sb2, double* C, long ldc, long sc2) {
  GemmLP g;
  g.M = (int)M;
  g.N = (int)N;
  g.K = (int)K;
  g.nb = nb;
  g.A = A;
  g.lda = lda;
  g.sa2 = sa2;
  g.B = B;
  g.ldb = ldb;
  g.sb2 = sb2;
  g.C = C;
  g.scm = ldc;
  g.scn = 1;
  g.sc2 = sc2;
  g.prec = (I->cur_prec == ASCC_PREC_BF16X3) ? kPrecBF16x3 : kPrecFP32;
  g.ws = I->splitk;
  g.ws_elems = kSplitKElems;
  if (g.prec == kPrecBF16x3) {  // one float of a shadow = one bf16 pair: strides in bf16 elements
    g.lda *= 2;
    g.sa2 *= 2;
    g.ldb *= 2;
    g.sb2 *= 2;
  }
  return g;
}

int lowp_kind(const ascc_ints* I) { return (I->cur_prec == ASCC_PREC_BF16X3) ? kPrecBF16x3 : kPrecFP32; }

// Low-precision shadow of a transpose: out row r = column r of in ([cols][ldi]), leading dimension
// lowp_ld(cols).
hipError_t shadow_t(const ascc_ints* I, float* out, const double* in, long ldi, long rows, long cols, hipStream_t s) {
  EACH_SLOT {
    const hipError_t e = to_lowp_t(lowp_kind(I), S(out), lowp_ld(cols), S(in), ldi, rows, cols, s);
    if (e != hipSuccess) return e;
  }
  return hipSuccess;
}

// Low-precision shadow of rows x cols FP64 (contiguous rows) with leading dimension lowp_ld(cols).
hipError_t shadow(const ascc_ints* I, float* out, const double* in, long rows, long cols, hipStream_t s) {
  const int prec = (I->cur_prec == ASCC_PREC_BF16X3) ? kPrecBF16x3 : kPrecFP32;
  EACH_SLOT {
    const hipError_t e = to_lowp_2d(prec, S(out), lowp_ld(cols), S(in), cols, rows, cols, s);
    if (e != hipSuccess) return e;
  }
  return hipSuccess;
}

// Particle-particle ladder RL_s[i][j][a][b] = sum_cd (t_s)_ij^cd (ac|bd) for S states in one
// launch, computed for pairs i <= j only (RL_ji^ba = RL_ij^ab) and through the (ab)-symmetric and
// antisymmetric halves: R+- = t+- V+- with t+-_ij^cd = (t_ij^cd +- t_ij^dc)/2 over c <= d and
// V+-[(ab)][(cd)] = (ac|bd) +- (ad|bc) over a <= b (diagonal cd: (ac|bc) and 0), both halves in
// one launch.  PACKED stores V+-; FULL stores the full (ac|bd) matrix in pair order, and its
// halves are V[n][k] +- V[pm[n]][k], formed while the FP64 contraction stages them (and rounded
// into the low-precision shadow); there the diagonal V+ is 2(ac|bc), so t+ carries t_ij^cc / 2.
// The S states' rows are stacked, so the vvvv operand is streamed once for all of them.  Tp/Rp
// hold [2][S*T(o)][T(v)].
int pp_ladder_states(ascc_ints* I, int S, const double* const* t2s, double* const* RLs, double* Tp, double* Rp,
                     float* Tpf, hipStream_t s) {
  const int o = I->no, v = I->nv;
  const long To = (long)o * (o + 1) / 2, Tv = (long)v * (v + 1) / 2;
  const long M = S * To;
  const bool lowp = I->cur_prec != ASCC_PREC_FP64;
  const bool full = I->vvvv_mode == ASCC_VVVV_FULL;
  const long ld = lowp_ld(Tv);
  // Phases: pp_pack (pair packing and low-precision operands), pp_ladder (the one contraction
  // launch, nothing else), pp_unpack (scatter back to [i][j][a][b]).
  phase_begin(I, PH_PACK, s);
  const double dscale = full ? 0.5 : 1.0;  // full: the combined diagonal V+ is doubled
  for (int k = 0; k < S; ++k) HIPCHK(pack_tpm(Tp + k * To * Tv, Tp + (M + k * To) * Tv, t2s[k], o, v, dscale, s));
  if (lowp) HIPCHK(shadow(I, Tpf, Tp, 2 * M, Tv, s));
  phase_end(I, s);
  phase_begin(I, PH_LADDER, s);
  if (lowp) {  // no split-K: a state's rows are summed in the same order whatever S is
    GemmLP g = lp_nt(I, M, Tv, Tv, 2, Tpf, ld, M * ld, I->Vf, ld, Tv * ld, Rp, Tv, M * Tv);
    g.ws = nullptr;
    g.m_dec = (int)To;  // the kernel choice of one state's rows
    HIPCHK(gemm_lowp(g, s));
  }
  else if (full)
    HIPCHK(gemm_f64_ladder((int)M, (int)Tv, Tp, I->V, I->vv, I->vv, pair_minus(I), Rp, s));
  else
    HIPCHK(gemm_f64_ladder((int)M, (int)Tv, Tp, I->V, Tv, 0, nullptr, Rp, s));
  phase_end(I, s);
  phase_begin(I, PH_UNPACK, s);
  for (int k = 0; k < S; ++k) HIPCHK(unpack_rpm(RLs[k], Rp + k * To * Tv, Rp + (M + k * To) * Tv, o, v, s));
  phase_end(I, s);
  return ASCC_OK;
}

// The ladder of every slot of a batch, each against its own integral set: the pair packing per
// slot, one contraction launch over the slots, the unpacking per slot.
int pp_ladder_slots(ascc_ints* I, const double* t2, hipStream_t s) {
  const int o = I->no, v = I->nv;
  const long To = (long)o * (o + 1) / 2, Tv = (long)v * (v + 1) / 2, M = To;
  const bool lowp = I->cur_prec != ASCC_PREC_FP64;
  const bool full = I->vvvv_mode == ASCC_VVVV_FULL;
  const long ld = lowp_ld(Tv);
  phase_begin(I, PH_PACK, s);
  EACH_SLOT HIPCHK(pack_tpm(S(I->Tp), S(I->Tp) + M * Tv, S(t2), o, v, full ? 0.5 : 1.0, s));
  if (lowp) HIPCHK(shadow(I, I->Tpf, I->Tp, 2 * M, Tv, s));
  phase_end(I, s);
  phase_begin(I, PH_LADDER, s);
  if (lowp) {
    GemmLP g = lp_nt(I, M, Tv, Tv, 2, I->Tpf, ld, M * ld, I->Vf, ld, Tv * ld, I->Rp, Tv, M * Tv);
    g.ws = nullptr;
    HIPCHK(glp(g, s));
  } else {
    LadderBatch lb;
    lb.n = g_sb->n;
    lb.tab = g_sb->dtab;
    lb.tab_max = g_sb->tab_max;
    lb.sa = slot_stride(I->Tp) / 8;
    lb.sv = slot_stride(I->V) / 8;
    lb.sc = slot_stride(I->Rp) / 8;
    if (g_sb->bad) return fail(ASCC_E_STATE, "ladder operands outside the batch's slot ranges");
    if (full)
      HIPCHK(gemm_f64_ladder((int)M, (int)Tv, I->Tp, I->V, I->vv, I->vv, pair_minus(I), I->Rp, s, lb));
    else
      HIPCHK(gemm_f64_ladder((int)M, (int)Tv, I->Tp, I->V, Tv, 0, nullptr, I->Rp, s, lb));
  }
  phase_end(I, s);
  phase_begin(I, PH_UNPACK, s);
  EACH_SLOT HIPCHK(unpack_rpm(S(I->RL), S(I->Rp), S(I->Rp) + M * Tv, o, v, s));
  phase_end(I, s);
  return ASCC_OK;
}

int pp_ladder(ascc_ints* I, const double* t2, hipStream_t s) {
  if (nslots() > 1) return pp_ladder_slots(I, t2, s);
  double* RL = I->RL;
  return pp_ladder_states(I, 1, &t2, &RL, I->Tp, I->Rp, I->Tpf, s);
}

size_t ints_footprint(long o, long v, long Q, int precision, int mode) {
  size_t off = 0;
  for (const auto& item : ints_plan(o, v, Q, mode))
    off = align_up(off) + std::max<size_t>((size_t)item.second, 1) * sizeof(double);
  if (precision != ASCC_PREC_FP64)
    for (const auto& item : lowp_plan(o, v, Q, mode))
      off = align_up(off) + std::max<size_t>((size_t)item.second, 1) * sizeof(float);
  const long temp = build_temp_elems(o, v, mode, nullptr);
  return align_up(off) + sizeof(double) * (size_t)std::max<long>(temp, 1);
}

// Partial linearisation (Sec. II.C): remove from the doubles residual every term with two powers
// of the mixed doubles t^M (amplitudes whose index set holds the hole h or the particle pa and is
// not all primary; Sec. II.B, Eq. (eqn: pnm split)).  With T1 fixed the doubles residual is of
// degree two in T2 and its quadratic part does not involve T1 (the (kc|ld) integrals are not
// dressed), so the removal is that quadratic part evaluated at t^M, taken out of the four
// intermediates that carry it before the assembly:
//   hole-hole ladder  RL -= Z^M t^M,  Z^M_ij[k,l] = sum_cd t^M_ij^cd (kc|ld)
//   rings             P1 += 1/2 Tx^M K Tx^M^T,  P2 -= 1/2 U^M L U^M^T   (K, L symmetric)
//   E terms           EM += t^M A^M(b,c) + B^M(k,j) t^M through N^M_Q[k,a] = sum_lc B_Q,lc u^M_kl^ac.
// The mixed amplitudes live on crosses (see Cross): as ov x ov matrices Tx^M and U^M vanish off
// the rows and columns of the (i, a) cross X (i = h or a = pa, m = o + v - 1); as oo x vv
// matrices, t^M rows ij of the occupied cross are full and the other rows hold only the virtual
// cross ab.  Every product is split along those crosses into slabs: N^5 work.  The ring term is a
// symmetric matrix; its (X, X) and (X, not X) blocks come from the X rows of Y = T K that the ring
// stage has just formed, the (not X, not X) block is C_p K_pp C_p^T with C_p the X columns of the
// rows outside X.  Runs after the rings and E terms, in G2, chi, Abc and Bkj, which those are
// done with, and in the compact buffers of ascc_set_plascc.
int plascc_remove(ascc_ints* I, const double* t2, double* RL, hipStream_t s) {
  const int o = I->no, v = I->nv, Q = I->naux, h = I->pl_hole, pa = I->pl_pa;
  const long ov = I->ov, oo = I->oo, vv = I->vv, ovov = I->ovov;
  const Cross X{o, v, h, pa}, Xo{o, o, h, h}, Xv{v, v, pa, pa};
  const long m = X.m(), mp = pad_even(m), mo = Xo.m(), mop = pad_even(mo), mvp = pad_even(Xv.m());
  double* tM = I->G2;
  HIPCHK(mixed_doubles(tM, t2, o, v, h, pa, s));
  // --- hole-hole ladder.  tA: the occupied-cross rows of t^M; tC: the virtual-cross columns of the
  // other rows
  const double* G = I->Gwz + ov * vv;  // (kc|ld) at [k*o + l][c*v + d]
  double* ZM = I->chi;
  HIPCHK(cross_gather_rows(I->plTa, vv, tM, vv, oo, vv, Xo, false, s));
  HIPCHK(cross_gather_cols(I->plTc, mvp, tM, vv, oo, Xv, &Xo, s));
  HIPCHK(cross_gather_cols(I->plGc, mvp, G, vv, oo, Xv, nullptr, s));
  HIPCHK(mm(I, gemm_rm(oo, oo, mvp, 1.0, I->plTc, mvp, false, I->plGc, mvp, true, 0.0, ZM, oo), s));
  HIPCHK(mm(I, gemm_rm(mo, oo, vv, 1.0, I->plTa, vv, false, G, vv, true, 0.0, I->plZo, oo), s));
  HIPCHK(cross_scatter_add_rows(ZM, oo, oo, I->plZo, oo, oo, 1.0, Xo, s));
  HIPCHK(cross_gather_cols(I->plZh, mop, ZM, oo, oo, Xo, nullptr, s));
  HIPCHK(mm(I, gemm_rm(oo, vv, mo, -1.0, I->plZh, mop, false, I->plTa, vv, false, 1.0, RL, vv), s));
  HIPCHK(mm(I, gemm_rm(oo, mvp, oo, 1.0, ZM, oo, false, I->plTc, mvp, false, 0.0, I->plRc, mvp), s));
  HIPCHK(cross_scatter_add_cols(RL, vv, oo, I->plRc, mvp, -1.0, Xv, s));
  // --- rings, z = 0: Tx with K into P1 (+1/2); z = 1: U with L into P2 (-1/2).  U's slabs stay in
  // plA / plC for the E terms.
  const double kappa[2] = {0.5, -0.5};
  for (int z = 0; z < 2; ++z) {
    const double* T = I->TU + z * ovov;
    const double* K = I->KL + z * ovov;
    const double* Y = I->Y + z * ovov;  // T K from the ring stage
    double* P = I->P + z * ovov;
    HIPCHK(cross_gather_rows(I->plA, ov, T, ov, ov, ov, X, true, s));  // X rows of T^M
    HIPCHK(cross_gather_cols(I->plC, mp, T, ov, ov, X, &X, s));         // C_p
    HIPCHK(cross_gather_rows(I->plKr, ov, K, ov, ov, ov, X, false, s));
    HIPCHK(cross_gather_cols(I->plKpp, mp, I->plKr, ov, m, X, nullptr, s));  // K_pp
    HIPCHK(cross_rows_without_corner(I->plYp, ov, Y, T, K, X, s));          // X rows of T^M K
    HIPCHK(cross_gather_cols(I->plYpp, mp, I->plYp, ov, m, X, nullptr, s));
    // (X, X) block
    HIPCHK(mm(I, gemm_rm(m, m, ov, 1.0, I->plYp, ov, false, I->plA, ov, true, 0.0, I->plS, mp), s));
    HIPCHK(cross_scatter_add_block(P, ov, I->plS, mp, kappa[z], X, s));
    // (X, not X) and, by symmetry, (not X, X)
    HIPCHK(mm(I, gemm_rm(m, ov, mp, 1.0, I->plYpp, mp, false, I->plC, mp, true, 0.0, I->plZ, ov), s));
    HIPCHK(cross_scatter_add_rows(P, ov, ov, I->plZ, ov, ov, kappa[z], X, s));
    HIPCHK(mm(I, gemm_rm(ov, m, mp, 1.0, I->plC, mp, false, I->plYpp, mp, true, 0.0, I->plZt, mp), s));
    HIPCHK(cross_scatter_add_cols(P, ov, ov, I->plZt, mp, kappa[z], X, s));
    // (not X, not X) = C_p K_pp C_p^T
    HIPCHK(mm(I, gemm_rm(ov, m, m, 1.0, I->plC, mp, false, I->plKpp, mp, false, 0.0, I->plW, mp), s));
    HIPCHK(mm(I, gemm_rm(ov, ov, mp, kappa[z], I->plW, mp, false, I->plC, mp, true, 1.0, P, ov), s));
  }
  // --- E terms.  N^M[Q][r] = sum_c B_Q,c U^M[r][c]: columns outside X from C_p, X columns from the
  // X rows of U^M
  HIPCHK(cross_gather_cols(I->plBp, mp, I->Bov, ov, Q, X, nullptr, s));
  HIPCHK(mm(I, gemm_rm(Q, ov, mp, 1.0, I->plBp, mp, false, I->plC, mp, true, 0.0, I->plN, ov), s));
  HIPCHK(mm(I, gemm_rm(Q, m, ov, 1.0, I->Bov, ov, false, I->plA, ov, true, 0.0, I->plNw, mp), s));
  HIPCHK(cross_scatter_add_cols(I->plN, ov, Q, I->plNw, mp, 1.0, X, s));
  // A^M[b][c] = sum_Qk N^M_Q[k,b] B_Q,kc;  EM[ij][a][b] += sum_c t^M_ij^ac A^M[b][c]
  HIPCHK(mm(I, gemm_rm(v, v, (long)Q * o, 1.0, I->plN, v, true, I->Bov, v, false, 0.0, I->Abc, v), s));
  HIPCHK(mm(I, gemm_rm(mo * v, v, v, 1.0, I->plTa, v, false, I->Abc, v, true, 0.0, I->plEc, v), s));
  HIPCHK(cross_scatter_add_rows(I->EM, vv, oo, I->plEc, vv, vv, 1.0, Xo, s));
  {  // rows outside the occupied cross, a = pa: EM[ij][pa][b] += sum_c t^M_ij^{pa c} A^M[b][c]
    Gemm g = gemm_rm(oo, v, v, 1.0, I->plTc, mvp, false, I->Abc, v, true, 1.0, I->EM + (long)pa * v, vv);
    HIPCHK(mm(I, g, s));
  }
  HIPCHK(em_cross_column(I->EM, I->plTc, mvp, I->Abc, o, v, pa, s));  // ... and a != pa, c = pa
  {  // B^M[k][j] = sum_Qd B_Q,kd N^M_Q[j,d]
    Gemm g;
    g.M = o;
    g.N = o;
    g.K = v;
    g.A = I->Bov;
    g.sam = v;
    g.sak = 1;
    g.sar = ov;
    g.B = I->plN;
    g.sbk = 1;
    g.sbn = v;
    g.sbr = ov;
    g.C = I->Bkj;
    g.scm = o;
    g.scn = 1;
    g.nred = Q;
    HIPCHK(mm(I, g, s));
  }
  {  // EM[i][j][ab] += sum_k B^M[k][j] t^M_ik^ab   (batched over i)
    Gemm g;
    g.M = o;
    g.N = vv;
    g.K = o;
    g.A = I->Bkj;
    g.sam = 1;
    g.sak = o;
    g.B = tM;
    g.sbk = vv;
    g.sbn = 1;
    g.sb2 = (long)o * vv;
    g.C = I->EM;
    g.scm = vv;
    g.scn = 1;
    g.sc2 = (long)o * vv;
    g.beta = 1.0;
    g.nb2 = o;
    HIPCHK(mm(I, g, s));
  }
  return ASCC_OK;
}

// One state's residual.  RLx == nullptr: the ladder is computed here into I->RL; otherwise RLx
// already holds this state's particle-particle ladder (from a batched launch).
int residual_core(ascc_ints* I, const double* t1, const double* t2, double* r1, double* r2, double* e,
                  double* RLx, hipStream_t s) {
  double* RL = RLx ? RLx : I->RL;
  const int o = I->no, v = I->nv, Q = I->naux;
  const long n = I->n, nn = n * n, ov = I->ov, oo = I->oo, vv = I->vv, ovov = I->ovov;
  const long wzl = ov + oo;  // row length of WZ and Gwz
  int rc;

  // --- T1 dressing of B and of the one-electron operator, dressed Fock matrix
  phase_begin(I, PH_DRESS, s);
  if ((rc = dress(I, I->B, I->Bc, I->Bh, t1, o, v, Q, s))) return rc;
  if ((rc = dress(I, I->h, I->hc, I->Fh, t1, o, v, 1, s))) return rc;
  if ((rc = add_two_electron_fock(I, I->Fh, I->Bh, I->J, o, v, Q, 1.0, s))) return rc;

  // --- contiguous dressed blocks
  EACH_SLOT {
    int d[4] = {o, v, Q, 1};
    Perm4In x = pin(S(I->Bh) + o * n, 1, n, nn, 0, 1.0);  // B^_ai -> [i][a][Q]
    HIPCHK(permute4(S(I->BvoTt), d, 0.0, &x, 1, s));
    int d2[4] = {Q, o, o, 1};
    x = pin(S(I->Bh), nn, n, 1, 0, 1.0);
    HIPCHK(permute4(S(I->Boo), d2, 0.0, &x, 1, s));
    int d3[4] = {Q, v, v, 1};
    x = pin(S(I->Bh) + o * n + o, nn, n, 1, 0, 1.0);
    HIPCHK(permute4(S(I->Bvv), d3, 0.0, &x, 1, s));
    int d4[4] = {o, v, 1, 1};
    x = pin(S(I->Fh) + o, n, 1, 0, 0, 1.0);  // F^_kc
    HIPCHK(permute4(S(I->Fovh), d4, 0.0, &x, 1, s));
  }

  phase_end(I, s);
  // --- permuted amplitude views: Tx[iajb] = t2[ijba], U[iajb] = 2 t2[ijab] - t2[ijba]
  phase_begin(I, PH_AMP, s);
  double* Tx = I->TU;
  double* U = I->TU + ovov;
  EACH_SLOT {
    int d[4] = {o, v, o, v};
    const long si = (long)o * vv, sj = vv;
    Perm4In x = pin(S(t2), si, 1, sj, v, 1.0);
    HIPCHK(permute4(S(Tx), d, 0.0, &x, 1, s));
    Perm4In y[2] = {pin(S(t2), si, v, sj, 1, 2.0), pin(S(t2), si, 1, sj, v, -1.0)};
    HIPCHK(permute4(S(U), d, 0.0, y, 2, s));
  }
  const bool lowp = I->cur_prec != ASCC_PREC_FP64;
  const long lov = lowp_ld(ov), lQ = lowp_ld(Q), loo = lowp_ld(oo);
  if (lowp) HIPCHK(shadow(I, I->TUf, I->TU, 2 * ov, ov, s));  // Tx|U rows, K = ov

  phase_end(I, s);
  // --- density-fitted dressed integral blocks (K = naux)
  phase_begin(I, PH_DF, s);
  // g^_aibj enters R2 unmultiplied by amplitudes: always FP64, so the low-precision residual's
  // rounding floor stays proportional to the amplitudes
  {  // g^_aibj: a symmetric product, its lower triangle computed and mirrored
    Gemm g = gemm_rm(ov, ov, Q, 1.0, I->BvoTt, Q, false, I->BvoTt, Q, true, 0.0, I->G1, ov);
    g.lower = true;
    HIPCHK(mm(I, g, s));
  }
  if (lowp) {  // the same products on K-contiguous low-precision shadows (B^_kc ones are constant)
    HIPCHK(shadow(I, I->BvoTtf, I->BvoTt, ov, Q, s));
    HIPCHK(shadow_t(I, I->BooTf, I->Boo, oo, oo, Q, s));
    HIPCHK(shadow_t(I, I->BvvTf, I->Bvv, vv, vv, Q, s));
    HIPCHK(glp(lp_nt(I, oo, vv, Q, 1, I->BooTf, lQ, 0, I->BvvTf, lQ, 0, I->G2, vv, 0), s));    // g^_kiac
    HIPCHK(glp(lp_nt(I, ov, ov, Q, 1, I->BvoTtf, lQ, 0, I->BovTf, lQ, 0, I->G3, ov, 0), s));   // g^_aikc
    // N_Q[k,a] = sum_lc B_Q,lc u_kl^ac: U is a symmetric ov x ov matrix, so its rows are its columns
    HIPCHK(glp(lp_nt(I, Q, ov, ov, 1, I->Bovf, lov, 0, I->TUf + ov * lov, lov, 0, I->Nq, ov, 0), s));
  } else {
    HIPCHK(mm(I, gemm_rm(oo, vv, Q, 1.0, I->Boo, oo, true, I->Bvv, vv, false, 0.0, I->G2, vv), s));    // g^_kiac
    HIPCHK(mm(I, gemm_rm(ov, ov, Q, 1.0, I->BvoTt, Q, false, I->BovT, Q, true, 0.0, I->G3, ov), s));   // g^_aikc
    // N_Q[k,a] = sum_lc B_Q,lc u_kl^ac (U is symmetric: its rows are its columns)
    HIPCHK(mm(I, gemm_rm(Q, ov, ov, 1.0, I->Bov, ov, false, U, ov, true, 0.0, I->Nq, ov), s));
  }
  HIPCHK(mm(I, gemm_rm(oo, oo, Q, 1.0, I->Boo, oo, true, I->Boo, oo, false, 0.0, I->G4, oo), s));      // g^_kilj

  phase_end(I, s);
  // --- W_ij[k,b], Z_ij[k,l] in one product against [(kc|bd) | (kc|ld)]
  phase_begin(I, PH_WZ, s);
  if (lowp) {
    const long ld = lowp_ld(vv);
    HIPCHK(shadow(I, I->t2f, t2, oo, vv, s));
    HIPCHK(glp(lp_nt(I, oo, wzl, vv, 1, I->t2f, ld, 0, I->GwzTf, ld, 0, I->WZ, wzl, 0), s));
  } else {
    HIPCHK(mm(I, gemm_rm(oo, wzl, vv, 1.0, t2, vv, false, I->Gwz, vv, true, 0.0, I->WZ, wzl), s));
  }

  phase_end(I, s);
  // --- chi[ij][kl] = g^_kilj + Z_ij[k,l]
  phase_begin(I, PH_HH, s);
  EACH_SLOT {
    int d[4] = {o, o, o, o};
    const long o2 = oo, o3 = oo * o;
    Perm4In x[2] = {pin(S(I->G4), o2, 1, o3, o, 1.0), pin(S(I->WZ) + ov, (long)o * wzl, wzl, o, 1, 1.0)};
    HIPCHK(permute4(S(I->chi), d, 0.0, x, 2, s));
  }

  phase_end(I, s);
  // --- particle-particle ladder over the undressed (ac|bd), plus the hole-hole ladder
  if (!RLx && (rc = pp_ladder(I, t2, s))) return rc;
  phase_begin(I, PH_HH, s);
  if (lowp) {  // RL[ij][ab] += sum_kl chi[ij][kl] t2[kl][ab], with t2 transposed to K = kl contiguous
    HIPCHK(shadow(I, I->chif, I->chi, oo, oo, s));
    HIPCHK(shadow_t(I, I->t2Tf, t2, vv, vv, oo, s));
    GemmLP g = lp_nt(I, oo, vv, oo, 1, I->chif, loo, 0, I->t2Tf, loo, 0, RL, vv, 0);
    g.beta = 1.0;
    HIPCHK(glp(g, s));
  } else {
    HIPCHK(mm(I, gemm_rm(oo, vv, oo, 1.0, I->chi, oo, false, t2, vv, false, 1.0, RL, vv), s));
  }
  phase_end(I, s);

  // --- rings: Y1 = Tx K, Y2 = U L (batched pair)
  phase_begin(I, PH_RING_Y, s);
  if (lowp) {  // K and L are symmetric matrices, so B[n][k] = B[k][n]
    const long ld = lov;
    HIPCHK(glp(lp_nt(I, ov, ov, ov, 2, I->TUf, ld, ov * ld, I->KLf, ld, ov * ld, I->Y, ov, ovov), s));
  } else {
    // K and L are symmetric, so B(k, n) = KL[n][k]: both operands K-contiguous
    Gemm g = gemm_rm(ov, ov, ov, 1.0, I->TU, ov, false, I->KL, ov, true, 0.0, I->Y, ov);
    g.sa2 = ovov;
    g.sb2 = ovov;
    g.sc2 = ovov;
    g.nb2 = 2;
    HIPCHK(mm(I, g, s));
  }
  phase_end(I, s);
  phase_begin(I, PH_RING_XZ, s);
  EACH_SLOT {
    int d[4] = {o, v, o, v};  // (i, a, k, c)
    const long si = vv, sa = v, sk = (long)o * vv, sc = 1;  // G2[k][i][a][c]
    Perm4In x[2] = {pin(S(I->G2), si, sa, sk, sc, 1.0), pin(S(I->Y), (long)v * o * v, (long)o * v, v, 1, -0.5)};
    HIPCHK(permute4(S(I->XZ), d, 0.0, x, 2, s));
    Perm4In z[3] = {pin(S(I->G3), (long)v * o * v, (long)o * v, v, 1, 2.0), pin(S(I->G2), si, sa, sk, sc, -1.0),
                    pin(S(I->Y) + ovov, (long)v * o * v, (long)o * v, v, 1, 0.5)};
    HIPCHK(permute4(S(I->XZ) + ovov, d, 0.0, z, 3, s));
  }
  phase_end(I, s);
  phase_begin(I, PH_RING_P, s);
  if (lowp) {  // P1 = Tx Xc^T, P2 = U Zd^T
    const long ld = lowp_ld(ov);
    HIPCHK(shadow(I, I->XZf, I->XZ, 2 * ov, ov, s));
    HIPCHK(glp(lp_nt(I, ov, ov, ov, 2, I->TUf, ld, ov * ld, I->XZf, ld, ov * ld, I->P, ov, ovov), s));
  } else {
    Gemm g = gemm_rm(ov, ov, ov, 1.0, I->TU, ov, false, I->XZ, ov, true, 0.0, I->P, ov);
    g.sa2 = ovov;
    g.sb2 = ovov;
    g.sc2 = ovov;
    g.nb2 = 2;
    HIPCHK(mm(I, g, s));
  }

  phase_end(I, s);
  phase_begin(I, PH_N5, s);
  // --- E term: F'_bc = F^_bc - sum_Qk N_Q[k,b] B_Q,kc ; F''_kj = F^_kj + sum_Qd B_Q,kd N_Q[j,d]
  HIPCHK(mm(I, gemm_rm(v, v, (long)Q * o, 1.0, I->Nq, v, true, I->Bov, v, false, 0.0, I->Abc, v), s));
  {
    Gemm g;
    g.M = o;
    g.N = o;
    g.K = v;
    g.A = I->Bov;
    g.sam = v;
    g.sak = 1;
    g.sar = ov;
    g.B = I->Nq;
    g.sbk = 1;
    g.sbn = v;
    g.sbr = ov;
    g.C = I->Bkj;
    g.scm = o;
    g.scn = 1;
    g.nred = Q;
    HIPCHK(mm(I, g, s));
  }
  EACH_SLOT {
    int d[4] = {v, v, 1, 1};
    Perm4In x[2] = {pin(S(I->Fh) + o * n + o, n, 1, 0, 0, 1.0), pin(S(I->Abc), v, 1, 0, 0, -1.0)};
    HIPCHK(permute4(S(I->Fvvp), d, 0.0, x, 2, s));
    int d2[4] = {o, o, 1, 1};
    Perm4In y[2] = {pin(S(I->Fh), n, 1, 0, 0, 1.0), pin(S(I->Bkj), o, 1, 0, 0, 1.0)};
    HIPCHK(permute4(S(I->Foop), d2, 0.0, y, 2, s));
  }
  // EM = sum_c t_ij^ac F'_bc
  HIPCHK(mm(I, gemm_rm(oo * v, v, v, 1.0, t2, v, false, I->Fvvp, v, true, 0.0, I->EM, v), s));
  {  // EM[i][j][ab] -= sum_k F''_kj t_ik^ab   (batched over i)
    Gemm g;
    g.M = o;
    g.N = vv;
    g.K = o;
    g.A = I->Foop;
    g.sam = 1;
    g.sak = o;
    g.B = t2;
    g.sbk = vv;
    g.sbn = 1;
    g.sb2 = (long)o * vv;
    g.C = I->EM;
    g.scm = vv;
    g.scn = 1;
    g.sc2 = (long)o * vv;
    g.alpha = -1.0;
    g.beta = 1.0;
    g.nb2 = o;
    HIPCHK(mm(I, g, s));
  }
  {  // W'_ij[k,b] = W_ij[k,b] - 1/2 sum_l Z_ij[k,l] t_l^b   (batched over ij, in place)
    Gemm g;
    g.M = o;
    g.N = v;
    g.K = o;
    g.A = I->WZ + ov;
    g.sam = o;
    g.sak = 1;
    g.sa2 = wzl;
    g.B = t1;
    g.sbk = v;
    g.sbn = 1;
    g.C = I->WZ;
    g.scm = v;
    g.scn = 1;
    g.sc2 = wzl;
    g.alpha = -0.5;
    g.beta = 1.0;
    g.nb2 = oo;
    HIPCHK(mm(I, g, s));
  }
  {  // EM[ij][a][b] -= sum_k t_k^a W'_ij[k,b]
    Gemm g;
    g.M = v;
    g.N = v;
    g.K = o;
    g.A = t1;
    g.sam = 1;
    g.sak = v;
    g.B = I->WZ;
    g.sbk = v;
    g.sbn = 1;
    g.sb2 = wzl;
    g.C = I->EM;
    g.scm = v;
    g.scn = 1;
    g.sc2 = vv;
    g.alpha = -1.0;
    g.beta = 1.0;
    g.nb2 = oo;
    HIPCHK(mm(I, g, s));
  }

  phase_end(I, s);
  if (I->pl_hole >= 0) {
    if (nslots() > 1) return fail(ASCC_E_STATE, "the PLASCC removal is not evaluated in a slot batch");
    phase_begin(I, PH_PLASCC, s);
    if ((rc = plascc_remove(I, t2, RL, s))) return rc;
    phase_end(I, s);
  }
  phase_begin(I, PH_N5, s);
  // --- singles
  {  // r1[i][a] = sum_Qd N_Q[i,d] B^_Q,ad
    Gemm g;
    g.M = o;
    g.N = v;
    g.K = v;
    g.A = I->Nq;
    g.sam = v;
    g.sak = 1;
    g.sar = ov;
    g.B = I->Bvv;
    g.sbk = 1;
    g.sbn = v;
    g.sbr = vv;
    g.C = r1;
    g.scm = v;
    g.scn = 1;
    g.nred = Q;
    HIPCHK(mm(I, g, s));
  }
  // r1 -= sum_Qk B^_Q,ki N_Q[k,a]
  HIPCHK(mm(I, gemm_rm(o, v, (long)Q * o, -1.0, I->Boo, o, true, I->Nq, v, false, 1.0, r1, v), s));
  {  // r1[(ia)] += sum_kc U[(ia),(kc)] F^_kc
    Gemm g;
    g.M = ov;
    g.N = 1;
    g.K = ov;
    g.A = U;
    g.sam = ov;
    g.sak = 1;
    g.B = I->Fovh;
    g.sbk = 1;
    g.sbn = 0;
    g.C = r1;
    g.scm = 1;
    g.scn = 0;
    g.beta = 1.0;
    HIPCHK(mm(I, g, s));
  }
  EACH_SLOT HIPCHK(add_fvo(S(r1), S(I->Fh), o, v, s));

  phase_end(I, s);
  // --- doubles assembly and energy
  phase_begin(I, PH_ASSEMBLE, s);
  EACH_SLOT HIPCHK(assemble_r2(S(r2), S(I->G1), S(RL), S(I->EM), S(I->P), S(I->P) + ovov, o, v, s));
  phase_end(I, s);
  phase_begin(I, PH_ENERGY, s);
  EACH_SLOT HIPCHK(energy(S(e), S(I->partial), S(t1), S(t2), S(I->Lijab), S(I->fov), o, v, s));
  if (g_sb && g_sb->bad) return fail(ASCC_E_STATE, "a residual array lies outside the batch's slot ranges");
  phase_end(I, s);
  return ASCC_OK;
}

int residual_fp64(ascc_ints* I, const double* t1, const double* t2, double* r1, double* r2, double* e,
                  hipStream_t s) {
  return residual_core(I, t1, t2, r1, r2, e, nullptr, s);
}

// Clears the slot-batch context however the batched pass ends.
struct SlotBatchScope {
  explicit SlotBatchScope(SlotBatch* b) {
    g_sb = b;
    g_slot = 0;
    g_enclosing_ok = true;
  }
  ~SlotBatchScope() {
    g_sb = nullptr;
    g_slot = 0;
    g_enclosing_ok = false;
  }
};

// hole >= 0: the integrals of Hbar = e^{S^dagger} H e^{-S^dagger} for S = (s/sqrt 2) sum_spin p^dagger h
// (hole h occupied, particle p virtual, s = s_sign = +-1; Sec. II.A, Eqs. (eqn:1CSF-S), (eqn: sim)).
// S^dagger is one-body with the spatial matrix K = s E_hp / sqrt 2 (K^2 = 0), so every integral index pair
// transforms as x -> (1 + K) x (1 - K): Bbar_Q and hbar, applied right after h is formed, so every
// constant block below is one of Hbar.  The Jacobi denominators keep the diagonal of the given Fock
// matrix; the f_ia of the energy is that of Hbar, fbar = hbar + sum_k [2 (pq|kk)bar - (pk|kq)bar].
int build_constants(ascc_ints* I, const double* Bsrc, const double* fock, int fock_is_diag, int hole, int particle,
                    int s_sign, hipStream_t s) {
  const int o = I->no, v = I->nv, Q = I->naux;
  const long n = I->n, nn = n * n, ov = I->ov, oo = I->oo, vv = I->vv, ovov = I->ovov;
  const long wzl = ov + oo;
  HIPCHK(d_copy(I->B, Bsrc, sizeof(double) * Q * nn, hipMemcpyDeviceToDevice, s));
  // Fock matrix -> h (start), eps, fov
  if (fock_is_diag) {
    HIPCHK(d_copy(I->eps, fock, sizeof(double) * n, hipMemcpyDeviceToDevice, s));
    int d[4] = {(int)n, (int)n, 1, 1};
    // h = diag(eps): write zeros (no inputs), then the diagonal
    HIPCHK(permute4(I->h, d, 0.0, nullptr, 0, s));
    long ostr[4] = {n + 1, 0, 0, 0};
    int dd[4] = {(int)n, 1, 1, 1};
    Perm4In x = pin(fock, 1, 0, 0, 0, 1.0);
    HIPCHK(permute4_strided(I->h, ostr, dd, 0.0, &x, 1, s));
  } else {
    HIPCHK(d_copy(I->h, fock, sizeof(double) * nn, hipMemcpyDeviceToDevice, s));
    int dd[4] = {(int)n, 1, 1, 1};
    Perm4In x = pin(fock, n + 1, 0, 0, 0, 1.0);
    HIPCHK(permute4(I->eps, dd, 0.0, &x, 1, s));
  }
  {
    int d[4] = {o, v, 1, 1};
    Perm4In x = pin(I->h + o, n, 1, 0, 0, 1.0);  // still the Fock matrix here
    HIPCHK(permute4(I->fov, d, 0.0, &x, 1, s));
  }
  // h = f - sum_k (2 (pq|kk) - (pk|kq))
  int rc = add_two_electron_fock(I, I->h, I->B, I->J, o, v, Q, -1.0, s);
  if (rc) return rc;
  if (hole >= 0) {
    const double c = s_sign / std::sqrt(2.0);
    HIPCHK(onebody_transform(I->B, Q, (int)n, hole, particle, c, s));
    HIPCHK(onebody_transform(I->h, 1, (int)n, hole, particle, c, s));
    HIPCHK(d_copy(I->Fh, I->h, sizeof(double) * nn, hipMemcpyDeviceToDevice, s));
    if ((rc = add_two_electron_fock(I, I->Fh, I->B, I->J, o, v, Q, 1.0, s))) return rc;  // fbar
    int d[4] = {o, v, 1, 1};
    Perm4In x = pin(I->Fh + o, n, 1, 0, 0, 1.0);
    HIPCHK(permute4(I->fov, d, 0.0, &x, 1, s));
    // the transformed reference energy, while Fh still holds fbar (residuals reuse Fh as work)
    HIPCHK(reference_energy(I->e0, I->h, n + 1, nn, I->Fh, n + 1, nn, o, s));
  } else {
    HIPCHK(reference_energy(I->e0, I->h, n + 1, nn, I->eps, 1, n, o, s));
  }

  // B_ov and the undressed B_vv, the latter as [a][c][Q] (K = Q contiguous, into the work array Bvv,
  // which every residual overwrites with the dressed [Q][a][c])
  {
    int d[4] = {Q, o, v, 1};
    Perm4In x = pin(I->B + o, nn, n, 1, 0, 1.0);
    HIPCHK(permute4(I->Bov, d, 0.0, &x, 1, s));
    int dt[4] = {o, v, Q, 1};
    Perm4In xt = pin(I->B + o, n, 1, nn, 0, 1.0);  // B_kc -> [k][c][Q]
    HIPCHK(permute4(I->BovT, dt, 0.0, &xt, 1, s));
    int d2[4] = {v, v, Q, 1};
    Perm4In y = pin(I->B + o * n + o, n, 1, nn, 0, 1.0);
    HIPCHK(permute4(I->Bvv, d2, 0.0, &y, 1, s));
  }
  // J = (ia|jb) into G1 (work), then K and L
  double* Jov = I->G1;
  HIPCHK(mm(I, gemm_rm(ov, ov, Q, 1.0, I->BovT, Q, false, I->BovT, Q, true, 0.0, Jov, ov), s));
  {
    int d[4] = {o, v, o, v};
    const long si = (long)v * o * v, sa = (long)o * v, sj = v, sb = 1;
    Perm4In x = pin(Jov, si, sb, sj, sa, 1.0);  // (ib|ja)
    HIPCHK(permute4(I->KL, d, 0.0, &x, 1, s));
    Perm4In y[2] = {pin(Jov, si, sa, sj, sb, 2.0), pin(Jov, si, sb, sj, sa, -1.0)};
    HIPCHK(permute4(I->KL + ovov, d, 0.0, y, 2, s));
    int d2[4] = {o, o, v, v};  // (i, j, a, b) <- L[i][a][j][b]
    Perm4In z = pin(I->KL + ovov, si, sj, sa, sb, 1.0);
    HIPCHK(permute4(I->Lijab, d2, 0.0, &z, 1, s));
  }
  // Gwz: (kc|bd) at [k*v + b][c][d] from a temporary [(k,c)][(b,d)] product (rows K-contiguous)
  {
    double* tmp = nullptr;
    Pool tmp_alloc = sub_pool(I->pool);
    int rc2 = dalloc(tmp_alloc, &tmp, (size_t)ov * vv);
    if (rc2) return rc2;
    hipError_t e = mm(I, gemm_rm(ov, vv, Q, 1.0, I->BovT, Q, false, I->Bvv, Q, true, 0.0, tmp, vv), s);
    if (e == hipSuccess) {
      int d[4] = {o, v, v, v};  // Gwz[k][b][c][d] <- tmp[k][c][b][d]: d contiguous on both sides
      Perm4In x = pin(tmp, (long)v * vv, v, vv, 1, 1.0);
      e = permute4(I->Gwz, d, 0.0, &x, 1, s);
    }
    if (e == hipSuccess) {
      int d[4] = {o, o, v, v};  // Gwz[ov + k*o + l][c][d] <- J[k][c][l][d]
      Perm4In x = pin(Jov, (long)v * o * v, v, (long)o * v, 1, 1.0);
      e = permute4(I->Gwz + ov * vv, d, 0.0, &x, 1, s);
    }
    if (e == hipSuccess && !tmp_alloc.base) e = d_sync(s);  // carved temporaries need no wait
    free_all(tmp_alloc);
    if (e != hipSuccess) {
      if (bounds_checking() && e == hipErrorInvalidValue) return ASCC_E_HIP;  // message already set
      set_error(std::string("building (kc|bd): ") + hipGetErrorString(e));
      return ASCC_E_HIP;
    }
  }
  // V[a][b][c][d] = (ac|bd) = sum_Q B_Q,ac B_Q,bd, batched over (a, b), in chunks of a.  Both
  // operands are rows of the [a][c][Q] B_vv: K-contiguous.  The packed halves read only the slabs
  // with b >= a (V[a][b][d][c] = (ad|bc) is the same slab), so a packed build starts b at the
  // chunk's first a; the full matrix needs every b.
  const bool full = I->vvvv_mode == ASCC_VVVV_FULL;
  auto vslab = [&](int a0, int na, double* dst) -> hipError_t {
    const int b0 = full ? 0 : a0;
    Gemm g;
    g.M = v;
    g.N = v;
    g.K = Q;
    g.A = I->Bvv + (long)a0 * v * Q;
    g.sam = Q;
    g.sak = 1;
    g.sa1 = (long)v * Q;
    g.B = I->Bvv + (long)b0 * v * Q;
    g.sbk = 1;
    g.sbn = Q;
    g.sb2 = (long)v * Q;
    g.C = dst + (long)b0 * vv;
    g.scm = v;
    g.scn = 1;
    g.sc1 = (long)v * vv;
    g.sc2 = vv;
    g.nb1 = na;
    g.nb2 = v - b0;
    return mm(I, g, s);
  };
  // in chunks of a through a temporary: scattered to the full matrix in pair order, or packed
  if (full) HIPCHK(pair_minus_rows(pair_minus(I), v, s));
  long ac = 1;
  const long elems = build_temp_elems(o, v, I->vvvv_mode, &ac);
  double* tmp = nullptr;
  Pool tmp_alloc = sub_pool(I->pool);
  int rc3 = dalloc(tmp_alloc, &tmp, (size_t)elems);
  if (rc3) return rc3;
  hipError_t e = hipSuccess;
  for (int a0 = 0; a0 < v && e == hipSuccess; a0 += (int)ac) {
    const int na = (int)std::min<long>(ac, v - a0);
    e = vslab(a0, na, tmp);
    if (e == hipSuccess) e = full ? pack_full(I->V, tmp, a0, a0 + na, v, s) : pack_vvvv(I->V, tmp, a0, a0 + na, v, s);
  }
  if (e == hipSuccess && !tmp_alloc.base) e = d_sync(s);  // carved temporaries need no wait
  free_all(tmp_alloc);
  if (e != hipSuccess) {
    if (!(bounds_checking() && e == hipErrorInvalidValue)) set_error(std::string("building vvvv: ") + hipGetErrorString(e));
    return ASCC_E_HIP;
  }
  return ASCC_OK;
}

// FP32 shadows of the constant operands: (ac|bd), [(kc|bd)|(kc|ld)] as [n][(cd)], K|L.
int build_lowp_shadows(ascc_ints* I, hipStream_t s) {
  const long vv = I->vv, ov = I->ov, oo = I->oo, wzl = ov + oo;
  const long Tv = (long)I->nv * (I->nv + 1) / 2;

  if (I->vvvv_mode == ASCC_VVVV_FULL) {  // the packed halves, formed from the full matrix
    const int prec = (I->cur_prec == ASCC_PREC_BF16X3) ? kPrecBF16x3 : kPrecFP32;
    HIPCHK(to_lowp_pm(prec, I->Vf, lowp_ld(Tv), I->V, vv, vv, pair_minus(I), Tv, s));
  } else {
    HIPCHK(shadow(I, I->Vf, I->V, 2 * Tv, Tv, s));
  }
  HIPCHK(shadow(I, I->KLf, I->KL, 2 * ov, ov, s));
  const long Q = I->naux;
  HIPCHK(shadow(I, I->BovTf, I->BovT, ov, Q, s));      // B_kc (undressed by T1) as [kc][Q]
  HIPCHK(shadow(I, I->Bovf, I->Bov, Q, ov, s));         // and as [Q][kc]
  const hipError_t e = shadow(I, I->GwzTf, I->Gwz, wzl, vv, s);  // Gwz rows are K-contiguous already
  if (e != hipSuccess) {
    if (!(bounds_checking() && e == hipErrorInvalidValue)) set_error(std::string("FP32 shadows: ") + hipGetErrorString(e));
    return ASCC_E_HIP;
  }
  return ASCC_OK;
}

int check_shape(int no, int nv, int naux) {
  if (no < 1 || nv < 1 || naux < 1) return fail(ASCC_E_SHAPE, "no, nv and naux must be >= 1");
  if (no > 256 || nv > 4096 || naux > 65535)
    return fail(ASCC_E_SHAPE, "no <= 256, nv <= 4096 and naux <= 65535 are supported");
  const double n4 = (double)nv * nv * nv * nv;
  if (n4 > 9.0e18) return fail(ASCC_E_SHAPE, "nv too large");
  return ASCC_OK;
}

// The residual work arrays of an integral set (what one state's residual writes; not the
// ladder operands, which a batch stacks separately), FP64 then low precision, in carving order.
bool is_constant(double* ascc_ints::*m) {
  return m == &ascc_ints::B || m == &ascc_ints::h || m == &ascc_ints::eps || m == &ascc_ints::fov ||
         m == &ascc_ints::e0 || m == &ascc_ints::Bov || m == &ascc_ints::KL || m == &ascc_ints::Lijab ||
         m == &ascc_ints::Gwz || m == &ascc_ints::BovT || m == &ascc_ints::V || m == &ascc_ints::pairtab ||
         m == &ascc_ints::Tp || m == &ascc_ints::Rp;
}
bool is_constant(float* ascc_ints::*m) {
  return m == &ascc_ints::Vf || m == &ascc_ints::GwzTf || m == &ascc_ints::KLf || m == &ascc_ints::BovTf ||
         m == &ascc_ints::Bovf || m == &ascc_ints::Tpf;
}
size_t work_block_bytes(long o, long v, long Q, int precision, int mode) {
  size_t off = 0;
  for (const auto& item : ints_plan(o, v, Q, mode))
    if (!is_constant(item.first)) off = align_up(off) + std::max<size_t>((size_t)item.second, 1) * sizeof(double);
  if (precision != ASCC_PREC_FP64)
    for (const auto& item : lowp_plan(o, v, Q, mode))
      if (!is_constant(item.first)) off = align_up(off) + std::max<size_t>((size_t)item.second, 1) * sizeof(float);
  return align_up(off);
}
// Stacked ladder operands and results for max_states states, then `group` work blocks (group > 1).
size_t batch_footprint(long o, long v, long Q, int precision, int mode, long max_states, int group) {
  const long To = o * (o + 1) / 2, Tv = v * (v + 1) / 2;
  const long rows = 2 * To * Tv, lrows = 2 * To * lowp_ld(Tv);
  size_t off = align_up(sizeof(double) * (size_t)(max_states * rows));
  off += align_up(sizeof(double) * (size_t)(max_states * rows));
  off += align_up(sizeof(double) * (size_t)(max_states * o * o * v * v));
  if (precision != ASCC_PREC_FP64) off += align_up(sizeof(float) * (size_t)(max_states * lrows));
  if (group > 1) off += (size_t)group * work_block_bytes(o, v, Q, precision, mode);
  return off;
}

int batch_reserve_impl(ascc_ints* I, int max_states, int group, void* ws, size_t ws_bytes) {
  if (max_states < 1 || max_states > 4096) return fail(ASCC_E_ARG, "max_states must be in 1..4096");
  if (group < 1 || group > max_states) return fail(ASCC_E_ARG, "group must be in 1..max_states");
  if (ws && (reinterpret_cast<uintptr_t>(ws) % kAlign)) return fail(ASCC_E_ARG, "workspace must be 256-byte aligned");
  const size_t need = batch_footprint(I->no, I->nv, I->naux, I->precision, I->vvvv_mode, max_states, group);
  if (ws && ws_bytes < need) return fail(ASCC_E_NOMEM, "batch workspace too small: needs " + std::to_string(need) + " bytes");
  free_all(I->batch);
  I->batch = Pool();
  I->max_states = 0;
  I->group = 1;
  I->group_base = nullptr;
  I->group_block = 0;
  I->Tp_all = I->Rp_all = I->RL_all = nullptr;
  I->Tpf_all = nullptr;
  if (ws) {
    I->batch.base = static_cast<char*>(ws);
    I->batch.size = ws_bytes;
  }
  const long o = I->no, v = I->nv, To = o * (o + 1) / 2, Tv = v * (v + 1) / 2;
  const long rows = 2 * To * Tv, lrows = 2 * To * lowp_ld(Tv);
  int rc = dalloc(I->batch, &I->Tp_all, (size_t)(max_states * rows));
  if (!rc) rc = dalloc(I->batch, &I->Rp_all, (size_t)(max_states * rows));
  if (!rc) rc = dalloc(I->batch, &I->RL_all, (size_t)(max_states * I->oovv));
  if (!rc && I->precision != ASCC_PREC_FP64) rc = dalloc(I->batch, &I->Tpf_all, (size_t)(max_states * lrows));
  if (!rc && group > 1) {
    I->group_block = work_block_bytes(o, v, I->naux, I->precision, I->vvvv_mode);
    rc = dalloc(I->batch, &I->group_base, (size_t)group * I->group_block);
  }
  if (rc) {
    free_all(I->batch);
    I->batch = Pool();
    return rc;
  }
  I->max_states = max_states;
  I->group = group;
  return ASCC_OK;
}

// The residual terms other than the pp ladder (already in RL) of n states as one batched pass: the
// handle's work arrays are pointed at the first of the group work blocks for the pass (the states'
// arrays sit one block apart), the shared integrals are used by every state, and the states' own
// arrays are evenly spaced (t1[k] = t1[0] + k (t1[1] - t1[0]), likewise t2, r1, r2; e[k]; RL[k] one
// o^2 v^2 block apart).
int residual_group(ascc_ints* I, int n, int nstates, const double* const* t1, const double* const* t2,
                   double* const* r1, double* const* r2, double* e, double* RL, hipStream_t s) {
  if (n == 1) return residual_core(I, t1[0], t2[0], r1[0], r2[0], e, RL, s);
  const long o = I->no, v = I->nv, Q = I->naux;
  // point every work array at block 0 (restored below)
  std::vector<std::pair<double* ascc_ints::*, double*>> saved;
  std::vector<std::pair<float* ascc_ints::*, float*>> savedf;
  size_t off = 0;
  for (const auto& item : ints_plan(o, v, Q, I->vvvv_mode))
    if (!is_constant(item.first)) {
      off = align_up(off);
      saved.push_back({item.first, I->*(item.first)});
      I->*(item.first) = reinterpret_cast<double*>(I->group_base + off);
      off += std::max<size_t>((size_t)item.second, 1) * sizeof(double);
    }
  if (I->precision != ASCC_PREC_FP64)
    for (const auto& item : lowp_plan(o, v, Q, I->vvvv_mode))
      if (!is_constant(item.first)) {
        off = align_up(off);
        savedf.push_back({item.first, I->*(item.first)});
        I->*(item.first) = reinterpret_cast<float*>(I->group_base + off);
        off += std::max<size_t>((size_t)item.second, 1) * sizeof(float);
      }
  SlotBatch sb;
  sb.n = n;
  auto add = [&](const void* p, size_t bytes, long stride) {
    const uintptr_t lo = reinterpret_cast<uintptr_t>(p);
    sb.ranges.push_back({lo, lo + bytes, stride});
  };
  auto step = [&](const void* const* a) {
    return nstates > 1 ? (long)((const char*)a[1] - (const char*)a[0]) : 0L;
  };
  add(I->group_base, I->group_block, (long)I->group_block);
  add(t1[0], sizeof(double) * I->ov, step((const void* const*)t1));
  add(t2[0], sizeof(double) * I->oovv, step((const void* const*)t2));
  add(r1[0], sizeof(double) * I->ov, step((const void* const*)r1));
  add(r2[0], sizeof(double) * I->oovv, step((const void* const*)r2));
  add(e, sizeof(double), (long)sizeof(double));
  add(RL, sizeof(double) * I->oovv, (long)(sizeof(double) * I->oovv));
  for (const auto& item : ints_plan(o, v, Q, I->vvvv_mode))  // shared integrals: stride 0
    if (is_constant(item.first) && I->*(item.first))
      add(I->*(item.first), std::max<size_t>((size_t)item.second, 1) * sizeof(double), 0);
  if (I->precision != ASCC_PREC_FP64)
    for (const auto& item : lowp_plan(o, v, Q, I->vvvv_mode))
      if (is_constant(item.first) && I->*(item.first))
        add(I->*(item.first), std::max<size_t>((size_t)item.second, 1) * sizeof(float), 0);
  int rc;
  {
    SlotBatchScope scope(&sb);
    rc = residual_core(I, t1[0], t2[0], r1[0], r2[0], e, RL, s);
  }
  for (auto& x : saved) I->*(x.first) = x.second;
  for (auto& x : savedf) I->*(x.first) = x.second;
  return rc;
}

// Work buffers of the PLASCC removal (compact cross slabs, see plascc_remove), in carving order.
std::vector<std::pair<double* ascc_ints::*, long>> plascc_plan(long o, long v, long Q) {
  const long ov = o * v, oo = o * o, vv = v * v;
  const long m = o + v - 1, mp = pad_even(m);
  const long mo = 2 * o - 1, mop = pad_even(mo), mvp = pad_even(2 * v - 1);
  return {
      {&ascc_ints::plA, m * ov},    {&ascc_ints::plC, ov * mp},   {&ascc_ints::plKr, m * ov},
      {&ascc_ints::plKpp, m * mp},  {&ascc_ints::plYp, m * ov},   {&ascc_ints::plYpp, m * mp},
      {&ascc_ints::plS, m * mp},    {&ascc_ints::plZ, m * ov},    {&ascc_ints::plZt, ov * mp},
      {&ascc_ints::plW, ov * mp},   {&ascc_ints::plN, Q * ov},    {&ascc_ints::plBp, Q * mp},
      {&ascc_ints::plNw, Q * mp},   {&ascc_ints::plTa, mo * vv},  {&ascc_ints::plTc, oo * mvp},
      {&ascc_ints::plGc, oo * mvp}, {&ascc_ints::plZo, mo * oo},  {&ascc_ints::plZh, oo * mop},
      {&ascc_ints::plRc, oo * mvp}, {&ascc_ints::plEc, mo * vv},
  };
}

size_t plascc_footprint(long o, long v, long Q) {
  size_t off = 0;
  for (const auto& item : plascc_plan(o, v, Q))
    off = align_up(off) + std::max<size_t>((size_t)item.second, 1) * sizeof(double);
  return align_up(off);
}

// ascc_set_plascc (ws == nullptr: library-allocated buffers, cleared synchronously) and
// ascc_set_plascc_ws (carved from the caller's workspace, cleared by a kernel on `s`; no
// allocation and no synchronisation).
int set_plascc_impl(ascc_ints* I, int hole, int particle, void* ws, size_t ws_bytes, hipStream_t s) {
  if (!I) return fail(ASCC_E_ARG, "NULL handle");
  if (hole < 0) {  // back to the full equations; the buffers stay for a later call
    I->pl_hole = I->pl_pa = -1;
    return ASCC_OK;
  }
  if (hole >= I->no || particle < I->no || particle >= I->n)
    return fail(ASCC_E_ARG, "hole must be an occupied and particle a virtual orbital index");
  if (ws && I->pl.total && I->pl.base != static_cast<char*>(ws))
    return fail(ASCC_E_STATE, "PLASCC buffers of this integral set already live elsewhere");
  if (!I->pl.total) {
    const auto plan = plascc_plan(I->no, I->nv, I->naux);
    if (ws) {
      if (reinterpret_cast<uintptr_t>(ws) % kAlign) return fail(ASCC_E_ARG, "workspace must be 256-byte aligned");
      const size_t need = plascc_footprint(I->no, I->nv, I->naux);
      if (ws_bytes < need)
        return fail(ASCC_E_NOMEM, "PLASCC workspace too small: needs " + std::to_string(need) + " bytes");
      I->pl.base = static_cast<char*>(ws);
      I->pl.size = ws_bytes;
    }
    int rc = ASCC_OK;
    for (const auto& item : plan)
      if (!rc) rc = dalloc(I->pl, &(I->*(item.first)), (size_t)item.second);
    // padding columns that products read but never write (plW) must hold zeros: clear them all
    for (const auto& item : plan) {
      if (rc) break;
      if (ws) {  // a fill kernel on the caller's stream, ordered before every later residual on it
        const int d[4] = {1, 1, 1, (int)std::max<long>(item.second, 1)};
        if (permute4(I->*(item.first), d, 0.0, nullptr, 0, s) != hipSuccess)
          rc = fail(ASCC_E_HIP, "clearing the PLASCC buffers failed");
      } else if (!dry_run() && hipMemset(I->*(item.first), 0, sizeof(double) * item.second) != hipSuccess) {
        rc = fail(ASCC_E_HIP, "clearing the PLASCC buffers failed");
      }
    }
    // the allocating form waits for its clears, so that work on any stream (non-blocking ones too)
    // sees zeros
    if (!rc && !ws && !dry_run() && hipStreamSynchronize(nullptr) != hipSuccess)
      rc = fail(ASCC_E_HIP, "clearing the PLASCC buffers failed");
    if (rc) {
      free_all(I->pl);
      I->pl = Pool();
      return rc;
    }
  }
  I->pl_hole = hole;
  I->pl_pa = particle - I->no;
  return ASCC_OK;
}

}  // namespace

extern "C" {

const char* ascc_last_error(void) { return g_last_error.c_str(); }

int ascc_workspace_bytes(int no, int nv, int naux, int precision, int vvvv_mode, int diis_size, size_t* ints_bytes,
                         size_t* diis_bytes) {
  int rc = check_shape(no, nv, naux);
  if (rc) return rc;
  if (precision < ASCC_PREC_FP64 || precision > ASCC_PREC_BF16X3) return fail(ASCC_E_ARG, "unsupported precision");
  if (vvvv_mode != ASCC_VVVV_FULL && vvvv_mode != ASCC_VVVV_PACKED) return fail(ASCC_E_ARG, "unsupported vvvv_mode");
  if (diis_size < 1 || diis_size > kMaxDiis) return fail(ASCC_E_ARG, "diis_size must be in 1..16");
  if (ints_bytes) *ints_bytes = ints_footprint(no, nv, naux, precision, vvvv_mode);
  if (diis_bytes) *diis_bytes = diis_footprint(no, nv, diis_size);
  return ASCC_OK;
}

int ascc_set_precision(ascc_ints* I, int precision) {
  if (!I) return fail(ASCC_E_ARG, "NULL handle");
  if (precision < ASCC_PREC_FP64 || precision > ASCC_PREC_BF16X3) return fail(ASCC_E_ARG, "unsupported precision");
  if (precision != ASCC_PREC_FP64 && I->precision == ASCC_PREC_FP64)
    return fail(ASCC_E_STATE, "integral set was built for FP64 only (no low-precision shadows)");
  if (precision != ASCC_PREC_FP64 && precision != I->precision)
    return fail(ASCC_E_STATE, "integral set holds shadows for its build precision only");
  I->cur_prec = precision;
  return ASCC_OK;
}

int ascc_get_precision(const ascc_ints* I) { return I ? I->cur_prec : -1; }

int ascc_phase_count(void) { return kNumPhases; }

const char* ascc_phase_name(int k) { return (k >= 0 && k < kNumPhases) ? kPhaseNames[k] : ""; }

int ascc_timing_enable(ascc_ints* I, int on) {
  if (!I) return fail(ASCC_E_ARG, "NULL handle");
  I->timing = (on != 0);
  return ASCC_OK;
}

int ascc_timing_read(ascc_ints* I, double* ms, int* counts, int n) {
  if (!I || !ms || !counts || n < kNumPhases) return fail(ASCC_E_ARG, "ascc_timing_read needs arrays of ascc_phase_count() entries");
  for (int k = 0; k < n; ++k) {
    ms[k] = 0.0;
    counts[k] = 0;
  }
  int rc = ASCC_OK;
  for (auto& m : I->marks) {
    float t = 0.f;
    hipError_t e = hipEventSynchronize(m.second.second);
    if (e == hipSuccess) e = hipEventElapsedTime(&t, m.second.first, m.second.second);
    if (e != hipSuccess && rc == ASCC_OK) rc = fail(ASCC_E_HIP, std::string("event timing: ") + hipGetErrorString(e));
    ms[m.first] += t;
    counts[m.first] += 1;
    I->event_pool.push_back(m.second.first);
    I->event_pool.push_back(m.second.second);
  }
  I->marks.clear();
  return rc;
}

int ascc_plascc_workspace_bytes(int no, int nv, int naux, size_t* bytes) {
  int rc = check_shape(no, nv, naux);
  if (rc) return rc;
  if (!bytes) return fail(ASCC_E_ARG, "NULL argument to ascc_plascc_workspace_bytes");
  *bytes = plascc_footprint(no, nv, naux);
  return ASCC_OK;
}

int ascc_set_plascc(ascc_ints* I, int hole, int particle) {
  return set_plascc_impl(I, hole, particle, nullptr, 0, nullptr);
}

int ascc_set_plascc_ws(ascc_ints* I, int hole, int particle, void* d_workspace, size_t ws_bytes, void* stream) {
  if (hole >= 0 && !d_workspace) return fail(ASCC_E_ARG, "NULL workspace for ascc_set_plascc_ws");
  return set_plascc_impl(I, hole, particle, d_workspace, ws_bytes, static_cast<hipStream_t>(stream));
}

int ascc_reference_energy(const ascc_ints* I, double* e0, void* stream) {
  if (!I || !e0) return fail(ASCC_E_ARG, "NULL argument to ascc_reference_energy");
  if (dry_run()) {
    *e0 = 0.0;
    return ASCC_OK;
  }
  hipStream_t s = static_cast<hipStream_t>(stream);
  if (d_copy(e0, I->e0, sizeof(double), hipMemcpyDeviceToHost, s) != hipSuccess || d_sync(s) != hipSuccess)
    return fail(ASCC_E_HIP, "reading the reference energy failed");
  return ASCC_OK;
}

int ascc_ints_shape(const ascc_ints* I, int* no, int* nv, int* naux) {
  if (!I) return fail(ASCC_E_ARG, "NULL handle");
  if (no) *no = I->no;
  if (nv) *nv = I->nv;
  if (naux) *naux = I->naux;
  return ASCC_OK;
}

static int build_ints_impl(const double* d_B, const double* d_fock, int fock_is_diag, int no, int nv, int naux,
                           int precision, int vvvv_mode, int hole, int particle, int s_sign, void* ws,
                           size_t ws_bytes, void* stream, ascc_ints** out);

int ascc_build_ints(const double* d_B, const double* d_fock, int fock_is_diag, int no, int nv, int naux, int precision,
                    int vvvv_mode, void* stream, ascc_ints** out) {
  return build_ints_impl(d_B, d_fock, fock_is_diag, no, nv, naux, precision, vvvv_mode, -1, -1, 1, nullptr, 0, stream,
                         out);
}

int ascc_build_ints_hbar(const double* d_B, const double* d_fock, int fock_is_diag, int no, int nv, int naux,
                         int precision, int vvvv_mode, int hole, int particle, int s_sign, void* stream,
                         ascc_ints** out) {
  if (out) *out = nullptr;
  if (hole < 0 || hole >= no || particle < no || particle >= no + nv)
    return fail(ASCC_E_ARG, "hole must be an occupied and particle a virtual orbital index");
  if (s_sign != 1 && s_sign != -1) return fail(ASCC_E_ARG, "s_sign must be +1 or -1");
  return build_ints_impl(d_B, d_fock, fock_is_diag, no, nv, naux, precision, vvvv_mode, hole, particle, s_sign, nullptr,
                         0, stream, out);
}

int ascc_build_ints_hbar_ws(const double* d_B, const double* d_fock, int fock_is_diag, int no, int nv, int naux,
                            int precision, int vvvv_mode, int hole, int particle, int s_sign, void* d_workspace,
                            size_t ws_bytes, void* stream, ascc_ints** out) {
  if (out) *out = nullptr;
  if (!d_workspace) return fail(ASCC_E_ARG, "d_workspace is NULL");
  if (hole < 0 || hole >= no || particle < no || particle >= no + nv)
    return fail(ASCC_E_ARG, "hole must be an occupied and particle a virtual orbital index");
  if (s_sign != 1 && s_sign != -1) return fail(ASCC_E_ARG, "s_sign must be +1 or -1");
  return build_ints_impl(d_B, d_fock, fock_is_diag, no, nv, naux, precision, vvvv_mode, hole, particle, s_sign,
                         d_workspace, ws_bytes, stream, out);
}

int ascc_initial_guess(double* d_t1, double* d_t2, int no, int nv, int hole, int particle, double beta, double gamma,
                       void* stream) {
  if (!d_t1 || !d_t2) return fail(ASCC_E_ARG, "NULL amplitude array");
  if (no < 1 || nv < 1 || hole < 0 || hole >= no || particle < no || particle >= no + nv)
    return fail(ASCC_E_ARG, "hole must be an occupied and particle a virtual orbital index");
  ScopedBuffers user;
  user.add(d_t1, sizeof(double) * no * nv);
  user.add(d_t2, sizeof(double) * no * no * nv * nv);
  HIPCHK(initial_guess(d_t1, d_t2, no, nv, hole, particle - no, beta / std::sqrt(2.0), gamma,
                       static_cast<hipStream_t>(stream)));
  return ASCC_OK;
}

int ascc_build_ints_ws(const double* d_B, const double* d_fock, int fock_is_diag, int no, int nv, int naux,
                       int precision, int vvvv_mode, void* d_workspace, size_t ws_bytes, void* stream,
                       ascc_ints** out) {
  if (!d_workspace) return fail(ASCC_E_ARG, "d_workspace is NULL");
  return build_ints_impl(d_B, d_fock, fock_is_diag, no, nv, naux, precision, vvvv_mode, -1, -1, 1, d_workspace,
                         ws_bytes, stream, out);
}

// Check mode only: the Jacobi denominators e_i - e_a (Sec. III.B) must all be negative, so the
// largest occupied orbital energy (the Fock diagonal) must lie below the smallest virtual one.
static int check_orbital_energies(const double* d_fock, int fock_is_diag, long o, long n, hipStream_t s) {
  if (!bounds_checking() || dry_run()) return ASCC_OK;
  std::vector<double> f(fock_is_diag ? n : n * n);
  if (d_copy(f.data(), d_fock, sizeof(double) * f.size(), hipMemcpyDeviceToHost, s) != hipSuccess ||
      d_sync(s) != hipSuccess)
    return fail(ASCC_E_HIP, "reading the Fock diagonal failed");
  double omax = -HUGE_VAL, vmin = HUGE_VAL;
  for (long p = 0; p < n; ++p) {
    const double e = fock_is_diag ? f[p] : f[p * n + p];
    if (p < o)
      omax = std::max(omax, e);
    else
      vmin = std::min(vmin, e);
  }
  if (!(omax < vmin))
    return fail(ASCC_E_ARG, "orbital energies: the largest occupied one (" + std::to_string(omax) +
                                ") is not below the smallest virtual one (" + std::to_string(vmin) + ")");
  return ASCC_OK;
}

static int build_ints_impl(const double* d_B, const double* d_fock, int fock_is_diag, int no, int nv, int naux,
                           int precision, int vvvv_mode, int hole, int particle, int s_sign, void* ws,
                           size_t ws_bytes, void* stream, ascc_ints** out) {
  if (!out) return fail(ASCC_E_ARG, "out is NULL");
  *out = nullptr;
  if (!d_B || !d_fock) return fail(ASCC_E_ARG, "d_B and d_fock must be device pointers");
  int rc = check_shape(no, nv, naux);
  if (rc) return rc;
  if (precision < ASCC_PREC_FP64 || precision > ASCC_PREC_BF16X3) return fail(ASCC_E_ARG, "unsupported precision");
  if (vvvv_mode != ASCC_VVVV_FULL && vvvv_mode != ASCC_VVVV_PACKED) return fail(ASCC_E_ARG, "unsupported vvvv_mode");
  hipStream_t s = static_cast<hipStream_t>(stream);
  ascc_ints* I = new ascc_ints();
  I->no = no;
  I->nv = nv;
  I->naux = naux;
  I->n = no + nv;
  I->precision = precision;
  I->vvvv_mode = vvvv_mode;
  if (!dry_run()) (void)hipGetDevice(&I->device);
  const long o = no, v = nv, Q = naux, n = o + v, nn = n * n;
  I->ov = o * v;
  I->oo = o * o;
  I->vv = v * v;
  I->ovov = I->ov * I->ov;
  I->oovv = I->oo * I->vv;
  if (ws) {
    if ((reinterpret_cast<uintptr_t>(ws) & (kAlign - 1)) != 0) {
      delete I;
      return fail(ASCC_E_ARG, "d_workspace must be 256-byte aligned");
    }
    I->pool.base = static_cast<char*>(ws);
    I->pool.size = ws_bytes;
    register_buffer(ws, ws_bytes);
  }
  rc = ASCC_OK;
  for (const auto& item : ints_plan(no, nv, naux, vvvv_mode)) {
    if (!rc) rc = dalloc(I->pool, &(I->*(item.first)), (size_t)item.second);
  }
  if (precision != ASCC_PREC_FP64) {
    for (const auto& item : lowp_plan(no, nv, naux, vvvv_mode)) {
      if (!rc) rc = dalloc(I->pool, &(I->*(item.first)), (size_t)item.second);
    }
  }
  I->cur_prec = precision;
  ScopedBuffers user;
  user.add(d_B, sizeof(double) * Q * nn);
  user.add(d_fock, sizeof(double) * (fock_is_diag ? n : nn));
  if (!rc) rc = check_orbital_energies(d_fock, fock_is_diag, o, n, s);
  if (!rc) rc = build_constants(I, d_B, d_fock, fock_is_diag, hole, particle, s_sign, s);
  if (!rc && precision != ASCC_PREC_FP64) rc = build_lowp_shadows(I, s);
  if (!rc && !ws) {  // a workspace build stays asynchronous on `stream`
    hipError_t e = d_sync(s);
    if (e != hipSuccess) rc = fail(ASCC_E_HIP, std::string("ascc_build_ints: ") + hipGetErrorString(e));
  }
  if (rc) {
    free_all(I->pool);
    if (ws) unregister_buffer(ws);
    delete I;
    return rc;
  }
  *out = I;
  return ASCC_OK;
}

void ascc_ints_free(ascc_ints* I) {
  if (!I) return;
  free_all(I->batch);
  free_all(I->pl);
  free_all(I->pool);
  if (I->pool.base) unregister_buffer(I->pool.base);
  for (auto& m : I->marks) {
    (void)hipEventDestroy(m.second.first);
    (void)hipEventDestroy(m.second.second);
  }
  for (hipEvent_t e : I->event_pool) (void)hipEventDestroy(e);
  delete I;
}

int ascc_residual(ascc_ints* I, const double* t1, const double* t2, double* r1, double* r2, double* e, void* stream) {
  if (!I || !t1 || !t2 || !r1 || !r2 || !e) return fail(ASCC_E_ARG, "NULL argument to ascc_residual");
  ScopedBuffers user;
  user.add(t1, sizeof(double) * I->ov);
  user.add(t2, sizeof(double) * I->oovv);
  user.add(r1, sizeof(double) * I->ov);
  user.add(r2, sizeof(double) * I->oovv);
  user.add(e, sizeof(double));
  return residual_fp64(I, t1, t2, r1, r2, e, static_cast<hipStream_t>(stream));
}

int ascc_batch_workspace_bytes(int no, int nv, int naux, int precision, int vvvv_mode, int max_states, int group,
                               size_t* bytes) {
  int rc = check_shape(no, nv, naux);
  if (rc) return rc;
  if (!bytes || max_states < 1 || max_states > 4096 || group < 1 || group > max_states)
    return fail(ASCC_E_ARG, "need 1 <= group <= max_states <= 4096 and an output pointer");
  if (precision < ASCC_PREC_FP64 || precision > ASCC_PREC_BF16X3) return fail(ASCC_E_ARG, "unsupported precision");
  *bytes = batch_footprint(no, nv, naux, precision, vvvv_mode, max_states, group);
  return ASCC_OK;
}

int ascc_batch_reserve(ascc_ints* I, int max_states) {
  if (!I) return fail(ASCC_E_ARG, "NULL handle");
  if (max_states <= I->max_states && I->group == 1) return ASCC_OK;
  return batch_reserve_impl(I, max_states, 1, nullptr, 0);
}

int ascc_batch_reserve_ws(ascc_ints* I, int max_states, int group, void* d_workspace, size_t ws_bytes) {
  if (!I) return fail(ASCC_E_ARG, "NULL handle");
  return batch_reserve_impl(I, max_states, group, d_workspace, ws_bytes);
}

int ascc_residual_batch(ascc_ints* I, int nstates, const double* const* t1, const double* const* t2,
                        double* const* r1, double* const* r2, double* e, void* stream) {
  if (!I || !t1 || !t2 || !r1 || !r2 || !e) return fail(ASCC_E_ARG, "NULL argument to ascc_residual_batch");
  if (nstates < 1 || nstates > I->max_states)
    return fail(ASCC_E_STATE, "nstates exceeds the capacity reserved with ascc_batch_reserve");
  for (int k = 0; k < nstates; ++k)
    if (!t1[k] || !t2[k] || !r1[k] || !r2[k]) return fail(ASCC_E_ARG, "NULL state pointer");
  hipStream_t s = static_cast<hipStream_t>(stream);
  // the other terms: groups of states as one batched pass when the state arrays are evenly spaced
  // (ascending)
  auto even = [&](const void* const* a, size_t bytes) {
    const long d = nstates > 1 ? (long)((const char*)a[1] - (const char*)a[0]) : 0;
    if (nstates > 1 && d < (long)bytes) return false;
    for (int k = 2; k < nstates; ++k)
      if ((const char*)a[k] - (const char*)a[0] != (long)k * d) return false;
    return true;
  };
  const bool grouped = I->group > 1 && I->pl_hole < 0 && even((const void* const*)t1, 8 * I->ov) &&
                       even((const void* const*)t2, 8 * I->oovv) && even((const void* const*)r1, 8 * I->ov) &&
                       even((const void* const*)r2, 8 * I->oovv);
  ScopedBuffers user;
  if (grouped) {  // each array family as one span (the batched launches cross the states)
    auto span = [&](const void* const* a, size_t bytes) {
      user.add(a[0], (size_t)((const char*)a[nstates - 1] - (const char*)a[0]) + bytes);
    };
    span((const void* const*)t1, sizeof(double) * I->ov);
    span((const void* const*)t2, sizeof(double) * I->oovv);
    span((const void* const*)r1, sizeof(double) * I->ov);
    span((const void* const*)r2, sizeof(double) * I->oovv);
  }
  for (int k = 0; k < nstates; ++k) {
    user.add(t1[k], sizeof(double) * I->ov);
    user.add(t2[k], sizeof(double) * I->oovv);
    user.add(r1[k], sizeof(double) * I->ov);
    user.add(r2[k], sizeof(double) * I->oovv);
  }
  user.add(e, sizeof(double) * nstates);
  std::vector<double*> RLs(nstates);
  for (int k = 0; k < nstates; ++k) RLs[k] = I->RL_all + (long)k * I->oovv;
  int rc = pp_ladder_states(I, nstates, t2, RLs.data(), I->Tp_all, I->Rp_all, I->Tpf_all, s);
  if (rc) return rc;
  if (!grouped) {
    for (int k = 0; k < nstates && !rc; ++k) rc = residual_core(I, t1[k], t2[k], r1[k], r2[k], e + k, RLs[k], s);
    return rc;
  }
  for (int g0 = 0; g0 < nstates && !rc; g0 += I->group)
    rc = residual_group(I, std::min(I->group, nstates - g0), nstates, t1 + g0, t2 + g0, r1 + g0, r2 + g0, e + g0,
                        RLs[g0], s);
  return rc;
}

static int diis_create_impl(const ascc_ints* I, int max_vectors, int start, void* ws, size_t ws_bytes, ascc_diis** out);

int ascc_diis_create(const ascc_ints* I, int max_vectors, int start, ascc_diis** out) {
  return diis_create_impl(I, max_vectors, start, nullptr, 0, out);
}

int ascc_diis_create_ws(const ascc_ints* I, int max_vectors, int start, void* d_workspace, size_t ws_bytes,
                        ascc_diis** out) {
  if (!d_workspace) return fail(ASCC_E_ARG, "d_workspace is NULL");
  return diis_create_impl(I, max_vectors, start, d_workspace, ws_bytes, out);
}

static int diis_create_impl(const ascc_ints* I, int max_vectors, int start, void* ws, size_t ws_bytes, ascc_diis** out) {
  if (!I || !out) return fail(ASCC_E_ARG, "NULL argument to ascc_diis_create");
  *out = nullptr;
  if (max_vectors < 1 || max_vectors > kMaxDiis) return fail(ASCC_E_ARG, "max_vectors must be in 1..16");
  if (start < 0) return fail(ASCC_E_ARG, "start must be >= 0");
  ascc_diis* D = new ascc_diis();
  D->no = I->no;
  D->nv = I->nv;
  D->m = max_vectors;
  D->start = start;
  D->calls = 0;
  D->len = I->ov + I->oovv;
  if (ws) {
    if ((reinterpret_cast<uintptr_t>(ws) & (kAlign - 1)) != 0) {
      delete D;
      return fail(ASCC_E_ARG, "d_workspace must be 256-byte aligned");
    }
    D->pool.base = static_cast<char*>(ws);
    D->pool.size = ws_bytes;
  }
  int rc = dalloc(D->pool, &D->hist_t, (size_t)D->m * D->len);
  if (!rc) rc = dalloc(D->pool, &D->hist_e, (size_t)D->m * D->len);
  if (!rc) rc = dalloc(D->pool, &D->partial, (size_t)update_partial_blocks() * (3 + kMaxDiis));
  if (!rc) rc = dalloc(D->pool, &D->st, 1);
  if (!rc) rc = ascc_diis_reset(D, nullptr);
  if (!rc) {
    hipError_t e = d_sync(nullptr);
    if (e != hipSuccess) rc = fail(ASCC_E_HIP, std::string("ascc_diis_create: ") + hipGetErrorString(e));
  }
  if (rc) {
    free_all(D->pool);
    delete D;
    return rc;
  }
  *out = D;
  return ASCC_OK;
}

int ascc_diis_reset(ascc_diis* D, void* stream) {
  if (!D) return fail(ASCC_E_ARG, "NULL diis");
  DiisState h;
  std::memset(&h, 0, sizeof(h));
  for (int k = 0; k < kMaxDiis; ++k) h.slot_age[k] = -1;
  // Kept in a static per-call host copy until the async copy has read it: use a blocking copy.
  HIPCHK(d_copy(D->st, &h, sizeof(h), hipMemcpyHostToDevice, static_cast<hipStream_t>(stream)));
  HIPCHK(d_sync(static_cast<hipStream_t>(stream)));
  D->calls = 0;
  return ASCC_OK;
}

void ascc_diis_free(ascc_diis* D) {
  if (!D) return;
  free_all(D->pool);
  delete D;
}

int ascc_update(ascc_ints* I, ascc_diis* D, double* t1, double* t2, const double* r1, const double* r2,
                const double* e, double level_shift, double* stats, void* stream) {
  if (!I || !D || !t1 || !t2 || !r1 || !r2 || !e || !stats) return fail(ASCC_E_ARG, "NULL argument to ascc_update");
  if (D->no != I->no || D->nv != I->nv) return fail(ASCC_E_STATE, "DIIS state and integrals differ in shape");
  if (!(level_shift >= 0.0)) return fail(ASCC_E_ARG, "level_shift must be >= 0");
  ScopedBuffers user;
  user.add(t1, sizeof(double) * I->ov);
  user.add(t2, sizeof(double) * I->oovv);
  user.add(r1, sizeof(double) * I->ov);
  user.add(r2, sizeof(double) * I->oovv);
  user.add(e, sizeof(double));
  user.add(stats, 8 * sizeof(double));
  UpdateArgs u;
  u.t1 = t1;
  u.t2 = t2;
  u.r1 = r1;
  u.r2 = r2;
  u.e = e;
  u.eps = I->eps;
  u.hist_t = D->hist_t;
  u.hist_e = D->hist_e;
  u.partial = D->partial;
  u.st = D->st;
  u.stats = stats;
  u.no = I->no;
  u.nv = I->nv;
  u.m = D->m;
  u.start = D->start;
  u.len = D->len;
  u.shift = level_shift;
  phase_begin(I, PH_UPDATE, static_cast<hipStream_t>(stream));
  HIPCHK(diis_update(u, static_cast<hipStream_t>(stream)));
  phase_end(I, static_cast<hipStream_t>(stream));
  D->calls += 1;
  return ASCC_OK;
}

}  // extern "C"

namespace ascc {

uintptr_t dry_run_address(size_t bytes) { return fake_alloc(bytes); }

int iterate_slots(ascc_ints* I, ascc_diis* D, int n, const int* dtab, const int* htab, const char* region,
                  long stride, double* t1, double* t2, double* r1, double* r2, double* e, double* stats,
                  hipStream_t s) {
  if (!I || !D || n < 1 || !htab || !region || stride <= 0 || !t1 || !t2 || !r1 || !r2 || !e || !stats)
    return fail(ASCC_E_ARG, "invalid slot batch");
  if (D->no != I->no || D->nv != I->nv) return fail(ASCC_E_STATE, "DIIS state and integrals differ in shape");
  SlotBatch sb;
  sb.n = n;
  sb.dtab = dtab;
  sb.htab = htab;
  for (int z = 0; z < n; ++z) {
    if (htab[z] < 0) return fail(ASCC_E_ARG, "slot table entries are offsets from the base slot (>= 0)");
    sb.tab_max = std::max(sb.tab_max, htab[z]);
  }
  const uintptr_t lo = reinterpret_cast<uintptr_t>(region);
  sb.ranges.push_back({lo, lo + (uintptr_t)stride, stride});
  int rc;
  {
    SlotBatchScope scope(&sb);
    rc = residual_core(I, t1, t2, r1, r2, e, nullptr, s);
  }
  if (rc) return rc;
  UpdateArgs u;
  u.t1 = t1;
  u.t2 = t2;
  u.r1 = r1;
  u.r2 = r2;
  u.e = e;
  u.eps = I->eps;
  u.hist_t = D->hist_t;
  u.hist_e = D->hist_e;
  u.partial = D->partial;
  u.st = D->st;
  u.stats = stats;
  u.no = I->no;
  u.nv = I->nv;
  u.m = D->m;
  u.start = D->start;
  u.len = D->len;
  u.shift = 0.0;
  u.nslot = n;
  u.ss = stride;
  u.tab = dtab;
  u.tab_max = sb.tab_max;
  phase_begin(I, PH_UPDATE, s);
  {
    g_enclosing_ok = true;
    const hipError_t e2 = diis_update(u, s);
    g_enclosing_ok = false;
    HIPCHK(e2);
  }
  phase_end(I, s);
  return ASCC_OK;
}

// Device bytes of the solver state that solve_impl carves from a workspace: the DIIS state, then
// r1, r2, e, the statistics block and the trial amplitudes t1s, t2s.
size_t solve_workspace_bytes(long o, long v, int diis_size) {
  const long ov = o * v, oovv = o * o * v * v;
  size_t off = diis_footprint(o, v, diis_size);
  for (long n : {ov, oovv, 1L, 8L, ov, oovv}) off = align_up(off) + sizeof(double) * (size_t)n;
  return align_up(off);
}

// The solve loop of ascc_solve.  ws == nullptr: the DIIS state and work arrays are allocated here and
// the statistics are read through pinned host memory; otherwise everything is carved from
// [ws, ws + ws_bytes) (>= solve_workspace_bytes) and no allocation is made.
int solve_impl(ascc_ints* I, const ascc_opts* opts, double* t1, double* t2, ascc_result* res, void* stream,
               char* ws, size_t ws_bytes) {
  if (!I || !opts || !t1 || !t2 || !res) return fail(ASCC_E_ARG, "NULL argument to ascc_solve");
  if (opts->maxiter < 1) return fail(ASCC_E_ARG, "maxiter must be >= 1");
  if (opts->diis_size < 1 || opts->diis_size > kMaxDiis) return fail(ASCC_E_ARG, "diis_size must be in 1..16");
  hipStream_t s = static_cast<hipStream_t>(stream);
  std::memset(res, 0, sizeof(*res));
  const int prec0 = I->cur_prec;
  bool lowp_phase = (prec0 != ASCC_PREC_FP64);
  size_t dbytes = 0;
  if (ws) {
    dbytes = diis_footprint(I->no, I->nv, opts->diis_size);
    if (ws_bytes < solve_workspace_bytes(I->no, I->nv, opts->diis_size))
      return fail(ASCC_E_NOMEM, "solver workspace too small");
  }
  ascc_diis* D = nullptr;
  int rc = diis_create_impl(I, opts->diis_size, opts->diis_start, ws, dbytes, &D);
  if (rc) return rc;
  Pool work;
  if (ws) {
    work.base = ws + dbytes;
    work.size = ws_bytes - dbytes;
  }
  double *r1 = nullptr, *r2 = nullptr, *e = nullptr, *stats = nullptr, *t1s = nullptr, *t2s = nullptr;
  rc = dalloc(work, &r1, I->ov);
  if (!rc) rc = dalloc(work, &r2, I->oovv);
  if (!rc) rc = dalloc(work, &e, 1);
  if (!rc) rc = dalloc(work, &stats, 8);
  if (!rc) rc = dalloc(work, &t1s, I->ov);
  if (!rc) rc = dalloc(work, &t2s, I->oovv);
  double* hstats = nullptr;
  static double dry_stats[8];
  double local_stats[8];
  if (dry_run()) {
    hstats = dry_stats;  // a dry run reports zeros: converged after one iteration
  } else if (ws) {
    hstats = local_stats;  // pageable: the copy completes before the stream synchronisation returns
  } else if (!rc && hipHostMalloc((void**)&hstats, 8 * sizeof(double), 0) != hipSuccess) {
    rc = fail(ASCC_E_NOMEM, "pinned host allocation failed");
  }
  ScopedBuffers user;
  user.add(t1, sizeof(double) * I->ov);
  user.add(t2, sizeof(double) * I->oovv);
  int status = ASCC_E_NOT_CONVERGED;
  int lowp_iters = 0;
  LowpStall stall;
  bool confirm = false;  // the next evaluation is the first FP64 one after a hand-over
  double handover_de = 0.0;
  for (int it = 0; !rc && it < opts->maxiter; ++it) {
    rc = residual_fp64(I, t1, t2, r1, r2, e, s);
    if (rc) break;
    // statistics of the residual at the current amplitudes, without changing them: run the
    // update on a copy (the copy also carries the DIIS bookkeeping of this iteration)
    if (d_copy(t1s, t1, sizeof(double) * I->ov, hipMemcpyDeviceToDevice, s) != hipSuccess ||
        d_copy(t2s, t2, sizeof(double) * I->oovv, hipMemcpyDeviceToDevice, s) != hipSuccess) {
      rc = fail(ASCC_E_HIP, "copy of amplitudes failed");
      break;
    }
    rc = ascc_update(I, D, t1s, t2s, r1, r2, e, opts->level_shift, stats, stream);
    if (rc) break;
    if (d_copy(hstats, stats, 8 * sizeof(double), hipMemcpyDeviceToHost, s) != hipSuccess || d_sync(s) != hipSuccess) {
      rc = fail(ASCC_E_HIP, "reading iteration statistics failed");
      break;
    }
    res->e_corr = hstats[0];
    res->de = hstats[1];
    res->rmax = hstats[2];
    res->rnorm = hstats[3];
    res->iterations = it + 1;
    if (((int)hstats[5]) & 1) {
      status = fail(ASCC_E_NONFINITE, "non-finite residual or energy at iteration " + std::to_string(it));
      break;
    }
    // the first FP64 evaluation after the hand-over is at the amplitudes of the last low-precision
    // iteration: its energy change is that iteration's
    if (confirm) res->de = handover_de;
    const bool ok = (opts->tol_rnorm <= 0 || res->rnorm <= opts->tol_rnorm) &&
                    (opts->tol_rmax <= 0 || res->rmax <= opts->tol_rmax) &&
                    (opts->tol_de <= 0 || std::fabs(res->de) < opts->tol_de);
    if (lowp_phase) {
      // low-precision bulk: hand over to FP64 (which decides convergence) once the statistics
      // already pass the convergence test, the residual is small enough, it stops improving (its
      // rounding floor), or the low-precision budget is spent
      ++lowp_iters;
      res->lowp_iterations = lowp_iters;
      const bool done = ok || (opts->lowp_rnorm > 0 && hstats[3] <= opts->lowp_rnorm) ||
                        (opts->lowp_maxiter > 0 && lowp_iters >= opts->lowp_maxiter) || stall.stalled(hstats[3]);
      if (done) {
        lowp_phase = false;
        I->cur_prec = ASCC_PREC_FP64;
        confirm = true;
        handover_de = hstats[1];
        continue;  // re-evaluate the same amplitudes in FP64
      }
    } else {
      if (ok) {
        res->converged = 1;
        status = ASCC_OK;
        break;
      }
      if (confirm) {
        // not converged in FP64 yet: the DIIS history restarts from this FP64 residual (the
        // low-precision pairs carry the rounding of those contractions), and the update is redone
        confirm = false;
        if ((rc = ascc_diis_reset(D, stream))) break;
        if (d_copy(t1s, t1, sizeof(double) * I->ov, hipMemcpyDeviceToDevice, s) != hipSuccess ||
            d_copy(t2s, t2, sizeof(double) * I->oovv, hipMemcpyDeviceToDevice, s) != hipSuccess) {
          rc = fail(ASCC_E_HIP, "copy of amplitudes failed");
          break;
        }
        if ((rc = ascc_update(I, D, t1s, t2s, r1, r2, e, opts->level_shift, stats, stream))) break;
      }
    }
    // accept the update, except after the last evaluation: a solve that ends unconverged returns the
    // amplitudes its reported energy and residual norms were evaluated at
    if (it + 1 == opts->maxiter) break;
    if (d_copy(t1, t1s, sizeof(double) * I->ov, hipMemcpyDeviceToDevice, s) != hipSuccess ||
        d_copy(t2, t2s, sizeof(double) * I->oovv, hipMemcpyDeviceToDevice, s) != hipSuccess) {
      rc = fail(ASCC_E_HIP, "copy of amplitudes failed");
      break;
    }
  }
  I->cur_prec = prec0;
  (void)d_sync(s);
  if (hstats && !dry_run() && !ws) (void)hipHostFree(hstats);
  free_all(work);
  ascc_diis_free(D);
  if (rc) return rc;
  if (status == ASCC_E_NOT_CONVERGED) {
    // near convergence: the energy no longer moves at the energy test's precision and every
    // residual test is missed by less than a factor 10
    const double tde = opts->tol_de > 0 ? opts->tol_de : 1e-7;
    res->stalled = res->iterations > 1 && std::fabs(res->de) < tde &&
                   (opts->tol_rnorm <= 0 || res->rnorm <= 10.0 * opts->tol_rnorm) &&
                   (opts->tol_rmax <= 0 || res->rmax <= 10.0 * opts->tol_rmax);
    set_error(res->stalled ? "stalled near convergence in maxiter iterations" : "not converged in maxiter iterations");
  }
  return status;
}

}  // namespace ascc

extern "C" {

int ascc_solve(ascc_ints* I, const ascc_opts* opts, double* t1, double* t2, ascc_result* res, void* stream) {
  return solve_impl(I, opts, t1, t2, res, stream, nullptr, 0);
}

int ascc_two_ansatz(const double* d_B, const double* d_fock, int fock_is_diag, int no, int nv, int naux, int precision,
                    int vvvv_mode, int hole, int particle, double alpha, const ascc_opts* opts, double* const* d_t1,
                    double* const* d_t2, ascc_two_ansatz_result* res, void* stream) {
  if (!opts || !d_t1 || !d_t2 || !res || !d_t1[0] || !d_t1[1] || !d_t2[0] || !d_t2[1])
    return fail(ASCC_E_ARG, "NULL argument to ascc_two_ansatz");
  if (!(std::fabs(alpha) < 1.0)) return fail(ASCC_E_ARG, "|alpha| must be below 1");
  std::memset(res, 0, sizeof(*res));
  res->beta[0] = 1.0 / (1.0 + alpha);  // (1 - beta)/beta = alpha
  res->beta[1] = 1.0 / (1.0 - alpha);  // hole sign flipped: (1 - beta)/beta = -alpha
  int status = ASCC_OK;
  for (int k = 0; k < 2; ++k) {
    const int sign = k == 0 ? 1 : -1;
    const double beta = res->beta[k];
    ascc_ints* I = nullptr;
    int rc = ascc_build_ints_hbar(d_B, d_fock, fock_is_diag, no, nv, naux, precision, vvvv_mode, hole, particle, sign,
                                  stream, &I);
    if (rc) return rc;
    rc = ascc_initial_guess(d_t1[k], d_t2[k], no, nv, hole, particle, sign * beta, -0.5 * beta * beta, stream);
    if (!rc) rc = ascc_solve(I, opts, d_t1[k], d_t2[k], &res->solve[k], stream);
    // a solve that ends without converging, or whose iteration diverged to non-finite values, is a
    // failed ansatz: recorded (converged = 0) and the other one still runs
    const bool failed_solve = rc == ASCC_E_NOT_CONVERGED || rc == ASCC_E_NONFINITE;
    double e0 = 0.0;
    if (!rc || failed_solve) {
      const int rc0 = ascc_reference_energy(I, &e0, stream);
      if (rc0) rc = rc0;
    }
    ascc_ints_free(I);
    if (failed_solve) {
      status = rc;
    } else if (rc) {
      return rc;
    }
    res->e_total[k] = e0 + res->solve[k].e_corr;
  }
  // the paper's rule for a state: the mean of the two solutions, the single converged one when the
  // other fails, and no energy when neither converges
  auto counts = [](const ascc_result& r) { return r.converged || r.stalled; };
  res->used = (counts(res->solve[0]) ? 1 : 0) | (counts(res->solve[1]) ? 2 : 0);
  if (res->used == 3 || res->used == 0)
    res->e_mean = 0.5 * (res->e_total[0] + res->e_total[1]);
  else
    res->e_mean = res->e_total[res->used == 1 ? 0 : 1];
  (void)status;
  if (res->used == 0) {
    set_error("neither two-ansatz solve converged (or stalled near convergence) in maxiter iterations" +
              std::string(status == ASCC_E_NONFINITE ? " (an iteration became non-finite)" : ""));
    return ASCC_E_NOT_CONVERGED;
  }
  return ASCC_OK;
}

}  // extern "C"
