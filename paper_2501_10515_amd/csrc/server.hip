// Request loop for many independent solves on one GPU (continuous batching at the iteration
// level).
//
// * Admission by HBM footprint: the server owns one device slab (allocated once) and carves from
//   it, in arrival order, the working set of each admitted request -- integral set, DIIS state,
//   amplitudes, residuals, staging for its DF tensor (and PLASCC buffers) -- with a first-fit free
//   list.  No device allocation happens while requests run.
// * Size buckets: ground-state requests of one shape (no, nv, naux) share a bucket, a slab region
//   of up to kMaxSlots equal slots (as many as a quarter of the budget holds) in which every slot
//   repeats one layout at a fixed stride.  The running slots of a bucket advance together: one
//   iteration of all of them is one batched pass (iterate_slots: every contraction one launch over
//   the slots, the update and DIIS one launch set), for the slots in low precision and for those
//   in FP64, each captured once per slot set into a hipGraph and replayed.  Excited-state and PLASCC
//   requests have buckets of one slot.  Each bucket has its own stream, so buckets overlap on the
//   device; requests join and leave their bucket between iterations as slab space and slots free.
// * The convergence test reads each slot's 8-double statistics row from one pinned copy of the
//   bucket's statistics block behind each iteration (polled with an event, never a blocking
//   wait).  A low-precision request runs its bulk iterations in that precision and finishes in
//   FP64 (the FP64 refinement of ascc_solve).
#include <algorithm>
#include <cmath>
#include <cstring>
#include <deque>
#include <map>
#include <string>
#include <vector>

#include "../../include/ascc.h"
#include "internal.h"

using namespace ascc;

namespace {

constexpr size_t kSlabAlign = 256;
constexpr int kMaxSlots = 8;  // slots per bucket

struct Request {
  int id = 0, o = 0, v = 0, Q = 0;
  std::vector<double> hB, heps;  // host copies until the first iteration has run
  double t_submit = 0, t_admit = -1, t_done = -1;
  int status = 1;  // 1 queued, 2 running, 0 converged, <0 ASCC_E_*
  size_t bytes = 0;  // the slot's footprint
  size_t ints_bytes = 0, diis_bytes = 0, plascc_bytes = 0;
  ascc_ints* ints = nullptr;
  ascc_diis* diis = nullptr;
  double *t1 = nullptr, *t2 = nullptr, *r1 = nullptr, *r2 = nullptr, *e = nullptr;
  double *dB = nullptr, *deps = nullptr;
  bool lowp_phase = false;
  LowpStall stall;
  int iterations = 0, lowp_iterations = 0;
  double e_corr = 0, rnorm = 0, rmax = 0, de = 0;
  int hole = -1, particle = -1, s_sign = 1;  // a 1-CSF state (hole >= 0) or the ground state
  double beta = 1.0, e_ref = 0.0;
  bool plascc = false;
  int bucket = -1, slot = -1;
  int last_bucket = -1, last_slot = -1;  // reported by ascc_server_info
};

// A slab region of equal slots for requests of one shape; slot k's working set starts at
// region + header + k * stride and is carved in the same order in every slot.
struct Bucket {
  int o = 0, v = 0, Q = 0;
  bool shared = false;  // ground-state bucket that later requests of this shape join
  int cap = 1;
  size_t stride = 0, header = 0, off = 0, bytes = 0;
  char* region = nullptr;
  double* dstats = nullptr;  // [cap][8] statistics rows, device
  int* dtab = nullptr;       // [2][cap] slot tables (low precision, FP64), device
  double* hstats = nullptr;  // pinned copy of dstats
  int* htab = nullptr;       // pinned [2][cap]
  std::vector<int> slot_req;  // request id per slot, -1 free
  hipStream_t stream = nullptr;
  hipEvent_t ev = nullptr;
  bool inflight = false;
  std::vector<int> launched;  // slots of the in-flight iteration
  std::map<std::pair<int, unsigned>, hipGraphExec_t> graphs;  // (phase, slot mask)
  char* slot_base(int k) const { return region + header + (size_t)k * stride; }
  int used() const {
    int n = 0;
    for (int r : slot_req) n += (r >= 0);
    return n;
  }
};

}  // namespace

struct ascc_server {
  ascc_server_opts opts{};
  char* slab = nullptr;
  size_t slab_bytes = 0;
  std::map<size_t, size_t> free_list;  // offset -> length
  std::vector<Request*> reqs;
  std::deque<int> queue;
  int running = 0;
  std::map<int, Bucket*> buckets;
  int next_bucket = 0;
  std::vector<hipStream_t> stream_pool;
  std::vector<hipEvent_t> event_pool;
  int n_done = 0;
};

namespace {

int sfail(int code, const std::string& msg) {
  set_error(msg);
  return code;
}

bool slab_take(ascc_server* S, size_t bytes, size_t* off) {
  bytes = (bytes + kSlabAlign - 1) / kSlabAlign * kSlabAlign;
  for (auto it = S->free_list.begin(); it != S->free_list.end(); ++it) {
    if (it->second >= bytes) {
      *off = it->first;
      const size_t rest = it->second - bytes;
      const size_t roff = it->first + bytes;
      S->free_list.erase(it);
      if (rest) S->free_list[roff] = rest;
      return true;
    }
  }
  return false;
}

void slab_give(ascc_server* S, size_t off, size_t bytes) {
  bytes = (bytes + kSlabAlign - 1) / kSlabAlign * kSlabAlign;
  auto it = S->free_list.emplace(off, bytes).first;
  auto next = std::next(it);
  if (next != S->free_list.end() && it->first + it->second == next->first) {
    it->second += next->second;
    S->free_list.erase(next);
  }
  if (it != S->free_list.begin()) {
    auto prev = std::prev(it);
    if (prev->first + prev->second == it->first) {
      prev->second += it->second;
      S->free_list.erase(it);
    }
  }
}

size_t align_s(size_t x) { return (x + kSlabAlign - 1) / kSlabAlign * kSlabAlign; }

// Layout of a request's slot: [ints | diis | t1 t2 r1 r2 e | eps | B staging | PLASCC buffers]
// (the last only for a PLASCC request): its whole device working set.
size_t request_bytes(const ascc_server* S, int o, int v, int Q, bool plascc, size_t* ib, size_t* db,
                     size_t* pb) {
  size_t ints_b = 0, diis_b = 0, pl_b = 0;
  if (ascc_workspace_bytes(o, v, Q, S->opts.precision, S->opts.vvvv_mode, S->opts.solve.diis_size, &ints_b, &diis_b))
    return 0;
  if (plascc && ascc_plascc_workspace_bytes(o, v, Q, &pl_b)) return 0;
  *ib = ints_b;
  *db = diis_b;
  *pb = pl_b;
  const size_t ov = (size_t)o * v, oovv = (size_t)o * o * v * v, n = (size_t)o + v;
  size_t b = align_s(ints_b) + align_s(diis_b);
  b += align_s(8 * ov) * 2 + align_s(8 * oovv) * 2 + align_s(8) + align_s(8 * n);
  b += align_s(8 * (size_t)Q * n * n);
  b += align_s(pl_b);
  return b;
}

size_t bucket_header(int cap) { return align_s(64 * (size_t)cap) + align_s(2 * sizeof(int) * (size_t)cap); }

void drop_graphs(Bucket* B) {
  for (auto& g : B->graphs) (void)hipGraphExecDestroy(g.second);
  B->graphs.clear();
}

void release_bucket(ascc_server* S, int bid) {
  Bucket* B = S->buckets[bid];
  drop_graphs(B);
  slab_give(S, B->off, B->bytes);
  if (B->stream) S->stream_pool.push_back(B->stream);
  if (B->ev) S->event_pool.push_back(B->ev);
  if (B->hstats) (void)hipHostFree(B->hstats);
  if (B->htab) (void)hipHostFree(B->htab);
  delete B;
  S->buckets.erase(bid);
}

// Frees a request's slot (its handles are host structs over slab memory).
void release_request(ascc_server* S, Request* R) {
  if (R->diis) ascc_diis_free(R->diis);
  if (R->ints) ascc_ints_free(R->ints);
  R->diis = nullptr;
  R->ints = nullptr;
  if (R->bucket >= 0) {
    Bucket* B = S->buckets[R->bucket];
    B->slot_req[R->slot] = -1;
    if (B->used() == 0 && !B->inflight) release_bucket(S, R->bucket);
  }
  R->bucket = R->slot = -1;
}

int open_bucket(ascc_server* S, const Request* R, size_t slot_bytes, int* bid) {
  const bool shared = R->hole < 0 && !R->plascc;
  int cap = 1;
  if (shared) {
    const size_t fit = S->slab_bytes / 4 / std::max<size_t>(slot_bytes, 1);
    cap = (int)std::min<size_t>(std::max<size_t>(fit, 1), std::min(kMaxSlots, S->opts.max_active));
  }
  size_t off = 0;
  while (!slab_take(S, bucket_header(cap) + (size_t)cap * slot_bytes, &off)) {
    if (cap == 1) return ASCC_E_NOMEM;  // not now: the head of the queue waits
    cap = 1;
  }
  Bucket* B = new Bucket();
  B->o = R->o;
  B->v = R->v;
  B->Q = R->Q;
  B->shared = shared;
  B->cap = cap;
  B->stride = slot_bytes;
  B->header = bucket_header(cap);
  B->off = off;
  B->bytes = B->header + (size_t)cap * slot_bytes;
  B->region = S->slab + off;
  B->dstats = reinterpret_cast<double*>(B->region);
  B->dtab = reinterpret_cast<int*>(B->region + align_s(64 * (size_t)cap));
  B->slot_req.assign(cap, -1);
  int rc = ASCC_OK;
  if (!S->stream_pool.empty()) {
    B->stream = S->stream_pool.back();
    S->stream_pool.pop_back();
  } else if (hipStreamCreateWithFlags(&B->stream, hipStreamNonBlocking) != hipSuccess) {
    rc = sfail(ASCC_E_HIP, "hipStreamCreate failed");
  }
  if (!rc) {
    if (!S->event_pool.empty()) {
      B->ev = S->event_pool.back();
      S->event_pool.pop_back();
    } else if (hipEventCreateWithFlags(&B->ev, hipEventDisableTiming) != hipSuccess) {
      rc = sfail(ASCC_E_HIP, "hipEventCreate failed");
    }
  }
  if (!rc && (hipHostMalloc((void**)&B->hstats, 64 * (size_t)cap, 0) != hipSuccess ||
              hipHostMalloc((void**)&B->htab, 2 * sizeof(int) * (size_t)cap, 0) != hipSuccess))
    rc = sfail(ASCC_E_NOMEM, "pinned host allocation failed");
  *bid = S->next_bucket++;
  S->buckets[*bid] = B;
  if (rc) {
    release_bucket(S, *bid);
    return rc;
  }
  return ASCC_OK;
}

// Carve the request's slot, upload its inputs and build its integral set, DIIS state and starting
// amplitudes on the bucket's stream.
int admit(ascc_server* S, Request* R, double now) {
  Bucket* B = S->buckets[R->bucket];
  const size_t ov = (size_t)R->o * R->v, oovv = (size_t)R->o * R->o * R->v * R->v, n = (size_t)R->o + R->v;
  char* base = B->slot_base(R->slot);
  size_t p = 0;
  char* ints_ws = base + p;
  p += align_s(R->ints_bytes);
  char* diis_ws = base + p;
  p += align_s(R->diis_bytes);
  auto carve = [&](size_t bytes) {
    double* q = reinterpret_cast<double*>(base + p);
    p += align_s(bytes);
    return q;
  };
  R->t1 = carve(8 * ov);
  R->t2 = carve(8 * oovv);
  R->r1 = carve(8 * ov);
  R->r2 = carve(8 * oovv);
  R->e = carve(8);
  R->deps = carve(8 * n);
  R->dB = carve(8 * (size_t)R->Q * n * n);
  char* plascc_ws = base + p;  // R->plascc_bytes (0 unless a PLASCC request)
  p += align_s(R->plascc_bytes);
  hipStream_t s = B->stream;
  if (hipMemcpyAsync(R->dB, R->hB.data(), 8 * R->hB.size(), hipMemcpyHostToDevice, s) != hipSuccess ||
      hipMemcpyAsync(R->deps, R->heps.data(), 8 * n, hipMemcpyHostToDevice, s) != hipSuccess)
    return sfail(ASCC_E_HIP, "upload of request inputs failed");
  int rc = R->hole < 0 ? ascc_build_ints_ws(R->dB, R->deps, 1, R->o, R->v, R->Q, S->opts.precision,
                                            S->opts.vvvv_mode, ints_ws, R->ints_bytes, s, &R->ints)
                       : ascc_build_ints_hbar_ws(R->dB, R->deps, 1, R->o, R->v, R->Q, S->opts.precision,
                                                 S->opts.vvvv_mode, R->hole, R->particle, R->s_sign, ints_ws,
                                                 R->ints_bytes, s, &R->ints);
  if (rc) return rc;
  rc = ascc_diis_create_ws(R->ints, S->opts.solve.diis_size, S->opts.solve.diis_start, diis_ws, R->diis_bytes,
                           &R->diis);
  if (rc) return rc;
  if (R->plascc && (rc = ascc_set_plascc_ws(R->ints, R->hole, R->particle, plascc_ws, R->plascc_bytes, s)))
    return rc;
  if (R->hole >= 0) {  // T^P(0) of the state
    if ((rc = ascc_initial_guess(R->t1, R->t2, R->o, R->v, R->hole, R->particle, R->s_sign * R->beta,
                                 -0.5 * R->beta * R->beta, s)))
      return rc;
  } else {
    int d1[4] = {(int)ov, 1, 1, 1}, d2[4] = {(int)oovv, 1, 1, 1};
    if (permute4(R->t1, d1, 0.0, nullptr, 0, s) != hipSuccess || permute4(R->t2, d2, 0.0, nullptr, 0, s) != hipSuccess)
      return sfail(ASCC_E_HIP, "amplitude initialisation failed");
  }
  R->lowp_phase = (S->opts.precision != ASCC_PREC_FP64);
  (void)ascc_set_precision(R->ints, R->lowp_phase ? S->opts.precision : ASCC_PREC_FP64);
  R->t_admit = now;
  R->status = 2;
  return ASCC_OK;
}

// One batched iteration of the slots `slots` (ascending) of a bucket, all in phase `phase`
// (0 low precision, 1 FP64): the slot table goes to the device, then the captured graph of this slot
// set is replayed (captured on first use) or the pass is issued directly.
int launch_group(ascc_server* S, Bucket* B, int phase, const std::vector<int>& slots) {
  const int n = (int)slots.size(), base = slots[0];
  int* ht = B->htab + phase * B->cap;
  int* dt = B->dtab + phase * B->cap;
  unsigned mask = 0;
  for (int z = 0; z < n; ++z) {
    ht[z] = slots[z] - base;
    mask |= 1u << slots[z];
  }
  Request* R0 = S->reqs[B->slot_req[base]];
  hipStream_t s = B->stream;
  if (hipMemcpyAsync(dt, ht, sizeof(int) * n, hipMemcpyHostToDevice, s) != hipSuccess)
    return sfail(ASCC_E_HIP, "slot table upload failed");
  const int prec = phase == 0 ? S->opts.precision : ASCC_PREC_FP64;
  int rc = ascc_set_precision(R0->ints, prec);
  if (rc) return rc;
  auto pass = [&]() {
    return iterate_slots(R0->ints, R0->diis, n, dt, ht, B->slot_base(base), (long)B->stride, R0->t1, R0->t2, R0->r1,
                         R0->r2, R0->e, B->dstats + 8 * base, s);
  };
  if (!S->opts.use_graphs) return pass();
  // A graph holds the launches of one slot set; it stays valid when the requests in those slots
  // change, since every slot keeps its addresses and the launch sequence depends only on the shape,
  // the precision and the options.
  auto key = std::make_pair(phase, mask);
  auto it = B->graphs.find(key);
  if (it == B->graphs.end()) {
    if (B->graphs.size() >= 64) drop_graphs(B);
    hipGraph_t g = nullptr;
    if (hipStreamBeginCapture(s, hipStreamCaptureModeThreadLocal) != hipSuccess)
      return sfail(ASCC_E_HIP, "hipStreamBeginCapture failed");
    rc = pass();
    hipError_t e = hipStreamEndCapture(s, &g);
    if (rc) {
      if (g) (void)hipGraphDestroy(g);
      return rc;
    }
    if (e != hipSuccess) return sfail(ASCC_E_HIP, std::string("hipStreamEndCapture: ") + hipGetErrorString(e));
    hipGraphExec_t x = nullptr;
    e = hipGraphInstantiate(&x, g, nullptr, nullptr, 0);
    (void)hipGraphDestroy(g);
    if (e != hipSuccess) return sfail(ASCC_E_HIP, std::string("hipGraphInstantiate: ") + hipGetErrorString(e));
    it = B->graphs.emplace(key, x).first;
  }
  if (hipGraphLaunch(it->second, s) != hipSuccess) return sfail(ASCC_E_HIP, "hipGraphLaunch failed");
  return ASCC_OK;
}

// Launch the next iteration of every running slot of an idle bucket.
int launch_bucket(ascc_server* S, Bucket* B) {
  std::vector<int> groups[2];
  for (int k = 0; k < B->cap; ++k) {
    const int id = B->slot_req[k];
    if (id < 0 || S->reqs[id]->status != 2) continue;
    groups[S->reqs[id]->lowp_phase ? 0 : 1].push_back(k);
  }
  B->launched.clear();
  for (int ph = 0; ph < 2; ++ph) {
    if (groups[ph].empty()) continue;
    const int rc = launch_group(S, B, ph, groups[ph]);
    if (rc) return rc;
    B->launched.insert(B->launched.end(), groups[ph].begin(), groups[ph].end());
  }
  if (B->launched.empty()) return ASCC_OK;
  if (hipMemcpyAsync(B->hstats, B->dstats, 64 * (size_t)B->cap, hipMemcpyDeviceToHost, B->stream) != hipSuccess ||
      hipEventRecord(B->ev, B->stream) != hipSuccess)
    return sfail(ASCC_E_HIP, "statistics copy failed");
  B->inflight = true;
  return ASCC_OK;
}

// Consume a finished iteration's statistics; returns true if the request is finished.
bool consume(ascc_server* S, Request* R, const double* st, hipStream_t s, double now) {
  const ascc_opts& o = S->opts.solve;
  if (R->iterations == 0) {  // the uploads ran before this iteration on the same stream
    std::vector<double>().swap(R->hB);
    std::vector<double>().swap(R->heps);
  }
  R->iterations += 1;
  R->e_corr = st[0];
  R->de = st[1];
  R->rmax = st[2];
  R->rnorm = st[3];
  if (((int)st[5]) & 1) {
    R->status = ASCC_E_NONFINITE;
    R->t_done = now;
    return true;
  }
  const bool ok = (o.tol_rnorm <= 0 || st[3] <= o.tol_rnorm) && (o.tol_rmax <= 0 || st[2] <= o.tol_rmax) &&
                  (o.tol_de <= 0 || std::fabs(st[1]) < o.tol_de);
  if (R->lowp_phase) {
    R->lowp_iterations += 1;
    // hand over when the low-precision statistics already pass the convergence test (FP64 then
    // confirms it), or on the residual / budget / rounding-floor rules
    const bool done = ok || (o.lowp_rnorm > 0 && st[3] <= o.lowp_rnorm) ||
                      (o.lowp_maxiter > 0 && R->lowp_iterations >= o.lowp_maxiter) || R->stall.stalled(st[3]);
    if (done) {
      R->lowp_phase = false;
      (void)ascc_set_precision(R->ints, ASCC_PREC_FP64);
      (void)ascc_diis_reset(R->diis, s);
    }
  } else if (ok) {
    R->status = ASCC_OK;
    R->t_done = now;
    (void)ascc_reference_energy(R->ints, &R->e_ref, s);  // the stream is idle: no wait
    return true;
  }
  if (R->iterations >= o.maxiter) {
    R->status = ASCC_E_NOT_CONVERGED;
    R->t_done = now;
    (void)ascc_reference_energy(R->ints, &R->e_ref, s);
    return true;
  }
  return false;
}

}  // namespace

extern "C" {

int ascc_server_create(const ascc_server_opts* opts, ascc_server** out) {
  if (!opts || !out) return sfail(ASCC_E_ARG, "NULL argument to ascc_server_create");
  *out = nullptr;
  if (opts->hbm_budget < (1u << 20) || opts->max_active < 1 || opts->solve.maxiter < 1 ||
      opts->solve.diis_size < 1 || opts->solve.diis_size > 16)
    return sfail(ASCC_E_ARG, "invalid server options");
  ascc_server* S = new ascc_server();
  S->opts = *opts;
  S->slab_bytes = opts->hbm_budget / kSlabAlign * kSlabAlign;
  if (hipMalloc((void**)&S->slab, S->slab_bytes) != hipSuccess) {
    (void)hipGetLastError();
    delete S;
    return sfail(ASCC_E_NOMEM, "cannot allocate the server slab of " + std::to_string(opts->hbm_budget) + " bytes");
  }
  register_buffer(S->slab, S->slab_bytes);
  S->free_list[0] = S->slab_bytes;
  *out = S;
  return ASCC_OK;
}

int ascc_server_submit_state(ascc_server* S, const double* h_B, const double* h_eps, int no, int nv, int naux,
                             int hole, int particle, int s_sign, double beta, int plascc, double t_submit,
                             int* id) {
  if (hole < 0 || hole >= no || particle < no || particle >= no + nv)
    return sfail(ASCC_E_ARG, "hole must be an occupied and particle a virtual orbital index");
  if (s_sign != 1 && s_sign != -1) return sfail(ASCC_E_ARG, "s_sign must be +1 or -1");
  if (!(beta > 0.0)) return sfail(ASCC_E_ARG, "beta must be positive");
  if (plascc && S) {
    size_t ib = 0, db = 0, pb = 0;
    const size_t bytes = request_bytes(S, no, nv, naux, true, &ib, &db, &pb);
    if (!bytes) return ASCC_E_SHAPE;
    if (bucket_header(1) + bytes > S->slab_bytes) return sfail(ASCC_E_NOMEM, "request larger than the whole HBM budget");
  }
  int rc = ascc_server_submit(S, h_B, h_eps, no, nv, naux, t_submit, id);
  if (rc) return rc;
  Request* R = S->reqs[*id];
  R->hole = hole;
  R->particle = particle;
  R->s_sign = s_sign;
  R->beta = beta;
  R->plascc = plascc != 0;
  return ASCC_OK;
}

int ascc_server_submit(ascc_server* S, const double* h_B, const double* h_eps, int no, int nv, int naux,
                       double t_submit, int* id) {
  if (!S || !h_B || !h_eps || !id) return sfail(ASCC_E_ARG, "NULL argument to ascc_server_submit");
  size_t ib = 0, db = 0, pb = 0;
  // the footprint of a PLASCC request (ascc_server_submit_state) is checked there
  const size_t bytes = request_bytes(S, no, nv, naux, false, &ib, &db, &pb);
  if (!bytes) return ASCC_E_SHAPE;  // message set by ascc_workspace_bytes
  if (bucket_header(1) + bytes > S->slab_bytes) return sfail(ASCC_E_NOMEM, "request larger than the whole HBM budget");
  Request* R = new Request();
  R->id = (int)S->reqs.size();
  R->o = no;
  R->v = nv;
  R->Q = naux;
  const size_t n = (size_t)no + nv;
  R->hB.assign(h_B, h_B + (size_t)naux * n * n);
  R->heps.assign(h_eps, h_eps + n);
  R->t_submit = t_submit;
  S->reqs.push_back(R);
  S->queue.push_back(R->id);
  *id = R->id;
  return ASCC_OK;
}

int ascc_server_step(ascc_server* S, double now, int* n_queued, int* n_running, int* n_done) {
  if (!S) return sfail(ASCC_E_ARG, "NULL server");
  // 1. finished iterations: every slot of a bucket whose iteration has completed
  std::vector<int> bids;
  for (auto& b : S->buckets) bids.push_back(b.first);
  for (int bid : bids) {
    Bucket* B = S->buckets[bid];
    if (!B->inflight) continue;
    const hipError_t q = hipEventQuery(B->ev);
    if (q == hipErrorNotReady) continue;
    B->inflight = false;
    for (int k : B->launched) {
      const int id = B->slot_req[k];
      if (id < 0) continue;
      Request* R = S->reqs[id];
      bool finished;
      if (q != hipSuccess) {
        R->status = ASCC_E_HIP;
        R->t_done = now;
        finished = true;
      } else {
        finished = consume(S, R, B->hstats + 8 * k, B->stream, now);
      }
      if (finished) {
        release_request(S, R);
        S->running -= 1;
        S->n_done += 1;
        if (!S->buckets.count(bid)) break;  // the bucket emptied and was released
      }
    }
    if (S->buckets.count(bid) && S->buckets[bid]->used() == 0) release_bucket(S, bid);
  }
  // 2. admission in arrival order while the head fits (a free slot of its shape's bucket, or a new
  //    bucket in the remaining budget) and fewer than max_active requests run
  while (!S->queue.empty() && S->running < S->opts.max_active) {
    Request* R = S->reqs[S->queue.front()];
    const size_t bytes = request_bytes(S, R->o, R->v, R->Q, R->plascc, &R->ints_bytes, &R->diis_bytes,
                                       &R->plascc_bytes);
    const bool shared = R->hole < 0 && !R->plascc;
    int bid = -1, slot = -1;
    if (shared)
      for (auto& b : S->buckets) {
        Bucket* B = b.second;
        if (!B->shared || B->o != R->o || B->v != R->v || B->Q != R->Q) continue;
        for (int k = 0; k < B->cap && slot < 0; ++k)
          if (B->slot_req[k] < 0) slot = k;
        if (slot >= 0) {
          bid = b.first;
          break;
        }
      }
    if (bid < 0) {
      const int rc = open_bucket(S, R, bytes, &bid);
      if (rc == ASCC_E_NOMEM) break;  // waits for memory
      if (rc) return rc;
      slot = 0;
    }
    Bucket* B = S->buckets[bid];
    S->queue.pop_front();
    R->bucket = R->last_bucket = bid;
    R->slot = R->last_slot = slot;
    R->bytes = bytes;
    B->slot_req[slot] = R->id;
    const int rc = admit(S, R, now);
    if (rc) {
      R->status = rc;
      R->t_done = now;
      (void)hipStreamSynchronize(B->stream);
      release_request(S, R);
      S->n_done += 1;
      continue;
    }
    S->running += 1;
  }
  // 3. one more iteration for the running slots of every idle bucket
  for (auto& b : S->buckets) {
    if (b.second->inflight) continue;
    const int rc = launch_bucket(S, b.second);
    if (rc) return rc;
  }
  if (n_queued) *n_queued = (int)S->queue.size();
  if (n_running) *n_running = S->running;
  if (n_done) *n_done = S->n_done;
  return ASCC_OK;
}

int ascc_server_info(const ascc_server* S, int id, ascc_request_info* info) {
  if (!S || !info || id < 0 || id >= (int)S->reqs.size()) return sfail(ASCC_E_ARG, "unknown request");
  const Request* R = S->reqs[id];
  info->id = R->id;
  info->no = R->o;
  info->nv = R->v;
  info->naux = R->Q;
  info->status = R->status;
  info->iterations = R->iterations;
  info->lowp_iterations = R->lowp_iterations;
  info->e_corr = R->e_corr;
  info->rnorm = R->rnorm;
  info->rmax = R->rmax;
  info->t_submit = R->t_submit;
  info->t_admit = R->t_admit;
  info->t_done = R->t_done;
  size_t ib = 0, db = 0, pb = 0;
  info->bytes = request_bytes(S, R->o, R->v, R->Q, R->plascc, &ib, &db, &pb);
  info->e_ref = R->e_ref;
  info->hole = R->hole;
  info->particle = R->particle;
  info->bucket = R->last_bucket;
  info->slot = R->last_slot;
  return ASCC_OK;
}

void ascc_server_free(ascc_server* S) {
  if (!S) return;
  (void)hipDeviceSynchronize();
  for (Request* R : S->reqs) {
    if (R->diis) ascc_diis_free(R->diis);
    if (R->ints) ascc_ints_free(R->ints);
    delete R;
  }
  std::vector<int> bids;
  for (auto& b : S->buckets) bids.push_back(b.first);
  for (int bid : bids) {
    S->buckets[bid]->inflight = false;
    release_bucket(S, bid);
  }
  for (hipStream_t s : S->stream_pool) (void)hipStreamDestroy(s);
  for (hipEvent_t e : S->event_pool) (void)hipEventDestroy(e);
  unregister_buffer(S->slab);
  (void)hipFree(S->slab);
  delete S;
}

}  // extern "C"
