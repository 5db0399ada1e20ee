// Request loop for many independent solves on one GPU (continuous batching at the iteration
// level).
//
// * Admission by HBM footprint: the server owns one device slab (allocated once) and carves
//   each admitted request's whole working set -- integral set, DIIS state, amplitudes,
//   residuals, staging for its DF tensor -- out of it with a first-fit free list, in arrival
//   order.  No device allocation happens while requests run.
// * Every running request has its own stream.  One iteration (residual + Jacobi/DIIS update)
//   is captured once per precision into a hipGraph and replayed; each step of the loop
//   launches one iteration for every running request whose previous iteration has finished,
//   so work of different requests overlaps on the device, and requests join and leave between
//   iterations as slab space and stream slots free up.
// * The convergence test reads an 8-double statistics block copied to pinned host memory
//   behind each iteration (polled with an event, never a blocking wait).  A low-precision
//   request runs its bulk iterations in that precision and finishes in FP64 (the FP64
//   refinement of ascc_solve).
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

struct Request {
  int id = 0, o = 0, v = 0, Q = 0;
  std::vector<double> hB, heps;  // host copies until admission
  double t_submit = 0, t_admit = -1, t_done = -1;
  int status = 1;  // 1 queued, 2 running, 0 converged, <0 ASCC_E_*
  size_t bytes = 0, off = 0;
  size_t ints_bytes = 0, diis_bytes = 0, plascc_bytes = 0;
  ascc_ints* ints = nullptr;
  ascc_diis* diis = nullptr;
  double *t1 = nullptr, *t2 = nullptr, *r1 = nullptr, *r2 = nullptr, *e = nullptr, *stats = nullptr;
  double *dB = nullptr, *deps = nullptr;
  double* hstats = nullptr;  // pinned, 8 doubles
  hipStream_t stream = nullptr;
  hipEvent_t ev = nullptr;
  hipGraphExec_t g_low = nullptr, g_fp64 = nullptr;
  bool inflight = false, lowp_phase = false;
  LowpStall stall;
  int iterations = 0, lowp_iterations = 0;
  double e_corr = 0, rnorm = 0, rmax = 0, de = 0;
  int hole = -1, particle = -1, s_sign = 1;  // a 1-CSF state (hole >= 0) or the ground state
  double beta = 1.0, e_ref = 0.0;
  bool plascc = false;
};

}  // namespace

struct ascc_server {
  ascc_server_opts opts{};
  char* slab = nullptr;
  size_t slab_bytes = 0;
  std::map<size_t, size_t> free_list;  // offset -> length
  std::vector<Request*> reqs;
  std::deque<int> queue;
  std::vector<int> running;
  std::vector<hipStream_t> stream_pool;
  std::vector<hipEvent_t> event_pool;
  std::vector<double*> pinned_pool;
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

// Layout of a request's region: [ints | diis | t1 t2 r1 r2 e stats eps | B staging | PLASCC buffers]
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
  b += align_s(8 * ov) * 2 + align_s(8 * oovv) * 2 + align_s(8) + align_s(64) + align_s(8 * n);
  b += align_s(8 * (size_t)Q * n * n);
  b += align_s(pl_b);
  return b;
}

void release(ascc_server* S, Request* R) {
  if (R->g_low) (void)hipGraphExecDestroy(R->g_low);
  if (R->g_fp64) (void)hipGraphExecDestroy(R->g_fp64);
  R->g_low = R->g_fp64 = nullptr;
  if (R->diis) ascc_diis_free(R->diis);
  if (R->ints) ascc_ints_free(R->ints);
  R->diis = nullptr;
  R->ints = nullptr;
  if (R->bytes) slab_give(S, R->off, R->bytes);
  R->bytes = 0;
  if (R->stream) S->stream_pool.push_back(R->stream);
  if (R->ev) S->event_pool.push_back(R->ev);
  if (R->hstats) S->pinned_pool.push_back(R->hstats);
  R->stream = nullptr;
  R->ev = nullptr;
  R->hstats = nullptr;
}

// One iteration (residual at t, then the update of t) on the request's stream.
int iteration(Request* R, hipStream_t s) {
  int rc = ascc_residual(R->ints, R->t1, R->t2, R->r1, R->r2, R->e, s);
  if (!rc) rc = ascc_update(R->ints, R->diis, R->t1, R->t2, R->r1, R->r2, R->e, 0.0, R->stats, s);
  return rc;
}

int capture(Request* R, int precision, hipGraphExec_t* out) {
  int rc = ascc_set_precision(R->ints, precision);
  if (rc) return rc;
  hipGraph_t g = nullptr;
  if (hipStreamBeginCapture(R->stream, hipStreamCaptureModeThreadLocal) != hipSuccess)
    return sfail(ASCC_E_HIP, "hipStreamBeginCapture failed");
  rc = iteration(R, R->stream);
  hipError_t e = hipStreamEndCapture(R->stream, &g);
  if (rc) {
    if (g) (void)hipGraphDestroy(g);
    return rc;
  }
  if (e != hipSuccess) return sfail(ASCC_E_HIP, std::string("hipStreamEndCapture: ") + hipGetErrorString(e));
  e = hipGraphInstantiate(out, g, nullptr, nullptr, 0);
  (void)hipGraphDestroy(g);
  if (e != hipSuccess) return sfail(ASCC_E_HIP, std::string("hipGraphInstantiate: ") + hipGetErrorString(e));
  return ASCC_OK;
}

int admit(ascc_server* S, Request* R, double now) {
  const size_t ov = (size_t)R->o * R->v, oovv = (size_t)R->o * R->o * R->v * R->v, n = (size_t)R->o + R->v;
  char* base = S->slab + R->off;
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
  R->stats = carve(64);
  R->deps = carve(8 * n);
  R->dB = carve(8 * (size_t)R->Q * n * n);
  char* plascc_ws = base + p;  // R->plascc_bytes (0 unless a PLASCC request)
  p += align_s(R->plascc_bytes);
  if (!S->stream_pool.empty()) {
    R->stream = S->stream_pool.back();
    S->stream_pool.pop_back();
  } else if (hipStreamCreateWithFlags(&R->stream, hipStreamNonBlocking) != hipSuccess) {
    return sfail(ASCC_E_HIP, "hipStreamCreate failed");
  }
  if (!S->event_pool.empty()) {
    R->ev = S->event_pool.back();
    S->event_pool.pop_back();
  } else if (hipEventCreateWithFlags(&R->ev, hipEventDisableTiming) != hipSuccess) {
    return sfail(ASCC_E_HIP, "hipEventCreate failed");
  }
  if (!S->pinned_pool.empty()) {
    R->hstats = S->pinned_pool.back();
    S->pinned_pool.pop_back();
  } else if (hipHostMalloc((void**)&R->hstats, 64, 0) != hipSuccess) {
    return sfail(ASCC_E_NOMEM, "pinned host allocation failed");
  }
  hipStream_t s = R->stream;
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
  if (R->plascc &&
      (rc = ascc_set_plascc_ws(R->ints, R->hole, R->particle, plascc_ws, R->plascc_bytes, s)))
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
  if (S->opts.use_graphs) {
    if (R->lowp_phase && (rc = capture(R, S->opts.precision, &R->g_low))) return rc;
    if ((rc = capture(R, ASCC_PREC_FP64, &R->g_fp64))) return rc;
  }
  (void)ascc_set_precision(R->ints, R->lowp_phase ? S->opts.precision : ASCC_PREC_FP64);
  R->t_admit = now;
  R->status = 2;
  return ASCC_OK;
}

int launch(Request* R) {
  hipStream_t s = R->stream;
  if (R->g_fp64) {
    if (hipGraphLaunch(R->lowp_phase ? R->g_low : R->g_fp64, s) != hipSuccess)
      return sfail(ASCC_E_HIP, "hipGraphLaunch failed");
  } else {
    int rc = iteration(R, s);
    if (rc) return rc;
  }
  if (hipMemcpyAsync(R->hstats, R->stats, 64, hipMemcpyDeviceToHost, s) != hipSuccess ||
      hipEventRecord(R->ev, s) != hipSuccess)
    return sfail(ASCC_E_HIP, "statistics copy failed");
  R->inflight = true;
  return ASCC_OK;
}

// Consume a finished iteration's statistics; returns true if the request is finished.
bool consume(ascc_server* S, Request* R, double now) {
  const ascc_opts& o = S->opts.solve;
  const double* st = R->hstats;
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
      (void)ascc_diis_reset(R->diis, R->stream);
    }
  } else {
    if (ok) {
      R->status = ASCC_OK;
      R->t_done = now;
      (void)ascc_reference_energy(R->ints, &R->e_ref, R->stream);  // the stream is idle: no wait
      return true;
    }
  }
  if (R->iterations >= o.maxiter) {
    R->status = ASCC_E_NOT_CONVERGED;
    R->t_done = now;
    (void)ascc_reference_energy(R->ints, &R->e_ref, R->stream);
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
    if (bytes > S->slab_bytes) return sfail(ASCC_E_NOMEM, "request larger than the whole HBM budget");
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
  if (bytes > S->slab_bytes) return sfail(ASCC_E_NOMEM, "request larger than the whole HBM budget");
  Request* R = new Request();
  R->id = (int)S->reqs.size();
  R->o = no;
  R->v = nv;
  R->Q = naux;
  const size_t n = (size_t)no + nv;
  R->hB.assign(h_B, h_B + (size_t)naux * n * n);
  R->heps.assign(h_eps, h_eps + n);
  R->t_submit = t_submit;
  R->ints_bytes = ib;
  R->diis_bytes = db;
  R->bytes = 0;
  S->reqs.push_back(R);
  S->queue.push_back(R->id);
  *id = R->id;
  (void)bytes;
  return ASCC_OK;
}

int ascc_server_step(ascc_server* S, double now, int* n_queued, int* n_running, int* n_done) {
  if (!S) return sfail(ASCC_E_ARG, "NULL server");
  // 1. finished iterations
  for (size_t k = 0; k < S->running.size();) {
    Request* R = S->reqs[S->running[k]];
    if (R->inflight) {
      const hipError_t q = hipEventQuery(R->ev);
      if (q == hipErrorNotReady) {
        ++k;
        continue;
      }
      R->inflight = false;
      if (q != hipSuccess) {
        R->status = ASCC_E_HIP;
        R->t_done = now;
      } else if (!consume(S, R, now)) {
        ++k;
        continue;
      }
      release(S, R);
      S->n_done += 1;
      S->running.erase(S->running.begin() + k);
      continue;
    }
    ++k;
  }
  // 2. admission in arrival order while the head fits the remaining budget and a slot is free
  while (!S->queue.empty() && (int)S->running.size() < S->opts.max_active) {
    Request* R = S->reqs[S->queue.front()];
    const size_t bytes = request_bytes(S, R->o, R->v, R->Q, R->plascc, &R->ints_bytes, &R->diis_bytes,
                                       &R->plascc_bytes);
    size_t off = 0;
    if (!slab_take(S, bytes, &off)) break;
    R->off = off;
    R->bytes = bytes;
    S->queue.pop_front();
    const int rc = admit(S, R, now);
    if (rc) {
      R->status = rc;
      R->t_done = now;
      if (R->stream) (void)hipStreamSynchronize(R->stream);
      release(S, R);
      S->n_done += 1;
      continue;
    }
    S->running.push_back(R->id);
  }
  // 3. one more iteration for every running request that is idle
  for (int id : S->running) {
    Request* R = S->reqs[id];
    if (!R->inflight) {
      const int rc = launch(R);
      if (rc) return rc;
    }
  }
  if (n_queued) *n_queued = (int)S->queue.size();
  if (n_running) *n_running = (int)S->running.size();
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
  return ASCC_OK;
}

void ascc_server_free(ascc_server* S) {
  if (!S) return;
  (void)hipDeviceSynchronize();
  for (Request* R : S->reqs) {
    release(S, R);
    delete R;
  }
  for (hipStream_t s : S->stream_pool) (void)hipStreamDestroy(s);
  for (hipEvent_t e : S->event_pool) (void)hipEventDestroy(e);
  for (double* p : S->pinned_pool) (void)hipHostFree(p);
  unregister_buffer(S->slab);
  (void)hipFree(S->slab);
  delete S;
}

}  // extern "C"
