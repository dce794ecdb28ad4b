// Request server: continuous batching of MINRES solves of mixed shapes on one GPU.
//
// A request waits in a FIFO queue until a slot can be given to it.  A slot is a
// plan (with its own HIP stream and workspace) plus the request's right-hand side
// and solution vectors; slots are cached per shape after their request finishes and
// evicted least-recently-used when the byte budget is needed for another shape.
// Admission is first fit in arrival order; once the oldest request has waited longer
// than kStarveSeconds the scan stops at it, so large requests are not starved.
// Every step() advances each active solve by at most one more queued iteration,
// keeping up to kAhead iterations in flight beyond the newest observed state (fewer
// when the observed residual decay predicts the stop), and retires solves whose
// snapshot shows that every right-hand side has stopped.
//
// Group lane (abac_server_group_lane): requests of at most a given number of unknowns,
// whose iterations are bound by launch latency, run as members of one group
// (abac_group_*): a step advances all of them together with one launch per MINRES
// step, on the server's own stream; requests join and leave the group as they are
// admitted and retired.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <chrono>
#include <climits>
#include <cmath>
#include <cstring>
#include <deque>
#include <map>
#include <string>
#include <vector>

#include "../../include/abac.h"
#include "abac_internal.h"
#include "plan_internal.h"

namespace {

constexpr int kAhead = 2;
constexpr double kStarveSeconds = 0.25;
constexpr int kGroupLaneMax = 64;   // members of the group lane (abac_group_set's limit)

struct Key {
  int nx, ny, nt, prec;
  double T, alpha;
  bool operator<(const Key& o) const {
    if (nx != o.nx) return nx < o.nx;
    if (ny != o.ny) return ny < o.ny;
    if (nt != o.nt) return nt < o.nt;
    if (prec != o.prec) return prec < o.prec;
    if (T != o.T) return T < o.T;
    return alpha < o.alpha;
  }
};

struct Slot {
  Key key;
  abac_plan* plan = nullptr;
  hipStream_t stream = nullptr;
  void* mem = nullptr;        // one allocation: workspace | f | u | zero level
  size_t bytes = 0;
  double* f = nullptr;
  double* u = nullptr;
  double* zero = nullptr;
  size_t n = 0;               // unknowns
  bool busy = false;
  long long last_used = 0;
};

enum Phase { QUEUED = 0, ACTIVE = 1, DONE = 2 };

struct Req {
  long long ticket;
  Key key;
  unsigned long long seed;
  double tol;
  int maxit;
  double arrival;
  bool keep;
  Phase phase = QUEUED;
  Slot* slot = nullptr;
  bool in_group = false;
  long long enq = 0, obs = 0, est = LLONG_MAX;
  double rel_last = -1.0;
  int iters = 0, status = 0;
  double relres = 0.0, t_done = 0.0;
};

size_t align256(size_t x) { return (x + 255) & ~(size_t)255; }

size_t slot_bytes(const Key& k) {
  const size_t ws = abac_workspace_bytes(k.nx, k.ny, k.nt, k.prec, 1);
  if (!ws) return 0;
  const size_t n = (size_t)k.nt * k.nx * (k.ny ? k.ny : 1);
  const size_t m = (size_t)k.nx * (k.ny ? k.ny : 1);
  return align256(ws) + 2 * align256(n * sizeof(double)) + align256(m * sizeof(double));
}

thread_local std::string g_server_error;

}  // namespace

struct abac_server {
  size_t budget = 0, used = 0;
  int max_active = 1;
  std::chrono::steady_clock::time_point t0;
  long long next_ticket = 1;
  long long tick = 0;
  std::deque<Req*> queue;
  std::vector<Req*> active;
  std::map<long long, Req*> reqs;
  std::vector<Slot*> slots;
  // group lane
  size_t group_max_n = 0;       // 0: no lane
  hipStream_t gstream = nullptr;
  abac_group* group = nullptr;
  std::vector<Req*> gmembers;
  bool gdirty = false;

  double now() const {
    return std::chrono::duration<double>(std::chrono::steady_clock::now() - t0).count();
  }
};

namespace {

void free_slot(abac_server* s, Slot* sl) {
  if (sl->plan) abac_plan_destroy(sl->plan);
  if (sl->stream) (void)hipStreamDestroy(sl->stream);
  if (sl->mem) (void)hipFree(sl->mem);
  s->used -= sl->bytes;
  s->slots.erase(std::find(s->slots.begin(), s->slots.end(), sl));
  delete sl;
}

// An idle cached slot of this shape, or a new one if the budget allows (evicting
// idle slots of other shapes, least recently used first).  nullptr if not now.
Slot* acquire_slot(abac_server* s, const Key& k, abac_status* err) {
  *err = ABAC_OK;
  for (Slot* sl : s->slots)
    if (!sl->busy && !(sl->key < k) && !(k < sl->key)) return sl;
  const size_t need = slot_bytes(k);
  if (s->used + need > s->budget) {
    std::vector<Slot*> idle;
    for (Slot* sl : s->slots)
      if (!sl->busy) idle.push_back(sl);
    std::sort(idle.begin(), idle.end(), [](const Slot* a, const Slot* b) { return a->last_used < b->last_used; });
    size_t freeable = 0;
    for (Slot* sl : idle) freeable += sl->bytes;
    if (s->used - freeable + need > s->budget) return nullptr;
    for (Slot* sl : idle) {
      if (s->used + need <= s->budget) break;
      free_slot(s, sl);
    }
  }
  Slot* sl = new Slot();
  sl->key = k;
  sl->bytes = need;
  sl->n = (size_t)k.nt * k.nx * (k.ny ? k.ny : 1);
  const size_t m = (size_t)k.nx * (k.ny ? k.ny : 1);
  const size_t ws = align256(abac_workspace_bytes(k.nx, k.ny, k.nt, k.prec, 1));
  if (hipMalloc(&sl->mem, need) != hipSuccess) {
    delete sl;
    *err = ABAC_ENOMEM;
    g_server_error = "hipMalloc failed for a request slot";
    return nullptr;
  }
  char* base = static_cast<char*>(sl->mem);
  sl->f = reinterpret_cast<double*>(base + ws);
  sl->u = reinterpret_cast<double*>(base + ws + align256(sl->n * sizeof(double)));
  sl->zero = reinterpret_cast<double*>(base + ws + 2 * align256(sl->n * sizeof(double)));
  if (hipStreamCreateWithFlags(&sl->stream, hipStreamNonBlocking) != hipSuccess) {
    (void)hipFree(sl->mem);
    delete sl;
    *err = ABAC_EDEVICE;
    return nullptr;
  }
  abac_status st = abac_plan_create(k.nx, k.ny, k.nt, k.T, k.alpha, k.prec, 1, sl->stream, sl->mem, ws, &sl->plan);
  if (st == ABAC_OK && abac::launch_fill_zero(sl->zero, m, sl->stream) != hipSuccess) st = ABAC_EDEVICE;
  if (st != ABAC_OK) {
    if (sl->plan) abac_plan_destroy(sl->plan);
    (void)hipStreamDestroy(sl->stream);
    (void)hipFree(sl->mem);
    delete sl;
    *err = st;
    return nullptr;
  }
  s->slots.push_back(sl);
  s->used += need;
  return sl;
}

abac_status start(abac_server* s, Req* r) {
  Slot* sl = r->slot;
  (void)s;
  if (abac::launch_fill_normal(sl->u, sl->n, r->seed, sl->stream) != hipSuccess) return ABAC_EDEVICE;
  abac_status st = abac_build_rhs(sl->plan, sl->u, sl->zero, sl->zero, sl->f);
  if (st != ABAC_OK) return st;
  st = abac_minres_begin(sl->plan, sl->f, sl->u, r->tol, r->maxit);
  if (st != ABAC_OK) return st;
  r->enq = 0;
  r->obs = 0;
  r->est = LLONG_MAX;
  r->rel_last = -1.0;
  r->phase = ACTIVE;
  r->in_group = s->group && sl->n <= s->group_max_n && (int)s->gmembers.size() < kGroupLaneMax &&
                (s->gmembers.empty() || s->gmembers[0]->key.prec == sl->key.prec) &&
                abac::group_accepts(sl->plan);
  if (r->in_group) {
    s->gmembers.push_back(r);
    s->gdirty = true;
  }
  return ABAC_OK;
}

// Unknowns of a request's right-hand side.
size_t req_unknowns(const Key& k) { return (size_t)k.nt * k.nx * (k.ny ? k.ny : 1); }

// Admission: max_active caps the solves on their own streams; requests small enough
// for the group lane are capped by the lane's size instead (they cost a share of the
// lane's launches, not launches of their own).
void admit(abac_server* s) {
  const double t = s->now();
  for (auto it = s->queue.begin(); it != s->queue.end();) {
    const int own = (int)(s->active.size() - s->gmembers.size());
    const bool lane_ok = s->group && (int)s->gmembers.size() < kGroupLaneMax;
    if (own >= s->max_active && !lane_ok) return;
    Req* r = *it;
    const bool small = s->group && req_unknowns(r->key) <= s->group_max_n;
    if (small ? !lane_ok : own >= s->max_active) {
      ++it;
      continue;
    }
    abac_status err;
    Slot* sl = acquire_slot(s, r->key, &err);
    if (!sl) {
      if (err != ABAC_OK) {   // cannot be served at all: finish with the error
        r->phase = DONE;
        r->status = err;
        r->t_done = s->now();
        it = s->queue.erase(it);
        continue;
      }
      if (it == s->queue.begin() && t - r->arrival > kStarveSeconds) return;   // hold memory for the oldest
      ++it;
      continue;
    }
    sl->busy = true;
    sl->last_used = ++s->tick;
    r->slot = sl;
    abac_status st = start(s, r);
    it = s->queue.erase(it);
    if (st != ABAC_OK) {
      r->phase = DONE;
      r->status = st;
      r->t_done = s->now();
      sl->busy = false;
      continue;
    }
    s->active.push_back(r);
  }
}

void finish_req(abac_server* s, Req* r) {
  int it = 0, stt = 0;
  double rr = 0;
  abac_minres_finish(r->slot->plan, &it, &rr, &stt);
  r->iters = it;
  r->relres = rr;
  r->status = stt;
  r->t_done = s->now();
}

// Whether a request wants another iteration queued: fewer than kAhead beyond the
// newest observed state, not past maxit or the predicted stop.
bool wants_more(const Req* r) { return r->enq < r->maxit && r->enq - r->obs <= kAhead && r->enq < r->est; }

// Advance one active request; returns true when it has finished.  Requests of the group
// lane are only observed here (the group advances them).
bool advance(abac_server* s, Req* r) {
  abac_plan* p = r->slot->plan;
  // observe every snapshot that has completed since the last look
  while (r->obs < r->enq) {
    int ready = 0;
    const MinresState* snap = nullptr;
    if (abac::plan_peek_snapshot(p, r->obs + 1, &ready, &snap) != ABAC_OK || !ready) break;
    ++r->obs;
    if (snap[0].state != abac::ST_RUNNING) {
      int it = 0, stt = 0;
      double rr = 0;
      abac_minres_finish(p, &it, &rr, &stt);
      r->iters = it;
      r->relres = rr;
      r->status = stt;
      r->t_done = s->now();
      return true;
    }
    const double rel = snap[0].bnorm2 > 0 ? std::sqrt(snap[0].rnorm2 / snap[0].bnorm2) : 0.0;
    if (r->rel_last > 0.0 && rel > 0.0 && rel < r->rel_last) {
      const double rem = std::ceil(std::log(r->tol / rel) / std::log(rel / r->rel_last));
      r->est = r->obs + (long long)std::max(1.0, std::min(rem, 1e6));
    } else {
      r->est = LLONG_MAX;
    }
    r->rel_last = rel;
  }
  if (r->obs == 0 && r->enq == 0) {
    // the set-up snapshot (number 0) may already report a stopped solve (zero source)
    int ready = 0;
    const MinresState* snap = nullptr;
    if (abac::plan_peek_snapshot(p, 0, &ready, &snap) == ABAC_OK && ready && snap[0].state != abac::ST_RUNNING) {
      int it = 0, stt = 0;
      double rr = 0;
      abac_minres_finish(p, &it, &rr, &stt);
      r->iters = it;
      r->relres = rr;
      r->status = stt;
      r->t_done = s->now();
      return true;
    }
  }
  if (r->in_group) {
    if (r->enq >= r->maxit && r->obs >= r->enq) {
      finish_req(s, r);
      return true;
    }
    if (r->obs >= r->enq && r->enq >= r->est) r->est = r->enq + 1;   // prediction was early
    return false;
  }
  if (wants_more(r)) {
    if (abac_minres_advance(p, 1) == ABAC_OK) ++r->enq;
  } else if (r->enq >= r->maxit && r->obs >= r->enq) {
    int it = 0, stt = 0;
    double rr = 0;
    abac_minres_finish(p, &it, &rr, &stt);
    r->iters = it;
    r->relres = rr;
    r->status = stt;
    r->t_done = s->now();
    return true;
  } else if (r->obs >= r->enq && r->enq >= r->est) {
    r->est = r->enq + 1;   // prediction was early
  }
  return false;
}

}  // namespace

extern "C" {

abac_status abac_fill_normal(void* stream, double* out, size_t n, unsigned long long seed) {
  if (!out) return ABAC_EINVAL;
  return abac::launch_fill_normal(out, n, seed, static_cast<hipStream_t>(stream)) == hipSuccess ? ABAC_OK
                                                                                                : ABAC_EDEVICE;
}

abac_status abac_server_create(size_t budget_bytes, int max_active, abac_server** out) {
  if (!out || budget_bytes == 0 || max_active < 1) return ABAC_EINVAL;
  abac_server* s = new abac_server();
  s->budget = budget_bytes;
  s->max_active = max_active;
  s->t0 = std::chrono::steady_clock::now();
  *out = s;
  return ABAC_OK;
}

abac_status abac_server_destroy(abac_server* s) {
  if (!s) return ABAC_OK;
  if (s->group) abac_group_destroy(s->group);
  if (s->gstream) (void)hipStreamDestroy(s->gstream);
  for (Slot* sl : s->slots)
    if (sl->stream) (void)hipStreamSynchronize(sl->stream);
  while (!s->slots.empty()) free_slot(s, s->slots.back());
  for (auto& kv : s->reqs) delete kv.second;
  delete s;
  return ABAC_OK;
}

abac_status abac_server_submit(abac_server* s, int nx, int ny, int nt, double T, double alpha, int prec,
                               unsigned long long seed, double tol, int maxit, double arrival_s, int keep_solution,
                               long long* ticket) {
  if (!s || !ticket) return ABAC_EINVAL;
  Key k{nx, ny, nt, prec, T, alpha};
  const size_t need = slot_bytes(k);
  if (!need || !(tol > 0) || maxit < 1 || !(alpha > 0) || alpha > 1 || !(T > 0)) return ABAC_EINVAL;
  if (need > s->budget) return ABAC_EBUDGET;
  Req* r = new Req();
  r->ticket = s->next_ticket++;
  r->key = k;
  r->seed = seed;
  r->tol = tol;
  r->maxit = maxit;
  r->arrival = arrival_s;
  r->keep = keep_solution != 0;
  s->reqs[r->ticket] = r;
  s->queue.push_back(r);
  *ticket = r->ticket;
  return ABAC_OK;
}

abac_status abac_server_group_lane(abac_server* s, size_t max_unknowns) {
  if (!s) return ABAC_EINVAL;
  if (!s->active.empty() || !s->queue.empty()) return ABAC_EINVAL;   // only while idle
  if (max_unknowns && !s->group) {
    if (hipStreamCreateWithFlags(&s->gstream, hipStreamNonBlocking) != hipSuccess) return ABAC_EDEVICE;
    abac_status st = abac_group_create(s->gstream, &s->group);
    if (st != ABAC_OK) return st;
  }
  s->group_max_n = max_unknowns;
  return ABAC_OK;
}

abac_status abac_server_step(abac_server* s, int* active, int* queued) {
  if (!s) return ABAC_EINVAL;
  admit(s);
  for (size_t i = 0; i < s->active.size();) {
    Req* r = s->active[i];
    if (advance(s, r)) {
      if (r->in_group) {
        s->gmembers.erase(std::find(s->gmembers.begin(), s->gmembers.end(), r));
        s->gdirty = true;
      }
      r->phase = DONE;
      if (!r->keep) {
        r->slot->busy = false;
        r->slot->last_used = ++s->tick;
        r->slot = nullptr;
      }
      s->active.erase(s->active.begin() + i);
      continue;
    }
    ++i;
  }
  // the group lane: new membership, then one more iteration of every member if any
  // of them wants it (members that have stopped skip the work on the device)
  if (s->group) {
    if (s->gdirty) {
      std::vector<abac_plan*> plans;
      for (Req* r : s->gmembers) plans.push_back(r->slot->plan);
      abac_status st = abac_group_set(s->group, plans.data(), (int)plans.size());
      if (st != ABAC_OK) return st;
      s->gdirty = false;
    }
    bool more = false;
    for (Req* r : s->gmembers) more = more || wants_more(r);
    if (more) {
      abac_status st = abac_group_advance(s->group, 1);
      if (st != ABAC_OK) return st;
      for (Req* r : s->gmembers) ++r->enq;
    }
  }
  if (active) *active = (int)s->active.size();
  if (queued) *queued = (int)s->queue.size();
  return ABAC_OK;
}

abac_status abac_server_result(abac_server* s, long long ticket, double* u_host, int* iters, double* relres,
                               int* status, double* latency_s) {
  if (!s) return ABAC_EINVAL;
  auto it = s->reqs.find(ticket);
  if (it == s->reqs.end()) return ABAC_EINVAL;
  Req* r = it->second;
  if (r->phase != DONE) return ABAC_EAGAIN;
  if (iters) *iters = r->iters;
  if (relres) *relres = r->relres;
  if (status) *status = r->status;
  if (latency_s) *latency_s = r->t_done - r->arrival;
  if (r->slot) {
    if (u_host)
      (void)hipMemcpy(u_host, r->slot->u, r->slot->n * sizeof(double), hipMemcpyDeviceToHost);
    r->slot->busy = false;
    r->slot->last_used = ++s->tick;
    r->slot = nullptr;
  }
  s->reqs.erase(it);
  delete r;
  return ABAC_OK;
}

double abac_server_clock(abac_server* s) { return s ? s->now() : 0.0; }

size_t abac_server_bytes_in_use(abac_server* s) { return s ? s->used : 0; }

}  // extern "C"
