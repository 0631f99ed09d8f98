// Request loop over resident HPS factorizations (not in the paper, whose solver handles
// one problem at a time): builds and solves of many problems run on a pool of work slots
// (a host thread and a stream each) so that their kernels overlap on the device; every
// work item is admitted against a device-memory budget; queued right-hand sides of one
// problem are merged into a single solve (continuous batching), and so are those of
// other idle problems that can share the solve's launches.
//
// Scheduling: a slot that is free takes the oldest admissible item, oldest meaning the
// earliest submission among the requests it would serve.  An item is a problem's
// (re)build or one solve over queued requests of one or more problems.  The first
// solve_slots slots take no builds.  At most one item per problem runs at a time.  An
// item is admissible when the bytes it needs fit beside the committed bytes (server
// copies of c, resident factors, running items); otherwise idle factors are freed least
// recently used first, when that makes it fit (for a solve, only while no other solve
// runs: a running solve's memory comes back soon).  Once the oldest item cannot start,
// younger ones start only if they leave its bytes free.  When nothing runs and the oldest item
// still cannot fit, it fails with HPS_E_NOMEM.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <chrono>
#include <cmath>
#include <condition_variable>
#include <deque>
#include <map>
#include <memory>
#include <mutex>
#include <string>
#include <thread>
#include <vector>

#include "../../include/hps.h"
#include "kernels.hpp"
#include "serve_hooks.hpp"

namespace hps {
namespace {

using Clock = std::chrono::steady_clock;

struct SolveReq {
  uint64_t id = 0;
  int nrhs = 0;
  const double* s = nullptr;
  const double* t = nullptr;
  double* u = nullptr;
  double t_submit = 0;
};

enum class PState { Queued, Building, Resident, Evicted, Failed };

struct Problem {
  uint64_t id = 0;
  hps_domain dom{};
  int p = 0;
  double kappa = 0, er = 0, ei = 0;
  hps_opts opts{};
  double* c = nullptr;       // server's device copy of c (kept for rebuilds)
  size_t c_bytes = 0;
  size_t peak = 0;           // estimated device bytes of its build
  size_t resident = 0;       // device bytes of its factor while resident
  long nl1 = 0, n = 0, ni = 0, nt = 0;
  PState state = PState::Queued;
  hps_factor* f = nullptr;
  int fail = HPS_OK;
  std::deque<SolveReq> pending;
  bool busy = false;         // a work item of the problem is running
  bool released = false;
  uint64_t build_req = 0;
  double build_submit = 0;
  uint64_t last_use = 0;     // LRU clock value of its last work item
  bool rebuilt = false;      // rebuilt after an eviction, not yet solved with since
};

// one problem's requests in a solve
struct Share {
  Problem* pr = nullptr;
  std::vector<SolveReq> reqs;
  bool after_rebuild = false;  // the first solve after a rebuild of its factor
};

struct Work {
  enum Kind { None, Build, Solve } kind = None;
  Problem* pr = nullptr;     // the build's problem, or the first problem of a solve
  std::vector<Share> shares; // a solve's problems, pr's first
  size_t mem = 0;            // bytes committed while it runs
  bool rebuild = false;
  int R = 0;                 // right-hand sides of a solve, over all its problems
  bool any_s = false;
};

struct Freed {
  hps_factor* f = nullptr;
  double* c = nullptr;
};

size_t align256(size_t b) { return (b + 255) & ~size_t(255); }

// Device bytes a solve's allocations take for `b` bytes of workspace and staging: the
// workspace cache rounds each buffer up by at most an eighth, plus its 2 MiB grain.
size_t with_rounding(size_t b) { return b + b / 8 + (size_t(8) << 20); }

// staging of a merged solve: S (if any request has s), T, U, each 256-byte aligned
size_t staging_bytes(const Problem& p, int R, bool any_s, size_t nreq) {
  if (nreq <= 1) return 0;
  return (any_s ? align256((size_t)R * p.nl1 * p.ni * 16) : 0) +
         align256((size_t)R * p.nt * 16) + align256((size_t)R * p.nl1 * p.n * 16);
}

}  // namespace
}  // namespace hps

struct hps_server {
  int device = 0;
  hps_server_opts opts{};
  size_t budget = 0, committed = 0, peak_committed = 0;
  std::mutex mu;
  std::condition_variable cv_work, cv_done;
  std::map<uint64_t, std::unique_ptr<hps::Problem>> problems;
  std::deque<hps_completion> done;
  std::vector<std::thread> threads;
  std::vector<hipStream_t> streams;
  bool stop = false;
  uint64_t next_id = 1, lru_clock = 0;
  hps::Clock::time_point t0;
  int running = 0, max_running = 0;
  int running_solves = 0;
  size_t running_mem = 0;  // bytes committed by running items
  bool nomem_wait = false; // after an item ran out of device memory beside running
                           // work: nothing new starts until one of those ends
  int64_t builds = 0, rebuilds = 0, evictions = 0, solves = 0, rhs = 0, batches = 0;
  int64_t rejected = 0, failed = 0, shared_batches = 0, shared_problems = 0, retried = 0;
  int solve_only = 0;  // slots [0, solve_only) take no builds
  std::vector<double> lat_ms;
  double first_submit = -1.0, last_end = 0.0;
  double now() const {
    return std::chrono::duration<double>(hps::Clock::now() - t0).count();
  }
};

namespace hps {
namespace {

void complete(hps_server& S, const Problem& p, int kind, uint64_t req, int status, int nrhs,
              int batch_rhs, int iters, bool rebuilt, double ts, double t_start, double t_end) {
  hps_completion c{};
  c.req = req;
  c.problem = p.id;
  c.kind = kind;
  c.status = status;
  c.nrhs = nrhs;
  c.batch_rhs = batch_rhs;
  c.iterations = iters;
  c.rebuilt = rebuilt ? 1 : 0;
  c.t_submit = ts;
  c.t_start = t_start;
  c.t_end = t_end;
  S.done.push_back(c);
  if (status != HPS_OK) ++S.failed;
  if (S.first_submit < 0 || ts < S.first_submit) S.first_submit = ts;
  S.last_end = std::max(S.last_end, t_end);
}

bool fits(const hps_server& S, size_t need) { return S.committed + need <= S.budget; }

// Free idle factors, least recently used first, until `need` fits; nothing is freed when
// even all of them would not make it fit.  Caller holds the lock.
bool evict_for(hps_server& S, size_t need, const Problem* keep, std::vector<Freed>& fr) {
  if (fits(S, need)) return true;
  if (!S.opts.evict_idle) return false;
  std::vector<Problem*> idle;
  size_t can = 0;
  for (auto& kv : S.problems) {
    Problem* p = kv.second.get();
    if (p != keep && p->state == PState::Resident && !p->busy && p->pending.empty()) {
      idle.push_back(p);
      can += p->resident;
    }
  }
  if (S.committed - can + need > S.budget) return false;
  std::sort(idle.begin(), idle.end(),
            [](const Problem* a, const Problem* b) { return a->last_use < b->last_use; });
  for (Problem* p : idle) {
    if (fits(S, need)) break;
    fr.push_back({p->f, nullptr});
    p->f = nullptr;
    p->state = PState::Evicted;
    S.committed -= p->resident;
    p->resident = 0;
    ++S.evictions;
  }
  return fits(S, need);
}

// bytes a solve of p over its first k queued requests needs; sets R and any_s
size_t solve_need(Problem& p, size_t k, int* R, bool* any_s) {
  int r = 0;
  bool s = false;
  for (size_t i = 0; i < k; ++i) {
    r += p.pending[i].nrhs;
    s = s || p.pending[i].s != nullptr;
  }
  *R = r;
  *any_s = s;
  size_t ws = 0;
  try {
    ws = solve_workspace_bytes(p.f, r, s);
  } catch (const std::exception&) {
    return ~size_t(0) / 4;  // cannot be sized: never admitted, fails once nothing runs
  }
  return with_rounding(ws + staging_bytes(p, r, s, k));
}

// the parts of a shared solve: every request of every share
std::vector<SolvePart> parts_of(const std::vector<Share>& sh) {
  std::vector<SolvePart> parts;
  for (const Share& x : sh)
    for (const SolveReq& r : x.reqs) parts.push_back({x.pr->f, r.nrhs, r.s, r.t, r.u});
  return parts;
}

// bytes a shared solve needs
size_t shared_need(const std::vector<Share>& sh) {
  size_t b = 0;
  try {
    solve_parts(parts_of(sh), nullptr, &b);
  } catch (const std::exception&) {
    return ~size_t(0) / 4;
  }
  return with_rounding(b);
}

// requests of p's queue that one merged solve takes (at least one)
size_t batch_len(const Problem& p, int max_rhs) {
  size_t k = 0;
  int r = 0;
  while (k < p.pending.size() && (k == 0 || r + p.pending[k].nrhs <= max_rhs)) {
    r += p.pending[k].nrhs;
    ++k;
  }
  return k;
}

// Choose the next work item (caller holds the lock).  Returns true when it changed
// anything (took work, queued frees, produced completions).
bool pick(hps_server& S, Work& w, std::vector<Freed>& fr, bool builds) {
  if (S.nomem_wait && S.running > 0) return false;
  bool progress = false;
  const double tnow = S.now();
  // failed problems answer their queued solves; released idle problems go away
  for (auto it = S.problems.begin(); it != S.problems.end();) {
    Problem& p = *it->second;
    if (p.state == PState::Failed && !p.pending.empty()) {
      for (auto& r : p.pending)
        complete(S, p, HPS_REQ_SOLVE, r.id, p.fail, r.nrhs, 0, 0, false, r.t_submit, tnow, tnow);
      p.pending.clear();
      progress = true;
    }
    if (p.released && !p.busy && p.pending.empty()) {
      if (p.state == PState::Queued)  // never built: its build request ends here
        complete(S, p, HPS_REQ_BUILD, p.build_req, HPS_E_INVALID, 0, 0, 0, false,
                 p.build_submit, tnow, tnow);
      fr.push_back({p.f, p.c});
      S.committed -= p.resident + p.c_bytes;
      it = S.problems.erase(it);
      progress = true;
      continue;
    }
    ++it;
  }
  struct Cand {
    double arrival;
    Problem* p;
    Work::Kind kind;
  };
  std::vector<Cand> cands;
  for (auto& kv : S.problems) {
    Problem* p = kv.second.get();
    if (p->busy) continue;
    if (p->state == PState::Queued) {
      if (builds) cands.push_back({p->build_submit, p, Work::Build});
    } else if (p->state == PState::Evicted && !p->pending.empty()) {
      if (builds) cands.push_back({p->pending.front().t_submit, p, Work::Build});
    }
    else if (p->state == PState::Resident && !p->pending.empty())
      cands.push_back({p->pending.front().t_submit, p, Work::Solve});
  }
  std::stable_sort(cands.begin(), cands.end(),
                   [](const Cand& a, const Cand& b) { return a.arrival < b.arrival; });
  // Bytes the oldest item that cannot start yet waits for: younger items start only
  // beside them, so that memory freed by running work collects for it (a large build
  // is not starved by a stream of solves).  Only an item that would fit once the
  // running items end (with idle factors evicted) reserves: one that needs younger
  // items to run first (to make their problems idle) must not block them.
  size_t ahead = 0;
  auto hold = [&](size_t need, const Problem* keep) {
    if (ahead) return;
    size_t idle = 0;
    if (S.opts.evict_idle)
      for (auto& kv : S.problems) {
        const Problem* q = kv.second.get();
        if (q != keep && q->state == PState::Resident && !q->busy && q->pending.empty())
          idle += q->resident;
      }
    const long long after = (long long)S.budget - (long long)(S.committed - S.running_mem) +
                            (long long)idle;
    if ((long long)need <= after) ahead = need;
  };
  for (const Cand& c : cands) {
    Problem& p = *c.p;
    if (c.kind == Work::Build) {
      if (!evict_for(S, p.peak + ahead, &p, fr)) {
        hold(p.peak, &p);
        continue;
      }
      w.kind = Work::Build;
      w.pr = &p;
      w.mem = p.peak;
      w.rebuild = p.state == PState::Evicted;
      p.state = PState::Building;
    } else {
      // A solve's memory returns when it ends, a factor's only with a rebuild: while
      // another solve runs, a solve that does not fit waits for it instead of evicting.
      const bool may_evict = S.running_solves == 0;
      auto admit = [&](size_t b) {
        return may_evict ? evict_for(S, b + ahead, &p, fr) : fits(S, b + ahead);
      };
      size_t k = batch_len(p, S.opts.max_batch_rhs);
      int R = 0;
      bool any_s = false;
      size_t need = solve_need(p, k, &R, &any_s);
      if (!admit(need)) {
        // the oldest request alone, else wait
        bool ok = false;
        if (k > 1) {
          k = 1;
          need = solve_need(p, k, &R, &any_s);
          ok = admit(need);
        }
        if (!ok) {
          hold(need, &p);
          continue;
        }
      }
      w.kind = Work::Solve;
      w.pr = &p;
      w.mem = need;
      w.R = R;
      w.any_s = any_s;
      Share mine;
      mine.pr = &p;
      mine.reqs.assign(p.pending.begin(), p.pending.begin() + (long)k);
      w.shares.push_back(std::move(mine));
      if (S.opts.share_problems) {
        // idle resident problems whose queued requests can ride along, oldest first
        std::vector<Problem*> more;
        for (auto& kv : S.problems) {
          Problem* q = kv.second.get();
          if (q != &p && !q->busy && q->state == PState::Resident && !q->pending.empty() &&
              solve_shareable(p.f, q->f))
            more.push_back(q);
        }
        std::stable_sort(more.begin(), more.end(), [](const Problem* a, const Problem* b) {
          return a->pending.front().t_submit < b->pending.front().t_submit;
        });
        if ((int)more.size() > solve_share_max() - 1) more.resize(solve_share_max() - 1);
        if (!more.empty()) {
          std::vector<Share> sh = w.shares;
          for (Problem* q : more) {
            Share x;
            x.pr = q;
            const size_t kq = batch_len(*q, S.opts.max_batch_rhs);
            x.reqs.assign(q->pending.begin(), q->pending.begin() + (long)kq);
            sh.push_back(std::move(x));
          }
          // riding along is opportunistic: it never evicts a factor
          const size_t need2 = shared_need(sh);
          if (fits(S, need2 + ahead)) {
            w.shares = std::move(sh);
            w.mem = need2;
            for (size_t i = 1; i < w.shares.size(); ++i) {
              Problem& q = *w.shares[i].pr;
              q.pending.erase(q.pending.begin(), q.pending.begin() + (long)w.shares[i].reqs.size());
              for (const SolveReq& r : w.shares[i].reqs) {
                w.R += r.nrhs;
                w.any_s = w.any_s || r.s != nullptr;
              }
            }
          }
        }
      }
      p.pending.erase(p.pending.begin(), p.pending.begin() + (long)k);
      for (Share& x : w.shares) {
        x.after_rebuild = x.pr->rebuilt;
        x.pr->rebuilt = false;
        x.pr->busy = true;
      }
    }
    p.busy = true;
    S.committed += w.mem;
    S.running_mem += w.mem;
    S.peak_committed = std::max(S.peak_committed, S.committed);
    ++S.running;
    if (w.kind == Work::Solve) ++S.running_solves;
    S.max_running = std::max(S.max_running, S.running);
    return true;
  }
  // nothing fits; with nothing running nothing will free up: the oldest item fails
  if (!cands.empty() && S.running == 0) {
    Problem& p = *cands.front().p;
    if (cands.front().kind == Work::Build) {
      const bool initial = p.state == PState::Queued;
      p.state = PState::Failed;
      p.fail = HPS_E_NOMEM;
      if (initial)
        complete(S, p, HPS_REQ_BUILD, p.build_req, HPS_E_NOMEM, 0, 0, 0, false, p.build_submit,
                 tnow, tnow);
    } else {
      SolveReq r = p.pending.front();
      p.pending.pop_front();
      complete(S, p, HPS_REQ_SOLVE, r.id, HPS_E_NOMEM, r.nrhs, r.nrhs, 0, false, r.t_submit,
               tnow, tnow);
    }
    progress = true;
  }
  return progress;
}

struct StreamFree {
  void* p = nullptr;
  hipStream_t st = nullptr;
  ~StreamFree() { ws_free(p, st); }
};

// One merged solve: requests' s and t side by side in staging, one solve, u scattered.
// A solve over several problems stages through the shared-solve path.
int run_solve(Problem& p, const Work& w, hipStream_t st, hps_solve_info* info,
              std::string* msg) {
  try {
    const long nl = p.nl1, n = p.n, ni = p.ni, nt = p.nt;
    const int R = w.R;
    const std::vector<SolveReq>& reqs = w.shares[0].reqs;
    if (w.shares.size() > 1) {
      *info = hps_solve_info{};
      solve_parts(parts_of(w.shares), st);
    } else if (reqs.size() == 1) {
      const SolveReq& r = reqs[0];
      solve_on(p.f, r.nrhs, r.s, r.t, r.u, st, info);
    } else {
      const size_t bs = w.any_s ? align256((size_t)R * nl * ni * 16) : 0;
      const size_t bt = align256((size_t)R * nt * 16);
      const size_t bu = align256((size_t)R * nl * n * 16);
      StreamFree stage;
      stage.st = st;
      stage.p = ws_alloc(bs + bt + bu, st);
      char* base = static_cast<char*>(stage.p);
      double* S = w.any_s ? reinterpret_cast<double*>(base) : nullptr;
      double* T = reinterpret_cast<double*>(base + bs);
      double* U = reinterpret_cast<double*>(base + bs + bt);
      long o = 0;
      for (const SolveReq& r : reqs) {
        if (S) {
          if (r.s)
            HPS_HIP(hipMemcpyAsync(S + 2 * o * nl * ni, r.s, (size_t)r.nrhs * nl * ni * 16,
                                   hipMemcpyDeviceToDevice, st));
          else
            fill_zero(S + 2 * o * nl * ni, 2L * r.nrhs * nl * ni, st);
        }
        HPS_HIP(hipMemcpyAsync(T + 2 * o * nt, r.t, (size_t)r.nrhs * nt * 16,
                               hipMemcpyDeviceToDevice, st));
        o += r.nrhs;
      }
      solve_on(p.f, R, S, T, U, st, info);
      o = 0;
      for (const SolveReq& r : reqs) {
        HPS_HIP(hipMemcpyAsync(r.u, U + 2 * o * nl * n, (size_t)r.nrhs * nl * n * 16,
                               hipMemcpyDeviceToDevice, st));
        o += r.nrhs;
      }
    }
    HPS_HIP(hipStreamSynchronize(st));
    return HPS_OK;
  } catch (const Error& e) {
    *msg = e.what();
    (void)hipStreamSynchronize(st);
    return e.code;
  } catch (const std::exception& e) {
    *msg = e.what();
    (void)hipStreamSynchronize(st);
    return HPS_E_DEVICE;
  }
}

void slot_main(hps_server* S, int slot) {
  (void)hipSetDevice(S->device);
  hipStream_t st = S->streams[slot];
  std::unique_lock<std::mutex> lk(S->mu);
  while (!S->stop) {
    Work w;
    std::vector<Freed> fr;
    if (!pick(*S, w, fr, slot >= S->solve_only)) {
      S->cv_work.wait(lk);
      continue;
    }
    lk.unlock();
    for (const Freed& x : fr) {
      hps_free(x.f);
      dev_free(x.c);
    }
    const double t_start = S->now();
    int status = HPS_OK;
    hps_solve_info info{};
    std::string msg;
    hps_factor* built = nullptr;
    size_t built_bytes = 0;
    if (w.kind == Work::Build) {
      // (idle cached buffers, outside the budget, are released by an allocation that
      // fails for want of their memory)
      Problem& p = *w.pr;  // fields read here are fixed while the problem is busy
      hps_opts o = p.opts;
      o.stream = st;
      o.profile = 0;
      status = hps_build(&p.dom, p.p, p.kappa, p.er, p.ei, p.c, &o, &built);
      if (status == HPS_OK) {
        hps_factor_info fi{};
        hps_factor_query(built, &fi);
        built_bytes = (size_t)fi.device_bytes;
      }
    } else if (w.kind == Work::Solve) {
      status = run_solve(*w.pr, w, st, &info, &msg);
    }
    const double t_end = S->now();
    lk.lock();
    if (w.kind != Work::None) {
      Problem& p = *w.pr;
      S->committed -= w.mem;
      S->running_mem -= w.mem;
      --S->running;
      if (w.kind == Work::Solve) --S->running_solves;
      S->nomem_wait = false;  // this item's memory is back
      p.busy = false;
      p.last_use = ++S->lru_clock;
      for (size_t i = 1; i < w.shares.size(); ++i) {
        w.shares[i].pr->busy = false;
        w.shares[i].pr->last_use = S->lru_clock;
      }
      if (w.kind == Work::Build && status == HPS_E_NOMEM && S->running > 0) {
        // device memory ran short beside other running work: build again later
        ++S->retried;
        S->nomem_wait = true;
        p.state = w.rebuild ? PState::Evicted : PState::Queued;
      } else if (w.kind == Work::Build) {
        if (status == HPS_OK) {
          p.f = built;
          p.resident = built_bytes;
          p.state = PState::Resident;
          S->committed += built_bytes;
          S->peak_committed = std::max(S->peak_committed, S->committed);
          p.rebuilt = w.rebuild;
          if (w.rebuild) ++S->rebuilds;
          else ++S->builds;
        } else {
          p.state = PState::Failed;
          p.fail = status;
        }
        if (!w.rebuild)
          complete(*S, p, HPS_REQ_BUILD, p.build_req, status, 0, 0, 0, false, p.build_submit,
                   t_start, t_end);
      } else if (status == HPS_E_NOMEM && S->running > 0) {
        // device memory ran short beside other running work (memory outside the
        // budget: another process, fragmentation): the requests go back to the front
        // of their queues and are retried once memory frees up
        ++S->retried;
        S->nomem_wait = true;
        for (auto it = w.shares.rbegin(); it != w.shares.rend(); ++it) {
          Problem& q = *it->pr;
          q.pending.insert(q.pending.begin(), it->reqs.begin(), it->reqs.end());
          q.rebuilt = q.rebuilt || it->after_rebuild;
        }
      } else {
        ++S->batches;
        if (w.shares.size() > 1) {
          ++S->shared_batches;
          S->shared_problems += (int64_t)w.shares.size();
        }
        for (const Share& x : w.shares)
          for (const SolveReq& r : x.reqs) {
            complete(*S, *x.pr, HPS_REQ_SOLVE, r.id, status, r.nrhs, w.R, info.iterations,
                     x.after_rebuild, r.t_submit, t_start, t_end);
            if (status == HPS_OK) {
              ++S->solves;
              S->rhs += r.nrhs;
              S->lat_ms.push_back(1e3 * (t_end - r.t_submit));
            }
          }
      }
    }
    S->cv_work.notify_all();
    S->cv_done.notify_all();
  }
}

template <class F>
int guarded(F&& fn) {
  try {
    set_last_error("");
    return fn();
  } catch (const Error& e) {
    set_last_error(e.what());
    return e.code;
  } catch (const std::bad_alloc&) {
    set_last_error("host allocation failed");
    return HPS_E_NOMEM;
  } catch (const std::exception& e) {
    set_last_error(e.what());
    return HPS_E_DEVICE;
  }
}

double percentile(std::vector<double> v, double q) {
  if (v.empty()) return 0.0;
  // nearest rank: the smallest value with at least a fraction q of the samples at or below
  const long rank = (long)std::ceil(q * (double)v.size());
  const size_t k = (size_t)std::min<long>((long)v.size() - 1, std::max<long>(0, rank - 1));
  std::nth_element(v.begin(), v.begin() + (long)k, v.end());
  return v[k];
}

}  // namespace
}  // namespace hps

using namespace hps;

extern "C" {

void hps_server_default_opts(hps_server_opts* o) {
  if (!o) return;
  o->slots = 4;
  o->max_batch_rhs = 64;
  o->max_pending_builds = 64;
  o->evict_idle = 1;
  o->solve_slots = 1;
  o->share_problems = 1;
}

int hps_server_create(size_t hbm_budget, const hps_server_opts* opts, hps_server** out) {
  if (out) *out = nullptr;
  return guarded([&]() -> int {
    if (!out) throw Error(HPS_E_INVALID, "out is NULL");
    hps_server_opts o;
    hps_server_default_opts(&o);
    if (opts) o = *opts;
    if (o.slots < 1 || o.slots > 16) throw Error(HPS_E_INVALID, "slots must be in [1, 16]");
    if (o.max_batch_rhs < 1) throw Error(HPS_E_INVALID, "max_batch_rhs must be >= 1");
    if (o.max_pending_builds < 1) throw Error(HPS_E_INVALID, "max_pending_builds must be >= 1");
    if (o.solve_slots < 0) throw Error(HPS_E_INVALID, "solve_slots must be >= 0");
    std::unique_ptr<hps_server> S(new hps_server);
    S->opts = o;
    S->solve_only = std::min(o.solve_slots, o.slots - 1);
    HPS_HIP(hipGetDevice(&S->device));
    if (hbm_budget == 0) {
      size_t fr = 0, tot = 0;
      HPS_HIP(hipMemGetInfo(&fr, &tot));
      hbm_budget = fr / 10 * 9;
    }
    S->budget = hbm_budget;
    S->t0 = Clock::now();
    for (int i = 0; i < o.slots; ++i) {
      hipStream_t st = nullptr;
      // default priority; the slots do not wait on the null stream
      HPS_HIP(hipStreamCreateWithFlags(&st, hipStreamNonBlocking));
      S->streams.push_back(st);
    }
    hps_server* raw = S.get();
    for (int i = 0; i < o.slots; ++i) S->threads.emplace_back(slot_main, raw, i);
    *out = S.release();
    return HPS_OK;
  });
}

int hps_server_submit_build(hps_server* S, const hps_domain* dom, int32_t p, double kappa,
                            double eta_re, double eta_im, const double* c,
                            const hps_opts* opts, uint64_t* problem, uint64_t* req) {
  return guarded([&]() -> int {
    if (!S || !problem || !req) throw Error(HPS_E_INVALID, "NULL argument");
    int64_t peak = 0, res = 0;
    if (int rc = hps_estimate_bytes(dom, p, opts, &peak, &res)) return rc;
    if (!c) throw Error(HPS_E_INVALID, "c_interior is NULL");
    if (!std::isfinite(kappa) || kappa < 0) throw Error(HPS_E_INVALID, "kappa must be finite, >= 0");
    if (!std::isfinite(eta_re) || !std::isfinite(eta_im) || eta_re == 0.0)
      throw Error(HPS_E_INVALID, "eta must be finite with Re(eta) != 0");
    auto P = std::make_unique<Problem>();
    P->dom = *dom;
    P->p = p;
    P->kappa = kappa; P->er = eta_re; P->ei = eta_im;
    if (opts) P->opts = *opts; else hps_default_opts(&P->opts);
    P->opts.stream = nullptr;
    P->opts.profile = 0;
    P->nl1 = (long)dom->nx * dom->ny;
    P->n = (long)p * p - 4;
    P->ni = (long)(p - 2) * (p - 2);
    P->nt = 2L * (dom->nx + dom->ny) * (p - 2);
    P->peak = (size_t)peak;
    P->c_bytes = (size_t)P->nl1 * P->ni * sizeof(double);
    {
      std::lock_guard<std::mutex> lk(S->mu);
      int queued = 0;
      for (auto& kv : S->problems) queued += kv.second->state == PState::Queued;
      if (P->peak + P->c_bytes > S->budget || queued >= S->opts.max_pending_builds) {
        ++S->rejected;
        throw Error(HPS_E_BUSY, P->peak + P->c_bytes > S->budget
                                    ? "build needs " + std::to_string(P->peak) +
                                          " bytes, more than the server's budget"
                                    : "too many builds queued");
      }
    }
    HPS_HIP(hipSetDevice(S->device));
    P->c = static_cast<double*>(dev_alloc(P->c_bytes));
    if (hipMemcpy(P->c, c, P->c_bytes, hipMemcpyDeviceToDevice) != hipSuccess) {
      (void)hipGetLastError();
      dev_free(P->c);
      P->c = nullptr;
      throw Error(HPS_E_DEVICE, "copy of c failed");
    }
    {
      std::lock_guard<std::mutex> lk(S->mu);
      P->id = S->next_id++;
      P->build_req = S->next_id++;
      P->build_submit = S->now();
      if (S->first_submit < 0) S->first_submit = P->build_submit;
      S->committed += P->c_bytes;
      S->peak_committed = std::max(S->peak_committed, S->committed);
      *problem = P->id;
      *req = P->build_req;
      S->problems[P->id] = std::move(P);
    }
    S->cv_work.notify_all();
    return HPS_OK;
  });
}

int hps_server_submit_solve(hps_server* S, uint64_t problem, int32_t nrhs, const double* s,
                            const double* t, double* u, uint64_t* req) {
  return guarded([&]() -> int {
    if (!S || !req) throw Error(HPS_E_INVALID, "NULL argument");
    if (!t || !u) throw Error(HPS_E_INVALID, "t and u must be non-NULL");
    if (nrhs < 1) throw Error(HPS_E_INVALID, "nrhs must be >= 1");
    {
      std::lock_guard<std::mutex> lk(S->mu);
      auto it = S->problems.find(problem);
      if (it == S->problems.end() || it->second->released)
        throw Error(HPS_E_INVALID, "unknown or released problem");
      Problem& p = *it->second;
      if (p.state == PState::Failed)
        throw Error(p.fail, "the problem's build failed");
      SolveReq r;
      r.id = S->next_id++;
      r.nrhs = nrhs;
      r.s = s; r.t = t; r.u = u;
      r.t_submit = S->now();
      if (S->first_submit < 0) S->first_submit = r.t_submit;
      p.pending.push_back(r);
      *req = r.id;
    }
    S->cv_work.notify_all();
    return HPS_OK;
  });
}

int hps_server_release(hps_server* S, uint64_t problem) {
  return guarded([&]() -> int {
    if (!S) throw Error(HPS_E_INVALID, "server is NULL");
    {
      std::lock_guard<std::mutex> lk(S->mu);
      auto it = S->problems.find(problem);
      if (it == S->problems.end() || it->second->released)
        throw Error(HPS_E_INVALID, "unknown or released problem");
      it->second->released = true;
    }
    S->cv_work.notify_all();
    return HPS_OK;
  });
}

int hps_server_poll(hps_server* S, hps_completion* out, int32_t max, int32_t timeout_ms,
                    int32_t* n) {
  if (n) *n = 0;
  return guarded([&]() -> int {
    if (!S || !n || (!out && max > 0)) throw Error(HPS_E_INVALID, "NULL argument");
    if (max < 0 || timeout_ms < 0) throw Error(HPS_E_INVALID, "max and timeout_ms must be >= 0");
    std::unique_lock<std::mutex> lk(S->mu);
    if (S->done.empty() && timeout_ms > 0)
      S->cv_done.wait_for(lk, std::chrono::milliseconds(timeout_ms),
                          [&] { return !S->done.empty() || S->stop; });
    int k = 0;
    while (k < max && !S->done.empty()) {
      out[k++] = S->done.front();
      S->done.pop_front();
    }
    *n = k;
    return HPS_OK;
  });
}

int hps_server_stats(hps_server* S, hps_stats* st) {
  return guarded([&]() -> int {
    if (!S || !st) throw Error(HPS_E_INVALID, "NULL argument");
    std::lock_guard<std::mutex> lk(S->mu);
    hps_stats z{};
    z.builds = S->builds; z.rebuilds = S->rebuilds; z.evictions = S->evictions;
    z.solves = S->solves; z.rhs = S->rhs; z.batches = S->batches;
    z.rejected = S->rejected; z.failed = S->failed;
    int resident = 0, pending = (int)S->done.size();
    for (auto& kv : S->problems) {
      const Problem& p = *kv.second;
      resident += p.state == PState::Resident;
      pending += (int)p.pending.size() + (p.state == PState::Queued ? 1 : 0);
    }
    z.resident = resident;
    z.pending = pending;
    z.max_concurrent = S->max_running;
    z.slots = S->opts.slots;
    z.p50_ms = percentile(S->lat_ms, 0.50);
    z.p99_ms = percentile(S->lat_ms, 0.99);
    z.max_ms = S->lat_ms.empty() ? 0.0 : *std::max_element(S->lat_ms.begin(), S->lat_ms.end());
    z.wall_s = S->first_submit >= 0 ? std::max(0.0, S->last_end - S->first_submit) : 0.0;
    z.rhs_per_s = z.wall_s > 0 ? S->rhs / z.wall_s : 0.0;
    z.solves_per_s = z.wall_s > 0 ? S->solves / z.wall_s : 0.0;
    z.budget_bytes = (int64_t)S->budget;
    z.committed_bytes = (int64_t)S->committed;
    z.peak_committed_bytes = (int64_t)S->peak_committed;
    z.shared_batches = S->shared_batches;
    z.shared_problems = S->shared_problems;
    z.retried = S->retried;
    *st = z;
    return HPS_OK;
  });
}

void hps_server_destroy(hps_server* S) {
  if (!S) return;
  {
    std::lock_guard<std::mutex> lk(S->mu);
    S->stop = true;
  }
  S->cv_work.notify_all();
  S->cv_done.notify_all();
  for (auto& th : S->threads) th.join();
  (void)hipSetDevice(S->device);
  for (auto& kv : S->problems) {
    hps_free(kv.second->f);
    dev_free(kv.second->c);
  }
  for (hipStream_t st : S->streams) (void)hipStreamDestroy(st);
  delete S;
}

}  // extern "C"
