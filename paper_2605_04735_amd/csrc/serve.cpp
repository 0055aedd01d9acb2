// Continuous-batching server for compliance + sensitivity requests.
//
// A request is one design (grid, boundary conditions, densities) to be solved
// to rtol with float32 inner CG and float64 refinement, then reduced to its
// compliance and sensitivity.  The server thread
//   - admits queued requests in arrival order while a slot is free and the
//     request's device footprint fits a first-fit arena carved from one
//     allocation of the HBM budget;
//   - keeps every admitted design's densities, moduli, preconditioner,
//     float64 solution and float32 CG state resident in its arena block;
//   - advances all designs that are in an inner CG solve together: one
//     launch of the batched product kernel and one of the batched update
//     kernel per iteration cover every such design (blocks map to designs
//     through a table), several iterations per tick;
//   - between ticks runs each design's float64 residual, inner-solve start,
//     solution update and final compliance/sensitivity, and retires finished
//     designs, freeing their slot and memory for the queue.
// A design's arithmetic does not depend on which others share the batch: its
// blocks, partial sums and reductions are its own, in a fixed order.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <atomic>
#include <chrono>
#include <cmath>
#include <condition_variable>
#include <cstdlib>
#include <cstring>
#include <deque>
#include <map>
#include <mutex>
#include <string>
#include <thread>
#include <vector>

#include "common.h"
#include "refine_rule.h"
#include "to.h"

using namespace topo;

namespace {

double now_ms() {
  using namespace std::chrono;
  return duration<double, std::milli>(steady_clock::now().time_since_epoch()).count();
}

// First-fit allocator over one device block; offsets are 256-byte aligned.
struct Arena {
  size_t size = 0;
  std::map<size_t, size_t> free_;  // offset -> bytes
  void init(size_t bytes) {
    size = bytes;
    free_.clear();
    free_[0] = bytes;
  }
  bool alloc(size_t bytes, size_t *off) {
    bytes = (bytes + 255) & ~size_t(255);
    for (auto it = free_.begin(); it != free_.end(); ++it) {
      if (it->second >= bytes) {
        *off = it->first;
        const size_t rest = it->second - bytes;
        const size_t at = it->first + bytes;
        free_.erase(it);
        if (rest) free_[at] = rest;
        return true;
      }
    }
    return false;
  }
  void release(size_t off, size_t bytes) {
    bytes = (bytes + 255) & ~size_t(255);
    auto it = free_.emplace(off, bytes).first;
    auto nx = std::next(it);
    if (nx != free_.end() && it->first + it->second == nx->first) {
      it->second += nx->second;
      free_.erase(nx);
    }
    if (it != free_.begin()) {
      auto pv = std::prev(it);
      if (pv->first + pv->second == it->first) {
        pv->second += it->second;
        free_.erase(it);
      }
    }
  }
};

struct Request {
  to_problem prob;
  std::vector<double> x;
  double *h_dc = nullptr;
  uint64_t tag = 0;
  double t_arrival = 0.0;
};

struct Done {
  uint64_t tag;
  double c;
  int32_t status;
  double latency_ms;
};

enum SlotState { FREE = 0, RESID, INNER, SENS };

struct Slot {
  int state = FREE;
  Request req;
  Grid g{};
  int kz = 2, tx = 1, ty = 1, nb_mv = 1, nb_up = 1;
  size_t off = 0, bytes = 0;
  double *x = nullptr, *E64 = nullptr, *dinv64 = nullptr, *f = nullptr, *u = nullptr,
         *r64 = nullptr, *dc = nullptr, *cgp = nullptr, *part = nullptr;
  float *E32 = nullptr, *dinv32 = nullptr, *v[6] = {};
  uint8_t *mask = nullptr;
  double *scal = nullptr;  // into the server-wide arrays
  int *flags = nullptr;
  double *h_stage = nullptr;  // pinned staging (x in, dc out)
  size_t stage_cap = 0;
  double fnorm = -1.0;
  int outer = 0, inner_total = 0;
  StagnationRule stall;  // float64 residual history (attainable accuracy)
  int32_t fail = TO_OK;
};

// Device footprint of one request (and the carve of its arena block).
size_t carve_slot(const Grid &g, char *base, Slot *s) {
  size_t off = 0;
  auto take = [&](size_t bytes) {
    off = (off + 255) & ~size_t(255);
    const size_t at = off;
    off += bytes;
    return at;
  };
  const size_t ox = take(g.nel * 8), oE64 = take(g.nel * 8), oE32 = take(g.nel * 4);
  const size_t oD64 = take(g.nn * 8), oD32 = take(g.nn * 4), oM = take(g.nn);
  const size_t of = take(g.ndof * 8), ou = take(g.ndof * 8), orr = take(g.ndof * 8);
  const size_t odc = take(g.nel * 8);
  size_t ov[6];
  for (int i = 0; i < 6; ++i) ov[i] = take(g.ndof * 4);
  const size_t ocgp = take((size_t)CGP_SIZE * 8), opart = take((size_t)2 * MAXB * 8);
  const size_t total = (off + 255) & ~size_t(255);
  if (base && s) {
    s->x = (double *)(base + ox);
    s->E64 = (double *)(base + oE64);
    s->E32 = (float *)(base + oE32);
    s->dinv64 = (double *)(base + oD64);
    s->dinv32 = (float *)(base + oD32);
    s->mask = (uint8_t *)(base + oM);
    s->f = (double *)(base + of);
    s->u = (double *)(base + ou);
    s->r64 = (double *)(base + orr);
    s->dc = (double *)(base + odc);
    for (int i = 0; i < 6; ++i) s->v[i] = (float *)(base + ov[i]);
    s->cgp = (double *)(base + ocgp);
    s->part = (double *)(base + opart);
  }
  return total;
}

Coef<float> coef32(double nu, double h) {
  const double lam = nu / ((1.0 + nu) * (1.0 - 2.0 * nu));
  const double mu = 1.0 / (2.0 * (1.0 + nu));
  const double F = h / 32.0;
  Coef<float> k;
  k.L2 = (float)(2.0 * lam * F);
  k.M4 = (float)(4.0 * mu * F);
  k.M2 = (float)(2.0 * mu * F);
  k.L2_3 = (float)(2.0 * lam * F / 3.0);
  k.M2_3 = (float)(2.0 * mu * F / 3.0);
  k.B9 = (float)((2.0 * lam + 8.0 * mu) / 9.0 * F);
  return k;
}

Coef<double> coef64(double nu, double h) {
  const double lam = nu / ((1.0 + nu) * (1.0 - 2.0 * nu));
  const double mu = 1.0 / (2.0 * (1.0 + nu));
  const double F = h / 32.0;
  Coef<double> k;
  k.L2 = 2.0 * lam * F;
  k.M4 = 4.0 * mu * F;
  k.M2 = 2.0 * mu * F;
  k.L2_3 = 2.0 * lam * F / 3.0;
  k.M2_3 = 2.0 * mu * F / 3.0;
  k.B9 = (2.0 * lam + 8.0 * mu) / 9.0 * F;
  return k;
}

}  // namespace

struct to_server {
  hipStream_t stream = nullptr;
  int device = 0;
  size_t budget = 0;
  int max_slots = 0;
  char *arena_base = nullptr;
  Arena arena;
  std::vector<Slot> slots;
  // server-wide device scalars/flags (one row per slot) and pinned mirrors
  double *d_scal = nullptr, *h_scal = nullptr;
  int *d_flags = nullptr, *h_flags = nullptr;
  // batch tables
  CgDesc<float> *d_desc = nullptr, *h_desc = nullptr;
  BlockEntry *d_bmv = nullptr, *d_bup = nullptr, *h_bmv = nullptr, *h_bup = nullptr;
  size_t bmap_cap = 0;
  int nb_mv = 0, nb_up = 0;
  bool batch_dirty = true;
  int parity = 0;
  // the chunk of batched iterations as a graph per starting parity, built
  // once a batch has stayed unchanged for a tick and dropped when it changes
  bool use_graph = true;
  int stable_ticks = 0;
  hipGraphExec_t graph[2] = {nullptr, nullptr};
  double eta = 1e-4;
  int chunk = 32;
  // queues
  std::mutex mu;
  std::condition_variable cv;
  std::deque<Request> queue;
  std::vector<Done> done;
  std::atomic<bool> stop{false};
  std::atomic<int> live{0};
  std::atomic<long long> ticks{0};
  std::atomic<int> hip_error{0};
  std::thread th;
  std::string err;
};

namespace {

thread_local std::string g_srv_error;

to_status srv_fail(to_server *s, to_status st, const std::string &m) {
  g_srv_error = m;
  if (s) {
    std::lock_guard<std::mutex> lk(s->mu);
    s->err = m;
  }
  return st;
}

bool check(to_server *s, hipError_t e) {
  if (e != hipSuccess) {
    s->hip_error = (int)e;
    return false;
  }
  return true;
}

void complete(to_server *s, Slot &sl, int32_t status, double c) {
  const double t = now_ms();
  if (status == TO_OK && sl.req.h_dc)
    std::memcpy(sl.req.h_dc, sl.h_stage, sl.g.nel * sizeof(double));
  {
    std::lock_guard<std::mutex> lk(s->mu);
    s->done.push_back(Done{sl.req.tag, c, status, t - sl.req.t_arrival});
    s->arena.release(sl.off, sl.bytes);
  }
  sl.state = FREE;
  sl.req = Request();
  s->live--;
  s->batch_dirty = true;
}

// Residual r = f - K u (float64) and its norm into the slot's scalars.
bool launch_resid(to_server *s, Slot &sl) {
  MvArgs<double> a{};
  a.nelx = sl.g.nelx;
  a.nely = sl.g.nely;
  a.nelz = sl.g.nelz;
  a.kz = sl.kz;
  a.E = sl.E64;
  a.in = sl.u;
  a.out = sl.r64;
  a.f = sl.f;
  a.mask = sl.mask;
  a.part = sl.part;
  a.k = coef64(sl.req.prob.nu, sl.req.prob.h);
  int nb = 0;
  return check(s, launch_matvec<double, MV_RESID>(a, &nb, s->stream)) &&
         check(s, launch_finish_sum(sl.part, nb, 0, sl.scal, S_NORM2, s->stream)) &&
         check(s, launch_set_scale(sl.scal, s->stream));
}

bool admit(to_server *s, Slot &sl, Request &&rq) {
  sl.req = std::move(rq);
  const to_problem &p = sl.req.prob;
  sl.g.nelx = p.nelx;
  sl.g.nely = p.nely;
  sl.g.nelz = p.nelz;
  sl.g.nel = (size_t)p.nelx * p.nely * p.nelz;
  sl.g.nn = (size_t)(p.nelx + 1) * (p.nely + 1) * (p.nelz + 1);
  sl.g.ndof = 3 * sl.g.nn;
  sl.kz = matvec_kz(sl.g, false);  // float32 inner solves
  sl.tx = (p.nelx + 1 + TNX - 1) / TNX;
  sl.ty = (p.nely + 1 + TNY - 1) / TNY;
  sl.nb_mv = matvec_blocks(sl.g, sl.kz);
  sl.nb_up = update_blocks(sl.g.nn);
  carve_slot(sl.g, s->arena_base + sl.off, &sl);
  sl.fnorm = -1.0;
  sl.outer = 0;
  sl.inner_total = 0;
  sl.stall = StagnationRule{};
  sl.fail = TO_OK;
  if (sl.stage_cap < sl.g.nel) {
    if (sl.h_stage) hipHostFree(sl.h_stage);
    sl.h_stage = nullptr;
    sl.stage_cap = 0;
    if (!check(s, hipHostMalloc((void **)&sl.h_stage, sl.g.nel * sizeof(double),
                                hipHostMallocDefault)))
      return false;
    sl.stage_cap = sl.g.nel;
  }
  std::memcpy(sl.h_stage, sl.req.x.data(), sl.g.nel * sizeof(double));
  hipStream_t st = s->stream;
  int nb = 0;
  const double kd = p.h * (p.nu / ((1 + p.nu) * (1 - 2 * p.nu)) + 4.0 / (2.0 * (1 + p.nu))) / 9.0;
  bool ok = check(s, hipMemcpyAsync(sl.x, sl.h_stage, sl.g.nel * sizeof(double),
                                    hipMemcpyHostToDevice, st)) &&
            check(s, launch_fill(sl.flags, F_COUNT * sizeof(int), st)) &&
            check(s, launch_mask_builtin(sl.g, p.bc, sl.mask, st)) &&
            check(s, launch_load_builtin(sl.g, p.bc, p.load_total, sl.mask, sl.f, st)) &&
            check(s, launch_dot(sl.f, sl.f, sl.g.ndof, sl.part, &nb, st)) &&
            check(s, launch_finish_sum(sl.part, nb, 0, sl.scal, S_TMP, st)) &&
            check(s, launch_modulus(sl.g, sl.x, p.E0, p.Emin, p.penal, sl.E64, sl.E32, sl.flags,
                                    st)) &&
            check(s, launch_diag(sl.g, sl.E64, kd, sl.mask, sl.dinv64, sl.dinv32, st)) &&
            check(s, launch_fill(sl.u, sl.g.ndof * sizeof(double), st)) && launch_resid(s, sl);
  sl.state = RESID;
  return ok;
}

CgDesc<float> make_desc(const Slot &sl) {
  CgDesc<float> d{};
  d.nelx = sl.g.nelx;
  d.nely = sl.g.nely;
  d.nelz = sl.g.nelz;
  d.kz = sl.kz;
  d.tx = sl.tx;
  d.ty = sl.ty;
  d.nb_mv = sl.nb_mv;
  d.nb_up = sl.nb_up;
  d.nn = (long long)sl.g.nn;
  d.k = coef32(sl.req.prob.nu, sl.req.prob.h);
  d.E = sl.E32;
  d.dinv = sl.dinv32;
  d.mask = sl.mask;
  d.x = sl.v[0];
  d.zfuse = cg_zfuse(sl.g);
  d.r = sl.v[1];
  d.z = sl.v[2];
  d.p[0] = sl.v[3];
  d.p[1] = sl.v[4];
  d.q = sl.v[5];
  d.np = 2;
  d.xgroup = 1;  // x advanced by the parity-0 update, two steps at a time
  d.cgp = sl.cgp;
  d.scal = sl.scal;
  d.flags = sl.flags;
  return d;
}

// Rebuilds the batch tables for the slots in INNER state: descriptors, and
// per kernel a block -> (design, local block, design's partials, scalars,
// flags, partial count) map.  Each design's blocks are padded to a multiple
// of 8 so that its tile ranges stay XCD-contiguous; padding entries name
// design -1 (no work).
bool rebuild_batch(to_server *s) {
  int nd = 0;
  std::vector<BlockEntry> bmv, bup;
  for (size_t i = 0; i < s->slots.size(); ++i) {
    Slot &sl = s->slots[i];
    if (sl.state != INNER) continue;
    s->h_desc[nd] = make_desc(sl);
    const int pad_mv = (sl.nb_mv + NXCD - 1) / NXCD * NXCD;
    for (int b = 0; b < pad_mv; ++b)
      bmv.push_back(b < sl.nb_mv
                        ? BlockEntry{sl.cgp, sl.scal, sl.flags, nd, xcd_local(b, sl.nb_mv), sl.nb_up, 0}
                        : BlockEntry{sl.cgp, sl.scal, sl.flags, -1, 0, 0, 0});
    for (int b = 0; b < sl.nb_up; ++b)
      bup.push_back(BlockEntry{sl.cgp, sl.scal, sl.flags, nd, b, sl.nb_mv, 0});
    ++nd;
  }
  s->nb_mv = (int)bmv.size();
  s->nb_up = (int)bup.size();
  if ((size_t)std::max(s->nb_mv, s->nb_up) > s->bmap_cap) return false;
  std::copy(bmv.begin(), bmv.end(), s->h_bmv);
  std::copy(bup.begin(), bup.end(), s->h_bup);
  hipStream_t st = s->stream;
  bool ok = true;
  if (nd) {
    ok = check(s, hipMemcpyAsync(s->d_desc, s->h_desc, nd * sizeof(CgDesc<float>),
                                 hipMemcpyHostToDevice, st)) &&
         check(s, hipMemcpyAsync(s->d_bmv, s->h_bmv, s->nb_mv * sizeof(BlockEntry),
                                 hipMemcpyHostToDevice, st)) &&
         check(s, hipMemcpyAsync(s->d_bup, s->h_bup, s->nb_up * sizeof(BlockEntry),
                                 hipMemcpyHostToDevice, st));
  }
  s->batch_dirty = false;
  return ok;
}

void server_loop(to_server *s) {
  hipSetDevice(s->device);
  while (!s->stop) {
    // ---- admission (arrival order; a request waits for memory or a slot)
    {
      std::unique_lock<std::mutex> lk(s->mu);
      if (s->queue.empty() && s->live == 0) {
        s->cv.wait_for(lk, std::chrono::milliseconds(2));
        if (s->stop) break;
      }
      while (!s->queue.empty()) {
        Request &rq = s->queue.front();
        Grid g;
        g.nelx = rq.prob.nelx;
        g.nely = rq.prob.nely;
        g.nelz = rq.prob.nelz;
        g.nel = (size_t)g.nelx * g.nely * g.nelz;
        g.nn = (size_t)(g.nelx + 1) * (g.nely + 1) * (g.nelz + 1);
        g.ndof = 3 * g.nn;
        const size_t need = carve_slot(g, nullptr, nullptr);
        int free_slot = -1;
        for (size_t i = 0; i < s->slots.size(); ++i)
          if (s->slots[i].state == FREE) {
            free_slot = (int)i;
            break;
          }
        size_t off = 0;
        if (free_slot < 0 || !s->arena.alloc(need, &off)) break;
        Slot &sl = s->slots[free_slot];
        sl.off = off;
        sl.bytes = need;
        Request r = std::move(rq);
        s->live++;  // counted before leaving the queue, so the server never looks idle
        s->queue.pop_front();
        lk.unlock();
        admit(s, sl, std::move(r));
        lk.lock();
      }
    }
    if (s->hip_error) break;
    if (s->live == 0) continue;
    // ---- batched inner CG iterations for every design in an inner solve
    if (s->batch_dirty) {
      for (hipGraphExec_t &g : s->graph)
        if (g) {
          hipGraphExecDestroy(g);  // no replay is queued: the last tick synchronised
          g = nullptr;
        }
      s->stable_ticks = 0;
      if (!rebuild_batch(s)) break;
    } else {
      s->stable_ticks++;
    }
    if (s->nb_mv > 0) {
      hipGraphExec_t &gx = s->graph[s->parity];
      if (s->use_graph && s->stable_ticks >= 1 && s->chunk % 2 == 0) {
        if (!gx && !check(s, build_cg_graph_batched<float>(s->d_desc, s->d_bmv, s->nb_mv, s->d_bup,
                                                           s->nb_up, s->parity, s->chunk, &gx)))
          break;
        if (!check(s, hipGraphLaunch(gx, s->stream))) break;  // an even chunk keeps the parity
      } else {
        for (int it = 0; it < s->chunk; ++it) {
          if (!check(s, launch_cg_matvec<float>(s->d_desc, s->d_bmv, s->nb_mv, s->parity,
                                                s->stream)) ||
              !check(s, launch_cg_update<float>(s->d_desc, s->d_bup, s->nb_up, s->parity,
                                                s->stream)))
            break;
          s->parity ^= 1;
        }
      }
    }
    // ---- read back every slot's scalars and flags
    const size_t ns = s->slots.size();
    if (!check(s, hipMemcpyAsync(s->h_scal, s->d_scal, ns * S_COUNT * sizeof(double),
                                 hipMemcpyDeviceToHost, s->stream)) ||
        !check(s, hipMemcpyAsync(s->h_flags, s->d_flags, ns * F_COUNT * sizeof(int),
                                 hipMemcpyDeviceToHost, s->stream)) ||
        !check(s, hipStreamSynchronize(s->stream)))
      break;
    s->ticks++;
    // ---- per-design outer steps
    for (size_t i = 0; i < ns; ++i) {
      Slot &sl = s->slots[i];
      if (sl.state == FREE) continue;
      const double *sc = s->h_scal + i * S_COUNT;
      const int *fl = s->h_flags + i * F_COUNT;
      const to_problem &p = sl.req.prob;
      if (sl.state == SENS) {
        complete(s, sl, sl.fail, sc[S_C]);
        continue;
      }
      if (sl.state == INNER) {
        if (!fl[F_DONE]) continue;
        sl.inner_total += fl[F_ITERS];
        sl.outer++;
        if (fl[F_STATUS] == 1 && fl[F_ITERS] == 0) sl.fail = TO_E_SINGULAR;
        if (fl[F_STATUS] == 2) sl.fail = TO_E_NONFINITE;
        {
          float *const ps[2] = {sl.v[3], sl.v[4]};  // the steps since the last grouped update
          check(s, launch_axpy_out<float>(sl.g, sl.u, sl.v[0], sl.scal, s->stream, 2, 1, ps,
                                          sl.flags));
        }
        launch_resid(s, sl);
        sl.state = RESID;
        s->batch_dirty = true;
        continue;
      }
      // RESID: the residual of the current u is in the scalars
      if (sl.fnorm < 0.0) {
        sl.fnorm = std::sqrt(sc[S_TMP]);
        if (fl[F_BADX] & 2) sl.fail = TO_E_NONFINITE;
        else if (fl[F_BADX] & 1) sl.fail = TO_E_INVALID;
      }
      const double rel = sl.fnorm > 0.0 ? std::sqrt(sc[S_NORM2]) / sl.fnorm : 0.0;
      bool finish = rel <= p.rtol || sl.fail != TO_OK;
      if (!finish && (!std::isfinite(rel))) {
        sl.fail = TO_E_NONFINITE;
        finish = true;
      }
      if (!finish && (sl.inner_total >= p.max_iters || sl.outer >= 200)) {
        sl.fail = TO_E_NOCONV;
        finish = true;
      }
      // attainable accuracy: four refinement passes that have not halved the
      // float64 residual end the request (same rule as the one-design solve)
      if (!finish) {
        if (sl.stall.record(rel)) {
          sl.fail = TO_E_NOCONV;
          finish = true;
        }
      }
      if (finish) {
        int nb = 0;
        check(s, launch_energy_sens(sl.g, sl.x, sl.u, sl.E64, coef64(p.nu, p.h), p.E0, p.Emin,
                                    p.penal, sl.dc, sl.part, &nb, s->stream));
        check(s, launch_dot(sl.f, sl.u, sl.g.ndof, sl.part, &nb, s->stream));
        check(s, launch_finish_sum(sl.part, nb, 0, sl.scal, S_C, s->stream));
        check(s, hipMemcpyAsync(sl.h_stage, sl.dc, sl.g.nel * sizeof(double),
                                hipMemcpyDeviceToHost, s->stream));
        sl.state = SENS;
        continue;
      }
      const double eta = std::max(s->eta, 0.5 * p.rtol / rel);
      const int slot_set = s->parity ^ 1;  // the next batched product runs with s->parity
      check(s, launch_cg_init<float>(sl.g, sl.r64, sl.scal, sl.v[0], sl.v[1], sl.v[2], sl.v[3],
                                     sl.v[4], sl.dinv32, sl.mask, sl.cgp, slot_set, sl.nb_up,
                                     s->stream));
      check(s, launch_finish_init(sl.cgp, sl.nb_up, slot_set, eta * eta,
                                  p.max_iters - sl.inner_total, sl.scal, sl.flags, s->stream,
                                  s->parity));
      sl.state = INNER;
      s->batch_dirty = true;
    }
  }
  if (s->hip_error) {
    // retire everything with the error
    for (auto &sl : s->slots)
      if (sl.state != FREE) complete(s, sl, TO_E_HIP, 0.0);
    std::lock_guard<std::mutex> lk(s->mu);
    for (auto &rq : s->queue) s->done.push_back(Done{rq.tag, 0.0, TO_E_HIP, now_ms() - rq.t_arrival});
    s->queue.clear();
  }
}

}  // namespace

extern "C" {

to_status to_server_create(size_t hbm_budget_bytes, int32_t max_slots, void *stream_unused,
                           to_server **out) {
  (void)stream_unused;
  if (!out) return srv_fail(nullptr, TO_E_INVALID, "out is NULL");
  *out = nullptr;
  if (max_slots < 1 || max_slots > 1024) return srv_fail(nullptr, TO_E_INVALID, "1 <= max_slots <= 1024");
  if (hbm_budget_bytes < (size_t)1 << 20) return srv_fail(nullptr, TO_E_INVALID, "budget < 1 MiB");
  to_server *s = new to_server();
  s->budget = hbm_budget_bytes;
  s->max_slots = max_slots;
  if (const char *e = std::getenv("TOPO_INNER_ETA")) s->eta = std::atof(e);
  if (const char *e = std::getenv("TOPO_CHUNK")) s->chunk = std::max(1, std::atoi(e));
  if (const char *e = std::getenv("TOPO_GRAPH")) s->use_graph = std::atoi(e) != 0;
  s->bmap_cap = (size_t)max_slots * (MAXB + NXCD);
  bool ok = hipGetDevice(&s->device) == hipSuccess &&
            hipStreamCreateWithFlags(&s->stream, hipStreamNonBlocking) == hipSuccess &&
            hipMalloc((void **)&s->arena_base, hbm_budget_bytes) == hipSuccess &&
            hipMalloc((void **)&s->d_scal, (size_t)max_slots * S_COUNT * sizeof(double)) ==
                hipSuccess &&
            hipMalloc((void **)&s->d_flags, (size_t)max_slots * F_COUNT * sizeof(int)) == hipSuccess &&
            hipMalloc((void **)&s->d_desc, (size_t)max_slots * sizeof(CgDesc<float>)) == hipSuccess &&
            hipMalloc((void **)&s->d_bmv, s->bmap_cap * sizeof(BlockEntry)) == hipSuccess &&
            hipMalloc((void **)&s->d_bup, s->bmap_cap * sizeof(BlockEntry)) == hipSuccess &&
            hipHostMalloc((void **)&s->h_scal, (size_t)max_slots * S_COUNT * sizeof(double),
                          hipHostMallocDefault) == hipSuccess &&
            hipHostMalloc((void **)&s->h_flags, (size_t)max_slots * F_COUNT * sizeof(int),
                          hipHostMallocDefault) == hipSuccess &&
            hipHostMalloc((void **)&s->h_desc, (size_t)max_slots * sizeof(CgDesc<float>),
                          hipHostMallocDefault) == hipSuccess &&
            hipHostMalloc((void **)&s->h_bmv, s->bmap_cap * sizeof(BlockEntry), hipHostMallocDefault) ==
                hipSuccess &&
            hipHostMalloc((void **)&s->h_bup, s->bmap_cap * sizeof(BlockEntry), hipHostMallocDefault) ==
                hipSuccess;
  if (ok) {
    ok = launch_fill(s->d_scal, (size_t)max_slots * S_COUNT * sizeof(double), s->stream) ==
             hipSuccess &&
         launch_fill(s->d_flags, (size_t)max_slots * F_COUNT * sizeof(int), s->stream) ==
             hipSuccess &&
         hipStreamSynchronize(s->stream) == hipSuccess;
  }
  if (!ok) {
    to_server_destroy(s);
    return srv_fail(nullptr, TO_E_OOM, "server allocation failed");
  }
  s->arena.init(hbm_budget_bytes);
  s->slots.resize(max_slots);
  for (int i = 0; i < max_slots; ++i) {
    s->slots[i].scal = s->d_scal + (size_t)i * S_COUNT;
    s->slots[i].flags = s->d_flags + (size_t)i * F_COUNT;
  }
  s->th = std::thread(server_loop, s);
  *out = s;
  return TO_OK;
}

to_status to_server_submit(to_server *s, const to_problem *prob, const double *h_x, double *h_dc_out,
                           uint64_t tag) {
  if (!s || !prob || !h_x) return srv_fail(s, TO_E_INVALID, "server, problem and h_x are required");
  size_t ws = 0;
  if (to_workspace_size(prob, &ws) != TO_OK) return srv_fail(s, TO_E_INVALID, to_last_error(nullptr));
  if (prob->bc == TO_BC_CUSTOM) return srv_fail(s, TO_E_INVALID, "serving takes built-in BCs only");
  if (prob->precision != TO_PREC_FP32_REFINE)
    return srv_fail(s, TO_E_INVALID, "serving runs the FP32_REFINE precision");
  Grid g;
  g.nelx = prob->nelx;
  g.nely = prob->nely;
  g.nelz = prob->nelz;
  g.nel = (size_t)g.nelx * g.nely * g.nelz;
  g.nn = (size_t)(g.nelx + 1) * (g.nely + 1) * (g.nelz + 1);
  g.ndof = 3 * g.nn;
  if (matvec_blocks(g, matvec_kz(g, false)) > MAXB)
    return srv_fail(s, TO_E_INVALID, "grid too large for serving");
  if (carve_slot(g, nullptr, nullptr) > s->budget)
    return srv_fail(s, TO_E_OOM, "request footprint exceeds the server's HBM budget");
  Request rq;
  rq.prob = *prob;
  rq.prob.fixed_mask = nullptr;
  rq.prob.load = nullptr;
  rq.x.assign(h_x, h_x + g.nel);
  rq.h_dc = h_dc_out;
  rq.tag = tag;
  rq.t_arrival = now_ms();
  {
    std::lock_guard<std::mutex> lk(s->mu);
    if (s->hip_error) return TO_E_HIP;
    if (s->queue.size() >= 65536) return TO_E_BUSY;
    s->queue.push_back(std::move(rq));
  }
  s->cv.notify_one();
  return TO_OK;
}

to_status to_server_poll(to_server *s, uint64_t *tags, double *c, int32_t *status,
                         double *latency_ms, int32_t cap, int32_t *n) {
  if (!s || !n || cap < 0) return srv_fail(s, TO_E_INVALID, "server and n are required");
  std::lock_guard<std::mutex> lk(s->mu);
  const int take = std::min<int>(cap, (int)s->done.size());
  for (int i = 0; i < take; ++i) {
    if (tags) tags[i] = s->done[i].tag;
    if (c) c[i] = s->done[i].c;
    if (status) status[i] = s->done[i].status;
    if (latency_ms) latency_ms[i] = s->done[i].latency_ms;
  }
  s->done.erase(s->done.begin(), s->done.begin() + take);
  *n = take;
  return s->hip_error ? TO_E_HIP : TO_OK;
}

to_status to_server_wait_idle(to_server *s, double timeout_ms) {
  if (!s) return srv_fail(nullptr, TO_E_INVALID, "server is NULL");
  const double t0 = now_ms();
  for (;;) {
    {
      std::lock_guard<std::mutex> lk(s->mu);
      if (s->queue.empty() && s->live == 0) return s->hip_error ? TO_E_HIP : TO_OK;
      if (s->hip_error) return TO_E_HIP;
    }
    if (now_ms() - t0 > timeout_ms) return TO_E_BUSY;
    std::this_thread::sleep_for(std::chrono::microseconds(200));
  }
}

to_status to_server_stats(to_server *s, int32_t *live, int32_t *queued, int64_t *ticks,
                          size_t *free_bytes) {
  if (!s) return srv_fail(nullptr, TO_E_INVALID, "server is NULL");
  std::lock_guard<std::mutex> lk(s->mu);
  if (live) *live = s->live;
  if (queued) *queued = (int32_t)s->queue.size();
  if (ticks) *ticks = s->ticks;
  if (free_bytes) {
    size_t f = 0;
    for (auto &kv : s->arena.free_) f += kv.second;
    *free_bytes = f;
  }
  return TO_OK;
}

void to_server_destroy(to_server *s) {
  if (!s) return;
  s->stop = true;
  s->cv.notify_all();
  if (s->th.joinable()) s->th.join();
  if (s->stream) hipStreamSynchronize(s->stream);
  for (hipGraphExec_t g : s->graph)
    if (g) hipGraphExecDestroy(g);
  for (auto &sl : s->slots)
    if (sl.h_stage) hipHostFree(sl.h_stage);
  hipFree(s->arena_base);
  hipFree(s->d_scal);
  hipFree(s->d_flags);
  hipFree(s->d_desc);
  hipFree(s->d_bmv);
  hipFree(s->d_bup);
  hipHostFree(s->h_scal);
  hipHostFree(s->h_flags);
  hipHostFree(s->h_desc);
  hipHostFree(s->h_bmv);
  hipHostFree(s->h_bup);
  if (s->stream) hipStreamDestroy(s->stream);
  delete s;
}

const char *to_server_last_error(const to_server *s) {
  if (s) return s->err.c_str();
  return g_srv_error.c_str();
}

}  // extern "C"
