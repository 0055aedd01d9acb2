// C ABI (include/to.h) and the host-side solver driver: Jacobi-PCG with
// float64 outer iterative refinement, compliance/sensitivity, filters and the
// density -> SDF transfer.  Every arithmetic step runs in the HIP kernels; the
// host only validates, sequences launches and polls small device flags.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <climits>
#include <chrono>
#include <cmath>
#include <cstdio>
#include <cstdlib>
#include <cstring>
#include <mutex>
#include <string>
#include <vector>

#include "common.h"
#include "refine_rule.h"
#include "stop_predict.h"
#include "to.h"

using namespace topo;

namespace {

thread_local std::string g_last_error;

constexpr int MAXOFS = 1024;        // filter stencil capacity (rmin <= 6)
constexpr int NCGV = 8;             // inner CG vectors of ndof entries
constexpr double MAX_RMIN = 6.0;

struct Layout {
  size_t off = 0;
  template <typename T>
  size_t take(size_t count) {
    off = (off + 255) & ~size_t(255);
    const size_t at = off;
    off += count * sizeof(T);
    return at;
  }
};

}  // namespace

struct to_ctx {
  to_problem p{};
  Grid g{};
  hipStream_t stream = nullptr;
  int device = 0;
  char *ws = nullptr;
  size_t ws_bytes = 0;
  bool owns_ws = false;

  double *E64 = nullptr, *dinv64 = nullptr, *f = nullptr, *r64 = nullptr;
  float *E32 = nullptr, *dinv32 = nullptr;
  uint8_t *mask = nullptr;
  // inner CG vectors (float64 or float32 inner): x, r, z, p0, p1, q, p2, p3
  double *v64[NCGV] = {};
  float *v32[NCGV] = {};
  double *part = nullptr, *scal = nullptr;
  int *flags = nullptr;
  double *ftmp = nullptr, *fw = nullptr;
  int *fofs = nullptr;
  double *rho_scratch = nullptr;
  int *cnt = nullptr, *toff = nullptr, *bsums = nullptr;

  // batched inner-CG tables for this single design
  CgDesc<float> hd32{};          // CG descriptors, passed by value to the CG kernels
  CgDesc<double> hd64{};
  double *cgp = nullptr;         // block partials of the batched CG kernels
  int nb_mv = 0, nb_up = 0;
  int slot = 0;  // direction slot of the next inner-CG product (partial sets by slot & 1)

  double *tri = nullptr;  // triangles, grown on demand by to_density_to_sdf
  size_t tri_cap = 0;
  double *shp = nullptr;  // 8 nel element contributions, allocated by the first to_shape_rhs

  double *h_scal = nullptr;
  int *h_flags = nullptr;
  // inner-CG chunk reads: two pinned slots (flags, then S_RR and S_TOL2) and
  // their events, so that the next chunk can run while the host reads one
  struct ChunkRead {
    int flags[F_COUNT];
    double rr_tol2[2];
  };
  ChunkRead *h_chunk = nullptr;
  hipEvent_t chunk_ev[2] = {nullptr, nullptr};

  Coef<double> k64{};
  Coef<float> k32{};
  double kd = 0.0;
  double fnorm = 0.0;
  int kz = 4;           // z chunk of the vector-ALU products (float64, residuals)
  // float32 inner products on the matrix cores (the A operand in the
  // workspace), or on the vector ALUs (mA == nullptr)
  const void *mA = nullptr;
  float mscale = 0.f;
  int kz_mf = 4;        // z chunk of the matrix-core products
  double last_rmin = -1.0;
  int nofs = 0;
  double eta = 1e-4;   // inner relative tolerance of the float32 refinement
  int chunk = 32;      // CG iterations queued between host polls
  int last_tri = 0;    // triangles of the last density -> SDF transfer
  bool trace = false;  // TOPO_TRACE=1: print the refinement history to stderr
  // optional HIP-event timing of every CG-mode product launch
  bool prof = false;
  std::vector<hipEvent_t> ev;  // start/stop pairs
  std::vector<int> ev_iter;    // the CG iteration of each pair's product launch
  size_t ev_used = 0;           // events handed out in this inner solve
  size_t ev_done = 0;           // of which read
  size_t ev_mark[2] = {0, 0};   // ev_used after each queued chunk (by chunk slot)
  double prof_ms = 0.0;
  long long prof_count = 0;
  int prof_every = 16;  // in a sampled chunk, bracket one product launch in this many
  // a chunk of CG iterations as one graph launch, per precision and starting
  // direction slot (built on first use); with timing on, one chunk in four runs as
  // separate launches so that product launches can be sampled
  bool use_graph = true;
  long long chunks = 0;
  hipGraphExec_t graph[2][CG_NP_MAX] = {};
  std::string err;
};

namespace {

to_status fail(to_ctx *c, to_status s, const std::string &msg) {
  g_last_error = msg;
  if (c) c->err = msg;
  return s;
}

#define HIPCHK(call)                                                                 \
  do {                                                                               \
    hipError_t e_ = (call);                                                          \
    if (e_ != hipSuccess)                                                            \
      return fail(c, TO_E_HIP, std::string(#call) + ": " + hipGetErrorString(e_));  \
  } while (0)

bool validate_problem(const to_problem *p, std::string *why) {
  if (!p) { *why = "problem is NULL"; return false; }
  if (p->nelx < 1 || p->nely < 1 || p->nelz < 1) { *why = "grid sizes must be >= 1"; return false; }
  // node counts in double: nelx + 1 in int overflows at INT_MAX
  const double NX = double(p->nelx) + 1.0, NY = double(p->nely) + 1.0, NZ = double(p->nelz) + 1.0;
  const double nn = NX * NY * NZ;
  // kernels address a vector with 32-bit byte offsets (2^31 marks a lane
  // outside the grid), so a float64 vector of 3 nn values stays below 2^31 bytes
  if (nn * 24.0 >= 2147483648.0) {
    *why = "grid too large (a float64 vector must stay below 2^31 bytes)";
    return false;
  }
  // the product keeps one partial sum per block: its x-y tiles must fit
  const double tiles =
      std::ceil(NX / double(TNX)) * std::ceil(NY / double(TNY));
  if (tiles > MAXB) { *why = "grid too wide in x and y for the product's block bound"; return false; }
  if (!(p->h > 0) || !std::isfinite(p->h)) { *why = "h must be > 0"; return false; }
  if (!(p->E0 > 0) || !std::isfinite(p->E0)) { *why = "E0 must be > 0"; return false; }
  if (!(p->Emin >= 0) || !(p->Emin < p->E0)) { *why = "need 0 <= Emin < E0"; return false; }
  if (!(p->nu > -1.0 && p->nu < 0.5)) { *why = "need -1 < nu < 0.5"; return false; }
  if (!(p->penal >= 1.0) || !std::isfinite(p->penal)) { *why = "need penal >= 1"; return false; }
  if (p->bc < 0 || p->bc > 4) { *why = "unknown bc"; return false; }
  if (p->bc == TO_BC_CUSTOM && (!p->fixed_mask || !p->load)) {
    *why = "CUSTOM bc needs fixed_mask and load"; return false;
  }
  if (p->bc != TO_BC_CUSTOM && !std::isfinite(p->load_total)) { *why = "bad load_total"; return false; }
  if (p->precision < 0 || p->precision > 2) { *why = "unknown precision"; return false; }
  if (!(p->rtol > 0) || !(p->rtol < 1)) { *why = "need 0 < rtol < 1"; return false; }
  if (p->max_iters < 1) { *why = "max_iters must be >= 1"; return false; }
  return true;
}

Grid make_grid(const to_problem *p) {
  Grid g;
  g.nelx = p->nelx;
  g.nely = p->nely;
  g.nelz = p->nelz;
  g.nel = (size_t)p->nelx * p->nely * p->nelz;
  g.nn = (size_t)(p->nelx + 1) * (p->nely + 1) * (p->nelz + 1);
  g.ndof = 3 * g.nn;
  return g;
}

// Whether the float32 inner products of this problem run on the matrix cores:
// only on request (TOPO_MFMA=1), for a float32 inner CG with float32 z, an
// element matrix exact in bfloat16 for this nu, and tiles within the
// partial-sum bound.  The vector-ALU modal product is the default: measured
// at 256 x 128 x 128 it is twice as fast, and its exact differencing of
// nodal values keeps the float32 operator accurate on elements that carry a
// large rigid translation, where the matrix cores' accumulation does not.
bool mfma_path(const Grid &g, int precision, double nu) {
  if (precision != TO_PREC_FP32_REFINE) return false;
  const char *e = std::getenv("TOPO_MFMA");
  if (!e || std::atoi(e) == 0) return false;
  uint16_t tab[2][64][8];
  float unit = 0.f;
  if (!mfma_operand_table(nu, tab, &unit)) return false;
  const long long tiles = (long long)((g.nelx + MN) / MN) * ((g.nely + MN) / MN);
  return tiles <= MAXB;
}

// Carves (or sizes, when base == nullptr) the workspace.
size_t carve(to_ctx *c, const Grid &g, int precision, double nu, char *base) {
  Layout L;
  const size_t oE64 = L.take<double>(g.nel), oE32 = L.take<float>(g.nel);
  const size_t oD64 = L.take<double>(g.nn), oD32 = L.take<float>(g.nn);
  const size_t oMask = L.take<uint8_t>(g.nn);
  const size_t oF = L.take<double>(g.ndof), oR64 = L.take<double>(g.ndof);
  // float64 keeps four direction slots (x grouped by four), float32 two
  const int ncgv = precision == TO_PREC_FP64 ? NCGV : NCGV - 2;
  size_t ov[NCGV] = {};
  if (precision == TO_PREC_FP64)
    for (int i = 0; i < ncgv; ++i) ov[i] = L.take<double>(g.ndof);
  else
    for (int i = 0; i < ncgv; ++i) ov[i] = L.take<float>(g.ndof);
  const size_t oPart = L.take<double>(2 * (size_t)MAXB);
  const size_t oScal = L.take<double>(S_COUNT);
  const size_t oFlags = L.take<int>(F_COUNT);
  const size_t oFtmp = L.take<double>(g.nel);
  const size_t oFw = L.take<double>(MAXOFS), oFofs = L.take<int>(3 * MAXOFS);
  const size_t oRho = L.take<double>(g.nn);
  const size_t oCnt = L.take<int>(g.nel), oToff = L.take<int>(g.nel);
  const size_t oBs = L.take<int>(g.nel / 1024 + 4);
  const bool mf = mfma_path(g, precision, nu);
  const int nbm = matvec_blocks(g, matvec_kz(g, precision == TO_PREC_FP64, mf), mf);
  const int nbu = update_blocks(g.nn);
  const size_t oCgp = L.take<double>(CGP_SIZE);
  const size_t oMfma = L.take<uint16_t>(2 * 64 * 8);
  const size_t total = (L.off + 255) & ~size_t(255);
  if (base) {
    c->E64 = (double *)(base + oE64);
    c->E32 = (float *)(base + oE32);
    c->dinv64 = (double *)(base + oD64);
    c->dinv32 = (float *)(base + oD32);
    c->mask = (uint8_t *)(base + oMask);
    c->f = (double *)(base + oF);
    c->r64 = (double *)(base + oR64);
    for (int i = 0; i < ncgv; ++i) {
      if (precision == TO_PREC_FP64) c->v64[i] = (double *)(base + ov[i]);
      else c->v32[i] = (float *)(base + ov[i]);
    }
    c->part = (double *)(base + oPart);
    c->scal = (double *)(base + oScal);
    c->flags = (int *)(base + oFlags);
    c->ftmp = (double *)(base + oFtmp);
    c->fw = (double *)(base + oFw);
    c->fofs = (int *)(base + oFofs);
    c->rho_scratch = (double *)(base + oRho);
    c->cnt = (int *)(base + oCnt);
    c->toff = (int *)(base + oToff);
    c->bsums = (int *)(base + oBs);
    c->cgp = (double *)(base + oCgp);
    c->mA = mf ? (const void *)(base + oMfma) : nullptr;
    c->nb_mv = nbm;
    c->nb_up = nbu;
  }
  return total;
}

template <typename T>
Coef<T> make_coef(double nu, double h) {
  const double lam = nu / ((1.0 + nu) * (1.0 - 2.0 * nu));
  const double mu = 1.0 / (2.0 * (1.0 + nu));
  const double F = h / 32.0;
  Coef<T> k;
  k.L2 = (T)(2.0 * lam * F);
  k.M4 = (T)(4.0 * mu * F);
  k.M2 = (T)(2.0 * mu * F);
  k.L2_3 = (T)(2.0 * lam * F / 3.0);
  k.M2_3 = (T)(2.0 * mu * F / 3.0);
  k.B9 = (T)((2.0 * lam + 8.0 * mu) / 9.0 * F);
  return k;
}

double now_ms() {
  using namespace std::chrono;
  return duration<double, std::milli>(steady_clock::now().time_since_epoch()).count();
}

to_status sync_read(to_ctx *c) {
  HIPCHK(hipMemcpyAsync(c->h_scal, c->scal, S_COUNT * sizeof(double), hipMemcpyDeviceToHost,
                        c->stream));
  HIPCHK(hipMemcpyAsync(c->h_flags, c->flags, F_COUNT * sizeof(int), hipMemcpyDeviceToHost,
                        c->stream));
  HIPCHK(hipStreamSynchronize(c->stream));
  return TO_OK;
}

// Accumulates the elapsed times of the event pairs [ev_done, upto), whose
// chunk has completed.  Only launches of iterations below `limit` count: a
// launch at or after the iteration where the CG stopped returned at once.
void prof_collect(to_ctx *c, size_t upto, int limit) {
  for (size_t i = c->ev_done; i + 1 < upto; i += 2) {
    float ms = 0.f;
    if (c->ev_iter[i / 2] < limit && hipEventElapsedTime(&ms, c->ev[i], c->ev[i + 1]) == hipSuccess) {
      c->prof_ms += ms;
      c->prof_count += 1;
    }
  }
  c->ev_done = std::max(c->ev_done, upto);
}

// Hands out the next start/stop event pair (created on first use).  The pair
// is attached to one product dispatch, so the elapsed time is that kernel's
// execution alone, without the latency of separate event packets.  The events
// carry no system-scope fence: with one, the timed dispatch also wrote back
// and invalidated the caches, which made it run about 8 us longer at
// 256x128x128.  They are read only after the chunk's own event (with the
// default fence), recorded later on the same stream, has completed.
hipError_t prof_pair(to_ctx *c, int iter, hipEvent_t *start, hipEvent_t *stop) {
  while (c->ev_used + 2 > c->ev.size()) {
    hipEvent_t e;
    hipError_t r = hipEventCreateWithFlags(&e, hipEventDisableSystemFence);
    if (r != hipSuccess) return r;
    c->ev.push_back(e);
  }
  c->ev_iter.resize(c->ev.size() / 2);
  c->ev_iter[c->ev_used / 2] = iter;
  *start = c->ev[c->ev_used++];
  *stop = c->ev[c->ev_used++];
  return hipSuccess;
}

to_status prepare_moduli(to_ctx *c, const double *d_x, bool check) {
  HIPCHK(launch_fill(c->flags, F_COUNT * sizeof(int), c->stream));
  HIPCHK(launch_modulus(c->g, d_x, c->p.E0, c->p.Emin, c->p.penal, c->E64, c->E32, c->flags,
                        c->stream));
  if (check) {
    to_status s = sync_read(c);
    if (s != TO_OK) return s;
    if (c->h_flags[F_BADX] & 2) return fail(c, TO_E_NONFINITE, "x holds NaN or Inf");
    if (c->h_flags[F_BADX] & 1) return fail(c, TO_E_INVALID, "x outside [0,1]");
  }
  return TO_OK;
}

// Forming z = D r inside the product (instead of storing z in the update and
// reading it back) saves 12 bytes per node and costs 4 plus a multiply per
// staged node: it pays where the CG vectors stream from HBM, not where they
// stay in the last-level cache.  TOPO_CG_ZFUSE=0/1 overrides the choice.
}  // namespace

int topo::cg_zfuse(const Grid &g) {
  if (const char *e = std::getenv("TOPO_CG_ZFUSE")) return std::atoi(e) != 0;
  return g.nn >= ZFUSE_MIN_NODES;
}

namespace {

template <typename T>
CgDesc<T> make_desc(to_ctx *c, T *const v[NCGV], const T *E, const T *dinv, const Coef<T> &k) {
  const Grid &g = c->g;
  CgDesc<T> d{};
  d.nelx = g.nelx;
  d.nely = g.nely;
  d.nelz = g.nelz;
  const bool mf = sizeof(T) == 4 && c->mA;
  d.kz = mf ? c->kz_mf : c->kz;
  d.tx = mf ? (g.nelx + MN) / MN : (g.nelx + 1 + TNX - 1) / TNX;
  d.ty = mf ? (g.nely + MN) / MN : (g.nely + 1 + TNY - 1) / TNY;
  if (mf) {
    d.mA = c->mA;
    d.mscale = c->mscale;
  }
  d.nb_mv = c->nb_mv;
  d.nb_up = c->nb_up;
  d.zbf16 = sizeof(T) == 4 && c->p.precision == TO_PREC_FP32_REFINE_BF16;
  d.zfuse = d.zbf16 ? 0 : cg_zfuse(g);
  d.nn = (long long)g.nn;
  d.k = k;
  d.E = E;
  d.dinv = dinv;
  d.mask = c->mask;
  d.x = v[0];
  d.r = v[1];
  d.z = v[2];
  d.p[0] = v[3];
  d.p[1] = v[4];
  d.p[2] = v[6];
  d.p[3] = v[7];
  d.q = v[5];
  // grouped x unless z is stored in bfloat16, whose update advances x itself:
  // groups of two in float32 (the two direction buffers; four gained no more
  // there), of four in float64 (13% per iteration at 256 x 128 x 128 against
  // 9% for two).  TOPO_XGROUP=0 / 2 / 4 selects x every iteration / groups
  // of two / groups of four.
  d.np = sizeof(T) == 8 ? 4 : 2;
  d.xgroup = !d.zbf16;
  if (const char *e = std::getenv("TOPO_XGROUP")) {
    const int v = std::atoi(e);
    d.xgroup = !d.zbf16 && v != 0;
    d.np = d.xgroup && v == 4 ? 4 : 2;
  }
  if (!v[6] || !v[7]) d.np = 2;  // four slots only where the workspace holds them
  d.cgp = c->cgp;
  d.scal = c->scal;
  d.flags = c->flags;
  return d;
}

// One inner Jacobi-PCG solve of K d = r64 / ||r64|| in precision T: two
// launches per iteration (the product with the direction update, then the
// vector update), each of whose blocks first sums the other kernel's block
// partials in a fixed order.
template <typename T>
to_status inner_pcg(to_ctx *c, T *const v[NCGV], const T *dinv, double eta, int cap, int *iters,
                    int *status) {
  const Grid &g = c->g;
  const CgDesc<T> *hd;
  if constexpr (sizeof(T) == 4) hd = &c->hd32;
  else hd = &c->hd64;
  const int np = hd->np == 4 ? 4 : 2;
  c->slot %= np;
  // the first product runs at direction slot c->slot and reads partial set
  // (slot & 1) ^ 1; every direction slot starts at zero
  const int pset = (c->slot & 1) ^ 1;
  const int zbf = sizeof(T) == 4 && c->p.precision == TO_PREC_FP32_REFINE_BF16;
  HIPCHK(launch_cg_init<T>(g, c->r64, c->scal, v[0], v[1], v[2], v[3], v[4], dinv, c->mask, c->cgp,
                           pset, c->nb_up, c->stream, zbf, np == 4 ? v[6] : nullptr,
                           np == 4 ? v[7] : nullptr));
  HIPCHK(launch_finish_init(c->cgp, c->nb_up, pset, eta * eta, cap, c->scal, c->flags, c->stream,
                            c->slot));
  // Chunks are queued ahead: each is followed by an asynchronous copy of the
  // flags and residual norms into one of two pinned slots and an event, and
  // the host waits for chunk k's copy while chunk k + 1 already runs, so the
  // GPU does not idle during the host's check.  A chunk queued after the CG
  // has stopped does nothing (every launch reads the done flag first), so
  // once the residual's decay over the last chunks predicts the stop within
  // the chunk already queued, no further chunk is queued until that one has
  // been read: a wrong guess costs one host round trip, a right one saves a
  // chunk of launches that return at once.  Timing samples are read chunk by
  // chunk as their chunks complete.
  int ahead = 2;
  int launched = 0, queued = 0, nread = 0;
  double prev_rr = 0.0;
  int prev_iters = -1;
  c->ev_used = c->ev_done = 0;
  *iters = 0;
  *status = 0;
  for (;;) {
    while (queued - nread < ahead && launched < cap) {
      const int n = std::min(c->chunk, cap - launched);
      hipGraphExec_t &gx = c->graph[sizeof(T) == 8][c->slot];
      const bool sample = c->prof && (c->chunks++ % 4 == 0);
      if (c->use_graph && !sample && n == c->chunk && c->chunk % np == 0) {
        if (!gx) HIPCHK(build_cg_graph<T>(*hd, c->slot, c->chunk, &gx));
        HIPCHK(hipGraphLaunch(gx, c->stream));  // a chunk of whole slot cycles keeps the slot
      } else {
        for (int it = 0, k = 0; it < n; ++it) {
          hipEvent_t e0 = nullptr, e1 = nullptr;
          // sampled away from the first launch after a host synchronisation,
          // at positions of both slot parities (the product after a grouped
          // x update and the one after a skipping update differ)
          const int at = c->prof_every / 2 + k * c->prof_every + (k & 1);
          if (sample && it == at) {
            HIPCHK(prof_pair(c, launched + it, &e0, &e1));
            ++k;
          }
          HIPCHK(launch_cg_matvec1<T>(*hd, c->slot, c->stream, e0, e1));
          HIPCHK(launch_cg_update1<T>(*hd, c->slot, c->stream));
          c->slot = (c->slot + 1) % np;
        }
      }
      launched += n;
      to_ctx::ChunkRead &cr = c->h_chunk[queued % 2];
      HIPCHK(hipMemcpyAsync(cr.flags, c->flags, F_COUNT * sizeof(int), hipMemcpyDeviceToHost,
                            c->stream));
      static_assert(S_TOL2 == S_RR + 1, "S_RR and S_TOL2 copied together");
      HIPCHK(hipMemcpyAsync(cr.rr_tol2, c->scal + S_RR, 2 * sizeof(double), hipMemcpyDeviceToHost,
                            c->stream));
      HIPCHK(hipEventRecord(c->chunk_ev[queued % 2], c->stream));
      c->ev_mark[queued % 2] = c->ev_used;
      ++queued;
    }
    if (nread == queued) break;  // every chunk up to the cap has been read
    HIPCHK(hipEventSynchronize(c->chunk_ev[nread % 2]));
    const to_ctx::ChunkRead &cr = c->h_chunk[nread % 2];
    if (c->prof)
      prof_collect(c, c->ev_mark[nread % 2], cr.flags[F_DONE] ? cr.flags[F_ITERS] : INT_MAX);
    ++nread;
    *iters = cr.flags[F_ITERS];
    *status = cr.flags[F_STATUS];
    if (c->trace)
      std::fprintf(stderr, "[topo]   inner chunk %d iters %d done %d status %d rr %.3e tol2 %.3e\n",
                   nread, *iters, cr.flags[F_DONE], *status, cr.rr_tol2[0], cr.rr_tol2[1]);
    if (cr.flags[F_DONE]) break;
    // the predicted iterations to the stop, from the decay of ||r||^2 since
    // the previous chunk's end
    const double rr = cr.rr_tol2[0], tol2 = cr.rr_tol2[1];
    ahead = 2;
    if (prev_iters >= 0 &&
        predicted_steps(prev_rr, prev_iters, rr, *iters, tol2) <= (double)(launched - *iters))
      ahead = 1;
    prev_rr = rr;
    prev_iters = *iters;
  }
  if (c->prof) {  // samples of a chunk still queued, then the pairs are free again
    if (c->ev_done < c->ev_used) {
      HIPCHK(hipEventSynchronize(c->chunk_ev[(queued - 1) % 2]));
      prof_collect(c, c->ev_used, *iters);
    }
    c->ev_used = c->ev_done = 0;
  }
  return TO_OK;
}

// u += the inner solution (with the grouped steps still pending)
template <typename T>
to_status axpy_correction(to_ctx *c, double *u, const CgDesc<T> &d) {
  HIPCHK(launch_axpy_out<T>(c->g, u, d.x, c->scal, c->stream, d.np == 4 ? 4 : 2, d.xgroup, d.p,
                            c->flags));
  return TO_OK;
}

to_status residual64(to_ctx *c, const double *u) {
  MvArgs<double> a{};
  a.nelx = c->g.nelx;
  a.nely = c->g.nely;
  a.nelz = c->g.nelz;
  a.kz = c->kz;
  a.E = c->E64;
  a.in = u;
  a.out = c->r64;
  a.f = c->f;
  a.mask = c->mask;
  a.part = c->part;
  a.k = c->k64;
  int nb = 0;
  HIPCHK((launch_matvec<double, MV_RESID>(a, &nb, c->stream)));
  HIPCHK(launch_finish_sum(c->part, nb, 0, c->scal, S_NORM2, c->stream));
  HIPCHK(launch_set_scale(c->scal, c->stream));
  return TO_OK;
}


}  // namespace

extern "C" {

to_status to_workspace_size(const to_problem *prob, size_t *bytes) {
  std::string why;
  if (!bytes) return fail(nullptr, TO_E_INVALID, "bytes is NULL");
  if (!validate_problem(prob, &why)) return fail(nullptr, TO_E_INVALID, why);
  *bytes = carve(nullptr, make_grid(prob), prob->precision, prob->nu, nullptr);
  return TO_OK;
}

to_status to_create(const to_problem *prob, void *d_workspace, size_t bytes, void *stream,
                    to_ctx **out) {
  std::string why;
  if (!out) return fail(nullptr, TO_E_INVALID, "out is NULL");
  *out = nullptr;
  if (!validate_problem(prob, &why)) return fail(nullptr, TO_E_INVALID, why);
  if (d_workspace && ((uintptr_t)d_workspace & 255u))
    return fail(nullptr, TO_E_INVALID, "workspace must be 256-byte aligned");
  to_ctx *c = new to_ctx();
  c->p = *prob;
  c->p.fixed_mask = nullptr;
  c->p.load = nullptr;
  c->g = make_grid(prob);
  c->stream = (hipStream_t)stream;
  if (const char *e = std::getenv("TOPO_INNER_ETA")) c->eta = std::atof(e);
  if (const char *e = std::getenv("TOPO_CHUNK")) c->chunk = std::max(1, std::atoi(e));
  if (const char *e = std::getenv("TOPO_TRACE")) c->trace = std::atoi(e) != 0;
  if (const char *e = std::getenv("TOPO_PROF_EVERY")) c->prof_every = std::max(2, std::atoi(e));
  if (const char *e = std::getenv("TOPO_GRAPH")) c->use_graph = std::atoi(e) != 0;
  auto bail = [&](to_status s, const std::string &m) {
    to_status r = fail(nullptr, s, m);
    to_destroy(c);
    return r;
  };
  if (hipGetDevice(&c->device) != hipSuccess) return bail(TO_E_HIP, "hipGetDevice failed");
  const size_t need = carve(nullptr, c->g, prob->precision, prob->nu, nullptr);
  if (d_workspace) {
    if (bytes < need) return bail(TO_E_OOM, "workspace smaller than to_workspace_size()");
    c->ws = (char *)d_workspace;
    c->ws_bytes = bytes;
  } else {
    if (hipMalloc((void **)&c->ws, need) != hipSuccess) return bail(TO_E_OOM, "hipMalloc failed");
    c->owns_ws = true;
    c->ws_bytes = need;
  }
  carve(c, c->g, prob->precision, prob->nu, c->ws);
  // S_COUNT scalars, then OC_STATE + 8 doubles of optimality-criteria state
  if (hipHostMalloc((void **)&c->h_scal, (S_COUNT + OC_STATE + 8) * sizeof(double),
                    hipHostMallocDefault) !=
          hipSuccess ||
      hipHostMalloc((void **)&c->h_flags, F_COUNT * sizeof(int), hipHostMallocDefault) != hipSuccess ||
      hipHostMalloc((void **)&c->h_chunk, 2 * sizeof(to_ctx::ChunkRead), hipHostMallocDefault) !=
          hipSuccess)
    return bail(TO_E_OOM, "hipHostMalloc failed");
  for (hipEvent_t &e : c->chunk_ev)
    if (hipEventCreateWithFlags(&e, hipEventDisableTiming) != hipSuccess)
      return bail(TO_E_HIP, "hipEventCreate failed");
  c->k64 = make_coef<double>(prob->nu, prob->h);
  c->k32 = make_coef<float>(prob->nu, prob->h);
  {
    const double lam = prob->nu / ((1.0 + prob->nu) * (1.0 - 2.0 * prob->nu));
    const double mu = 1.0 / (2.0 * (1.0 + prob->nu));
    c->kd = prob->h * (lam + 4.0 * mu) / 9.0;
  }
  c->kz = matvec_kz(c->g, prob->precision == TO_PREC_FP64);
  c->kz_mf = matvec_kz(c->g, false, true);
  hipStream_t s = c->stream;
  if (c->mA) {
    uint16_t tab[2][64][8];
    float unit = 0.f;
    mfma_operand_table(prob->nu, tab, &unit);
    c->mscale = (float)(unit * prob->h);
    if (hipMemcpyAsync((void *)c->mA, tab, sizeof(tab), hipMemcpyHostToDevice, s) != hipSuccess ||
        hipStreamSynchronize(s) != hipSuccess)
      return bail(TO_E_HIP, "uploading the matrix-core operand failed");
  }
  // descriptors of the CG kernels (passed by value at each launch)
  if (prob->precision == TO_PREC_FP64) c->hd64 = make_desc<double>(c, c->v64, c->E64, c->dinv64, c->k64);
  else c->hd32 = make_desc<float>(c, c->v32, c->E32, c->dinv32, c->k32);
  if (prob->bc == TO_BC_CUSTOM) {
    // host arrays -> device: the per-DOF mask goes through the triangle
    // scratch (int array of nel >= ... may be small), so use a temporary
    uint8_t *dm = nullptr;
    if (hipMalloc((void **)&dm, c->g.ndof) != hipSuccess) return bail(TO_E_OOM, "hipMalloc failed");
    bool ok = hipMemcpy(dm, prob->fixed_mask, c->g.ndof, hipMemcpyHostToDevice) == hipSuccess &&
              hipMemcpy(c->f, prob->load, c->g.ndof * sizeof(double), hipMemcpyHostToDevice) ==
                  hipSuccess &&
              launch_mask_custom(c->g, dm, c->mask, c->f, s) == hipSuccess &&
              hipStreamSynchronize(s) == hipSuccess;
    hipFree(dm);
    if (!ok) return bail(TO_E_HIP, "uploading the custom mask/load failed");
  } else {
    if (launch_mask_builtin(c->g, prob->bc, c->mask, s) != hipSuccess ||
        launch_load_builtin(c->g, prob->bc, prob->load_total, c->mask, c->f, s) != hipSuccess)
      return bail(TO_E_HIP, "building the mask/load failed");
  }
  // ||f||
  int nb = 0;
  if (launch_dot(c->f, c->f, c->g.ndof, c->part, &nb, s) != hipSuccess ||
      launch_finish_sum(c->part, nb, 0, c->scal, S_TMP, s) != hipSuccess)
    return bail(TO_E_HIP, "norm of f failed");
  if (sync_read(c) != TO_OK) return bail(TO_E_HIP, "sync failed");
  c->fnorm = std::sqrt(c->h_scal[S_TMP]);
  *out = c;
  return TO_OK;
}

void to_destroy(to_ctx *c) {
  if (!c) return;
  if (c->stream) hipStreamSynchronize(c->stream);
  else hipDeviceSynchronize();
  for (hipEvent_t e : c->ev) hipEventDestroy(e);
  for (auto &row : c->graph)
    for (hipGraphExec_t &g : row)
      if (g) hipGraphExecDestroy(g);
  if (c->owns_ws && c->ws) hipFree(c->ws);
  if (c->tri) hipFree(c->tri);
  if (c->shp) hipFree(c->shp);
  if (c->h_scal) hipHostFree(c->h_scal);
  if (c->h_flags) hipHostFree(c->h_flags);
  if (c->h_chunk) hipHostFree(c->h_chunk);
  for (hipEvent_t e : c->chunk_ev)
    if (e) hipEventDestroy(e);
  delete c;
}

const char *to_last_error(const to_ctx *c) {
  if (c) return c->err.c_str();
  return g_last_error.c_str();
}

to_status to_solve(to_ctx *c, const double *d_x, const double *d_u0, double *d_u,
                   to_solve_info *info) {
  if (!c) return fail(nullptr, TO_E_INVALID, "ctx is NULL");
  if (!d_x || !d_u) return fail(c, TO_E_INVALID, "d_x and d_u are required");
  const double t0 = now_ms();
  HIPCHK(hipSetDevice(c->device));
  const Grid &g = c->g;
  to_status st = prepare_moduli(c, d_x, false);
  if (st != TO_OK) return st;
  HIPCHK(launch_diag(g, c->E64, c->kd, c->mask, c->dinv64, c->dinv32, c->stream));
  if (d_u0 && d_u0 != d_u)
    HIPCHK(hipMemcpyAsync(d_u, d_u0, g.ndof * sizeof(double), hipMemcpyDeviceToDevice, c->stream));
  else if (!d_u0)
    HIPCHK(launch_fill(d_u, g.ndof * sizeof(double), c->stream));
  st = sync_read(c);
  if (st != TO_OK) return st;
  if (c->h_flags[F_BADX] & 2) return fail(c, TO_E_NONFINITE, "x holds NaN or Inf");
  if (c->h_flags[F_BADX] & 1) return fail(c, TO_E_INVALID, "x outside [0,1]");

  const bool fp64 = c->p.precision == TO_PREC_FP64;
  int outer = 0, total_inner = 0;
  double rel = 0.0;
  StagnationRule stall;
  to_status result = TO_OK;
  std::string msg;
  if (c->fnorm == 0.0) {
    HIPCHK(launch_fill(d_u, g.ndof * sizeof(double), c->stream));
  } else {
    for (;;) {
      st = residual64(c, d_u);
      if (st != TO_OK) return st;
      st = sync_read(c);
      if (st != TO_OK) return st;
      rel = std::sqrt(c->h_scal[S_NORM2]) / c->fnorm;
      if (c->trace)
        std::fprintf(stderr, "[topo] outer %d rel %.3e inner_total %d\n", outer, rel, total_inner);
      if (!std::isfinite(rel)) { result = TO_E_NONFINITE; msg = "non-finite residual"; break; }
      if (rel <= c->p.rtol) break;
      if (total_inner >= c->p.max_iters || outer >= 200) {
        result = TO_E_NOCONV;
        msg = "iteration cap reached";
        break;
      }
      // attainable accuracy: stop when four refinement passes have not halved
      // the float64 residual
      if (stall.record(rel)) {
        result = TO_E_NOCONV;
        msg = "residual stagnated above rtol (attainable accuracy reached)";
        break;
      }
      // inner relative tolerance: the whole remaining reduction in float64,
      // eta (or the remaining reduction if smaller) in float32
      const double need = 0.5 * c->p.rtol / rel;
      const double eta = fp64 ? need : std::max(c->eta, need);
      int it = 0, status = 0;
      const int cap = c->p.max_iters - total_inner;
      if (fp64) {
        st = inner_pcg<double>(c, c->v64, c->dinv64, eta, cap, &it, &status);
        if (st != TO_OK) return st;
        st = axpy_correction<double>(c, d_u, c->hd64);
      } else {
        st = inner_pcg<float>(c, c->v32, c->dinv32, eta, cap, &it, &status);
        if (st != TO_OK) return st;
        st = axpy_correction<float>(c, d_u, c->hd32);
      }
      if (st != TO_OK) return st;
      total_inner += it;
      ++outer;
      // A breakdown after some progress ends the inner solve like convergence
      // (the float64 residual decides what happens next); without progress
      // the system is singular or indefinite.
      if (status == 1 && it == 0) { result = TO_E_SINGULAR; msg = "CG breakdown: p^T K p <= 0"; }
      if (status == 2) { result = TO_E_NONFINITE; msg = "non-finite value in CG"; }
      if (result != TO_OK) {
        st = residual64(c, d_u);
        if (st == TO_OK) st = sync_read(c);
        if (st == TO_OK) rel = std::sqrt(c->h_scal[S_NORM2]) / c->fnorm;
        break;
      }
    }
  }
  HIPCHK(hipStreamSynchronize(c->stream));
  if (info) {
    info->outer_iters = outer;
    info->inner_iters = total_inner;
    info->rel_res = rel;
    info->ms = now_ms() - t0;
  }
  if (result != TO_OK) return fail(c, result, msg);
  return TO_OK;
}

to_status to_compliance_sensitivity(to_ctx *c, const double *d_x, const double *d_u, double *h_c,
                                    double *d_dc) {
  if (!c) return fail(nullptr, TO_E_INVALID, "ctx is NULL");
  if (!d_x || !d_u || !h_c) return fail(c, TO_E_INVALID, "d_x, d_u and h_c are required");
  HIPCHK(hipSetDevice(c->device));
  to_status st = prepare_moduli(c, d_x, false);
  if (st != TO_OK) return st;
  int nb = 0;
  HIPCHK(launch_energy_sens(c->g, d_x, d_u, c->E64, c->k64, c->p.E0, c->p.Emin, c->p.penal, d_dc,
                            c->part, &nb, c->stream));
  HIPCHK(launch_finish_sum(c->part, nb, 0, c->scal, S_ES, c->stream));
  HIPCHK(launch_dot(c->f, d_u, c->g.ndof, c->part, &nb, c->stream));
  HIPCHK(launch_finish_sum(c->part, nb, 0, c->scal, S_C, c->stream));
  st = sync_read(c);
  if (st != TO_OK) return st;
  if (c->h_flags[F_BADX] & 2) return fail(c, TO_E_NONFINITE, "x holds NaN or Inf");
  if (c->h_flags[F_BADX] & 1) return fail(c, TO_E_INVALID, "x outside [0,1]");
  *h_c = c->h_scal[S_C];
  if (!std::isfinite(*h_c)) return fail(c, TO_E_NONFINITE, "non-finite compliance");
  return TO_OK;
}

double to_last_energy_sum(const to_ctx *c) { return c ? c->h_scal[S_ES] : 0.0; }

to_status to_filter(to_ctx *c, double rmin, int32_t mode, const double *d_x, const double *d_in,
                    double *d_out) {
  if (!c) return fail(nullptr, TO_E_INVALID, "ctx is NULL");
  if (!(rmin > 0.0) || !(rmin <= MAX_RMIN)) return fail(c, TO_E_INVALID, "need 0 < rmin <= 6");
  if (mode < 0 || mode > 2) return fail(c, TO_E_INVALID, "unknown filter mode");
  if (!d_in || !d_out) return fail(c, TO_E_INVALID, "d_in and d_out are required");
  if (d_in == d_out) return fail(c, TO_E_INVALID, "d_out must not alias d_in");
  if (mode == TO_FILTER_SENS && !d_x) return fail(c, TO_E_INVALID, "SENS mode needs d_x");
  HIPCHK(hipSetDevice(c->device));
  if (rmin != c->last_rmin) {
    // offsets with distance < rmin in (dz, dy, dx) lexicographic order
    std::vector<int> ofs;
    std::vector<double> w;
    const int m = (int)std::ceil(rmin);
    for (int dz = -m; dz <= m; ++dz)
      for (int dy = -m; dy <= m; ++dy)
        for (int dx = -m; dx <= m; ++dx) {
          const double d = std::sqrt((double)(dx * dx + dy * dy + dz * dz));
          if (d < rmin) {
            ofs.push_back(dx);
            ofs.push_back(dy);
            ofs.push_back(dz);
            w.push_back(rmin - d);
          }
        }
    if ((int)w.size() > MAXOFS) return fail(c, TO_E_INVALID, "filter stencil too large");
    HIPCHK(hipStreamSynchronize(c->stream));
    HIPCHK(hipMemcpy(c->fofs, ofs.data(), ofs.size() * sizeof(int), hipMemcpyHostToDevice));
    HIPCHK(hipMemcpy(c->fw, w.data(), w.size() * sizeof(double), hipMemcpyHostToDevice));
    c->nofs = (int)w.size();
    c->last_rmin = rmin;
  }
  const double V = c->p.h * c->p.h * c->p.h;
  HIPCHK(launch_filter(c->g, mode, c->nofs, c->fofs, c->fw, V, d_x, d_in, c->ftmp, d_out,
                       c->stream));
  return TO_OK;
}

namespace {

// Density -> SDF on a context.  tri_fixed == nullptr: triangles in the
// context's buffer, grown by hipMalloc when a design needs more; otherwise
// the caller's fixed device array of tri_max triangles, and a design that
// needs more is rejected (after the count pass, before any triangle is
// written).
to_status density_to_sdf(to_ctx *c, const double *d_x, double rho_t, double *d_phi,
                         double *d_rho_nodes, double *d_vf, double *tri_fixed, size_t tri_max) {
  if (!c) return fail(nullptr, TO_E_INVALID, "ctx is NULL");
  if (!d_x || !d_phi) return fail(c, TO_E_INVALID, "d_x and d_phi are required");
  if (!std::isfinite(rho_t)) return fail(c, TO_E_INVALID, "rho_t must be finite");
  HIPCHK(hipSetDevice(c->device));
  const Grid &g = c->g;
  double *rho = d_rho_nodes ? d_rho_nodes : c->rho_scratch;
  HIPCHK(launch_node_mean(g, d_x, rho, c->stream));
  HIPCHK(launch_mt_count(g, rho, rho_t, c->cnt, c->stream));
  HIPCHK(launch_scan(c->cnt, c->toff, g.nel, c->bsums, c->stream));
  const int nt = (int)((g.nel + 1023) / 1024);
  HIPCHK(hipMemcpyAsync(c->h_flags + F_COUNT - 1, c->bsums + nt, sizeof(int),
                        hipMemcpyDeviceToHost, c->stream));
  HIPCHK(hipStreamSynchronize(c->stream));
  const int total = c->h_flags[F_COUNT - 1];
  c->last_tri = total;
  if (total < 0) return fail(c, TO_E_INVALID, "triangle count overflow");
  if (total > 0) {
    double *tri = tri_fixed;
    if (tri_fixed) {
      if ((size_t)total > tri_max)
        return fail(c, TO_E_OOM,
                    "the design's iso-surface has " + std::to_string(total) +
                        " triangles; to_density_to_sdf_noalloc holds at most " +
                        std::to_string(tri_max) + " (use to_density_to_sdf)");
    } else {
      const size_t need = (size_t)total * 9;
      if (need > c->tri_cap) {
        if (c->tri) HIPCHK(hipFree(c->tri));
        c->tri = nullptr;
        c->tri_cap = 0;
        const size_t cap = need + need / 4;
        if (hipMalloc((void **)&c->tri, cap * sizeof(double)) != hipSuccess)
          return fail(c, TO_E_OOM, "cannot allocate the triangle buffer");
        c->tri_cap = cap;
      }
      tri = c->tri;
    }
    HIPCHK(launch_mt_emit(g, rho, rho_t, c->p.h, c->toff, c->cnt, tri, c->stream));
    // the coarse occupancy bitmask reuses the filter scratch (nel doubles, far more than
    // the nel/2048 words it needs)
    HIPCHK(launch_udist(g, c->p.h, c->cnt, c->toff, tri, (int *)c->ftmp, rho, rho_t, d_phi,
                        c->stream));
  } else {
    HIPCHK(launch_sign_inf(g, rho, rho_t, d_phi, c->stream));
  }
  if (d_vf) HIPCHK(launch_vf(g, d_phi, d_vf, c->stream));
  return TO_OK;
}

}  // namespace

to_status to_density_to_sdf(to_ctx *c, const double *d_x, double rho_t, double *d_phi,
                            double *d_rho_nodes, double *d_vf) {
  return density_to_sdf(c, d_x, rho_t, d_phi, d_rho_nodes, d_vf, nullptr, 0);
}

// ---- the variant that allocates nothing.  Its triangles live in `scratch`,
// a fixed device array that every GPU the library runs on holds until the
// process ends.  In host code the array's name is only a host-side stand-in:
// its device address, per device, comes from hipGetSymbolAddress on that
// device's first call and is what kernels receive.
namespace {
constexpr size_t NOALLOC_TRI_MAX = TO_NOALLOC_MAX_TRIANGLES;  // 72 bytes each: 18.9 MB
constexpr int NOALLOC_MAX_DEVICES = 64;
}  // namespace

static __device__ __align__(256) double scratch[NOALLOC_TRI_MAX * 9];

namespace {
std::mutex g_scratch_mu;
double *g_scratch_dev[NOALLOC_MAX_DEVICES] = {};

// device address of `scratch` on the current device c->device
to_status scratch_address(to_ctx *c, double **out) {
  if (c->device < 0 || c->device >= NOALLOC_MAX_DEVICES)
    return fail(c, TO_E_INVALID, "device ordinal beyond the no-allocation variant's table");
  std::lock_guard<std::mutex> lock(g_scratch_mu);
  if (!g_scratch_dev[c->device]) {
    void *ptr = nullptr;
    const hipError_t e = hipGetSymbolAddress(&ptr, HIP_SYMBOL(scratch));
    if (e != hipSuccess || !ptr)
      return fail(c, TO_E_HIP, std::string("hipGetSymbolAddress(scratch): ") + hipGetErrorString(e));
    g_scratch_dev[c->device] = (double *)ptr;
  }
  *out = g_scratch_dev[c->device];
  return TO_OK;
}
}  // namespace

to_status to_density_to_sdf_noalloc(to_ctx *c, const double *d_x, double rho_t, double *d_phi,
                                    double *d_rho_nodes, double *d_vf) {
  if (!c) return fail(nullptr, TO_E_INVALID, "ctx is NULL");
  HIPCHK(hipSetDevice(c->device));
  double *tri = nullptr;
  const to_status st = scratch_address(c, &tri);
  if (st != TO_OK) return st;
  return density_to_sdf(c, d_x, rho_t, d_phi, d_rho_nodes, d_vf, tri, NOALLOC_TRI_MAX);
}

int32_t to_last_triangle_count(const to_ctx *c) { return c ? c->last_tri : 0; }

to_status to_volume_fraction(to_ctx *c, const double *d_phi, double *d_vf) {
  if (!c) return fail(nullptr, TO_E_INVALID, "ctx is NULL");
  if (!d_phi || !d_vf) return fail(c, TO_E_INVALID, "d_phi and d_vf are required");
  HIPCHK(hipSetDevice(c->device));
  HIPCHK(launch_vf(c->g, d_phi, d_vf, c->stream));
  return TO_OK;
}

to_status to_oc_update(to_ctx *c, const double *d_x, const double *d_dc, double vf, double move,
                       double eta, double *d_xnew, to_oc_info *info) {
  if (!c) return fail(nullptr, TO_E_INVALID, "ctx is NULL");
  if (!d_x || !d_dc || !d_xnew) return fail(c, TO_E_INVALID, "d_x, d_dc and d_xnew are required");
  if (d_xnew == d_dc) return fail(c, TO_E_INVALID, "d_xnew must not alias d_dc");
  if (!(vf > 0.0 && vf <= 1.0)) return fail(c, TO_E_INVALID, "need 0 < vf <= 1");
  if (!(move > 0.0 && move <= 1.0)) return fail(c, TO_E_INVALID, "need 0 < move <= 1");
  if (!(eta > 0.0 && eta <= 1.0)) return fail(c, TO_E_INVALID, "need 0 < eta <= 1");
  static_assert(OC_SCRATCH <= 2 * MAXB, "OC scratch lives in the partial-sum array");
  HIPCHK(hipSetDevice(c->device));
  const size_t nel = c->g.nel;
  double *scr = c->part, *h = c->h_scal + S_COUNT;
  const double target = vf * (double)nel;
  HIPCHK(launch_fill(c->flags, F_COUNT * sizeof(int), c->stream));
  // one launch per midpoint plus the one that ends the loop; most updates
  // take 40-50, so the first batch usually covers them and one host poll
  // suffices
  int k = 0;
  for (int batch = 64;; batch = 32) {
    HIPCHK(launch_oc_steps(d_x, d_dc, nel, move, eta, target, OC_TOL, OC_L2_0, OC_MAX_STEPS, scr,
                           k, batch, c->flags, c->stream));
    k += batch;
    HIPCHK(hipMemcpyAsync(h, scr + OC_STATE_OFS + (k & 1) * OC_STATE, OC_STATE * sizeof(double),
                          hipMemcpyDeviceToHost, c->stream));
    HIPCHK(hipMemcpyAsync(c->h_flags, c->flags, F_COUNT * sizeof(int), hipMemcpyDeviceToHost,
                          c->stream));
    HIPCHK(hipStreamSynchronize(c->stream));
    if ((c->h_flags[F_BADX] & 2) || c->h_flags[F_BADG])
      return fail(c, TO_E_NONFINITE, "x or dc holds NaN or Inf");
    if (c->h_flags[F_BADX] & 1) return fail(c, TO_E_INVALID, "x outside [0,1]");
    if (h[OC_DONE] != 0.0) break;
    if (k > OC_MAX_STEPS + 64) return fail(c, TO_E_HIP, "OC bisection state did not advance");
  }
  if (h[OC_DONE] != 1.0)
    return fail(c, TO_E_NOCONV,
                "OC bisection: no multiplier within 200 midpoints (volume target unreachable)");
  HIPCHK(launch_oc_apply(d_x, d_dc, d_xnew, nel, move, eta, scr, k, c->stream));
  HIPCHK(hipMemcpyAsync(h + OC_STATE, scr + OC_OUT_OFS, 8 * sizeof(double), hipMemcpyDeviceToHost,
                        c->stream));
  HIPCHK(hipStreamSynchronize(c->stream));
  if (info) {
    info->lambda = h[OC_STATE + 0];
    info->change = h[OC_STATE + 1];
    info->volume = h[OC_STATE + 2] / (double)nel;
    info->bisections = (int32_t)h[OC_STATE + 3];
    info->reserved = 0;
  }
  return TO_OK;
}

// Level-set scratch: the second field buffer is the node-density scratch of
// the SDF transfer (nn doubles, only used inside to_density_to_sdf); the
// change slots, the loop state and the max|v| word live in the partial-sum
// array, cleared here before every call.
// NaN/Inf check of d_phi (and d_v) with max|v|; `what` names the inputs in
// the error message
to_status ls_check(to_ctx *c, const double *d_phi, const double *d_v, double *vmax,
                   const char *what = "phi or v holds NaN or Inf") {
  static_assert(LS_SCRATCH <= 2 * MAXB, "level-set scratch lives in the partial-sum array");
  unsigned long long *words = (unsigned long long *)c->part;
  HIPCHK(launch_fill(c->flags, F_COUNT * sizeof(int), c->stream));
  HIPCHK(launch_fill(c->part, LS_SCRATCH * sizeof(double), c->stream));
  HIPCHK(launch_ls_check(c->g, d_phi, d_v, c->flags, words + LS_VMAX_OFS, c->stream));
  double *h = c->h_scal + S_COUNT;
  HIPCHK(hipMemcpyAsync(h, words + LS_VMAX_OFS, sizeof(double), hipMemcpyDeviceToHost,
                        c->stream));
  HIPCHK(hipMemcpyAsync(c->h_flags, c->flags, F_COUNT * sizeof(int), hipMemcpyDeviceToHost,
                        c->stream));
  HIPCHK(hipStreamSynchronize(c->stream));
  if (c->h_flags[F_BADX] & 2) return fail(c, TO_E_NONFINITE, what);
  *vmax = h[0];
  return TO_OK;
}

to_status to_ls_advect(to_ctx *c, double *d_phi, const double *d_v, double gamma, int32_t nsteps,
                       double *h_dt) {
  if (!c) return fail(nullptr, TO_E_INVALID, "ctx is NULL");
  if (!d_phi || !d_v) return fail(c, TO_E_INVALID, "d_phi and d_v are required");
  if (d_phi == d_v) return fail(c, TO_E_INVALID, "d_v must not alias d_phi");
  if (!(gamma > 0.0 && gamma <= 1.0)) return fail(c, TO_E_INVALID, "need 0 < gamma <= 1");
  if (nsteps < 0) return fail(c, TO_E_INVALID, "nsteps must be >= 0");
  HIPCHK(hipSetDevice(c->device));
  double vmax = 0.0;
  to_status st = ls_check(c, d_phi, d_v, &vmax);
  if (st != TO_OK) return st;
  const double h = c->p.h;
  const double dt = vmax == 0.0 ? 0.0 : gamma * h / vmax;
  if (h_dt) *h_dt = dt;
  if (dt == 0.0 || nsteps == 0) return TO_OK;
  double *buf[2] = {d_phi, c->rho_scratch};
  for (int k = 0; k < nsteps; ++k)
    HIPCHK(launch_ls_advect(c->g, h, dt, buf[k & 1], d_v, buf[(k + 1) & 1], c->stream));
  if (nsteps & 1)
    HIPCHK(hipMemcpyAsync(d_phi, buf[1], c->g.nn * sizeof(double), hipMemcpyDeviceToDevice,
                          c->stream));
  return TO_OK;
}

to_status to_ls_reinit(to_ctx *c, double *d_phi, double gamma, double tol, int32_t max_steps,
                       int32_t *h_steps, double *h_change) {
  if (!c) return fail(nullptr, TO_E_INVALID, "ctx is NULL");
  if (!d_phi) return fail(c, TO_E_INVALID, "d_phi is required");
  if (!(gamma > 0.0 && gamma <= 1.0)) return fail(c, TO_E_INVALID, "need 0 < gamma <= 1");
  if (!(tol > 0.0) || !std::isfinite(tol)) return fail(c, TO_E_INVALID, "need tol > 0");
  if (max_steps < 1) return fail(c, TO_E_INVALID, "max_steps must be >= 1");
  HIPCHK(hipSetDevice(c->device));
  double vmax = 0.0;
  to_status st = ls_check(c, d_phi, nullptr, &vmax);
  if (st != TO_OK) return st;
  const double h = c->p.h, dtau = gamma * h;
  unsigned long long *slots = (unsigned long long *)c->part;
  double *state = c->part + LS_STATE_OFS, *hs = c->h_scal + S_COUNT;
  double *buf[2] = {d_phi, c->rho_scratch};
  // one launch per pseudo-step plus the one that sees the stop; the host
  // looks at the state once per batch of at most 64.  Launches after the stop
  // return at once, so once the decay of the largest change between two looks
  // predicts the stop, the next batch is cut to the predicted count (a short
  // guess costs one more host round trip).
  int k = 0, batch = 64, k_prev = -1;
  double ch_prev = 0.0;
  for (;;) {
    for (int b = 0; b < batch; ++b, ++k)
      HIPCHK(launch_ls_reinit(c->g, h, dtau, tol, max_steps, k, buf[k & 1], buf[(k + 1) & 1],
                              slots, state, c->stream));
    HIPCHK(hipMemcpyAsync(hs, state, 4 * sizeof(double), hipMemcpyDeviceToHost, c->stream));
    HIPCHK(hipStreamSynchronize(c->stream));
    if (hs[0] != 0.0) break;
    if (k > max_steps + 128) return fail(c, TO_E_HIP, "reinitialisation state did not advance");
    // hs[3]: the largest change of step k - 1 (taken by launch k - 1)
    const double ch = hs[3];
    batch = 64;
    if (k_prev >= 0) {
      const double remaining = predicted_steps(ch_prev, k_prev, ch, k, tol);
      batch = (int)std::min(64.0, std::max(4.0, std::ceil(1.1 * remaining) + 2.0));
    }
    k_prev = k;
    ch_prev = ch;
  }
  const int steps = (int)hs[1];
  if (steps & 1)
    HIPCHK(hipMemcpyAsync(d_phi, buf[1], c->g.nn * sizeof(double), hipMemcpyDeviceToDevice,
                          c->stream));
  HIPCHK(hipStreamSynchronize(c->stream));
  if (h_steps) *h_steps = steps;
  if (h_change) *h_change = hs[2];
  if (hs[0] != 1.0)
    return fail(c, TO_E_NOCONV, "reinitialisation: change still >= tol after max_steps");
  return TO_OK;
}

to_status to_shape_rhs(to_ctx *c, const double *d_u, const double *d_phi, double eta, double c_s,
                       double c_0, double *d_g) {
  if (!c) return fail(nullptr, TO_E_INVALID, "ctx is NULL");
  if (!d_phi || !d_g) return fail(c, TO_E_INVALID, "d_phi and d_g are required");
  if (c_s != 0.0 && !d_u) return fail(c, TO_E_INVALID, "d_u is required when c_s != 0");
  if (d_g == d_phi) return fail(c, TO_E_INVALID, "d_g must not alias d_phi");
  if (!(eta > 0.0) || !std::isfinite(eta)) return fail(c, TO_E_INVALID, "need eta > 0");
  if (!std::isfinite(c_s) || !std::isfinite(c_0))
    return fail(c, TO_E_INVALID, "c_s and c_0 must be finite");
  HIPCHK(hipSetDevice(c->device));
  const double nu = c->p.nu, E0 = c->p.E0;
  const double lam = E0 * nu / ((1.0 + nu) * (1.0 - 2.0 * nu)), mu = E0 / (2.0 * (1.0 + nu));
  if (!c->shp && hipMalloc((void **)&c->shp, 8 * c->g.nel * sizeof(double)) != hipSuccess) {
    c->shp = nullptr;
    return fail(c, TO_E_OOM, "cannot allocate the shape-derivative element buffer");
  }
  // the per-element band bytes use the triangle-count scratch of the SDF
  // transfer (nel ints)
  HIPCHK(launch_shape_rhs(c->g, d_u, d_phi, c->p.h, lam, mu, eta, c_s, c_0, (uint8_t *)c->cnt,
                          c->shp, d_g, c->stream));
  return TO_OK;
}

to_status to_hilbert_extend(to_ctx *c, double ell, const double *d_g, double *d_v, double rtol,
                            int32_t max_iters, int32_t *h_iters, double *h_rel) {
  if (!c) return fail(nullptr, TO_E_INVALID, "ctx is NULL");
  if (!d_g || !d_v) return fail(c, TO_E_INVALID, "d_g and d_v are required");
  if (d_g == d_v) return fail(c, TO_E_INVALID, "d_v must not alias d_g");
  if (!(ell >= 0.0) || !std::isfinite(ell)) return fail(c, TO_E_INVALID, "need ell >= 0");
  if (!(rtol > 0.0 && rtol < 1.0)) return fail(c, TO_E_INVALID, "need 0 < rtol < 1");
  if (max_iters < 1) return fail(c, TO_E_INVALID, "max_iters must be >= 1");
  static_assert(HCG_SCRATCH <= 2 * MAXB, "extension scratch lives in the partial-sum array");
  HIPCHK(hipSetDevice(c->device));
  double gmax = 0.0;
  to_status chk = ls_check(c, d_g, nullptr, &gmax, "g holds NaN or Inf");
  if (chk != TO_OK) return chk;
  // r, z, p, q: nn doubles each in the CG vector arrays (each holds at least
  // 3 nn floats); the Gamma_N mask in the node scratch
  double *vec[4];
  for (int i = 0; i < 4; ++i)
    vec[i] = c->p.precision == TO_PREC_FP64 ? c->v64[i] : (double *)c->v32[i];
  uint8_t *gm = (uint8_t *)c->rho_scratch;
  double *scal = c->part + HCG_SCAL_OFS, *hs = c->h_scal + S_COUNT;
  HIPCHK(launch_fill(c->flags, F_COUNT * sizeof(int), c->stream));
  // chunks of at most 32 iterations; launches after the stop return at once,
  // so once the residual's mean decay so far predicts the stop, the next
  // chunk is cut to the predicted count (a short guess costs one more host
  // round trip)
  int it = 0, n_next = 32;
  for (;;) {
    const int n = std::min(n_next, max_iters + 1 - it);
    HIPCHK(launch_hilbert(c->g, c->p.h, ell, rtol, max_iters, c->f, d_g, d_v, vec, gm, c->part,
                          scal, c->flags, it, n, c->stream));
    it += n;
    HIPCHK(hipMemcpyAsync(hs, scal, 4 * sizeof(double), hipMemcpyDeviceToHost, c->stream));
    HIPCHK(hipMemcpyAsync(c->h_flags, c->flags, sizeof(int), hipMemcpyDeviceToHost, c->stream));
    HIPCHK(hipStreamSynchronize(c->stream));
    if (c->h_flags[0] != 0) break;
    if (it > max_iters) return fail(c, TO_E_HIP, "extension CG state did not advance");
    // hs: [0] the stopping r^T r, [1] r^T r after [2] iterations, [3] the first r^T r
    const double remaining = predicted_steps(hs[3], 0.0, hs[1], hs[2], hs[0]);
    n_next = (int)std::min(32.0, std::max(1.0, std::ceil(1.1 * remaining) + 1.0));
  }
  const int st = c->h_flags[0];
  if (h_iters) *h_iters = (int32_t)hs[2];
  if (h_rel) *h_rel = hs[3] > 0.0 ? std::sqrt(hs[1] / hs[3]) : 0.0;
  if (st == 2) return fail(c, TO_E_NOCONV, "extension CG: iteration cap reached");
  if (st == 3) return fail(c, TO_E_SINGULAR, "extension CG breakdown: p^T A p <= 0");
  return TO_OK;
}

to_status to_simp(to_ctx *c, const to_simp_params *sp, double *d_x, double *d_u, double *d_work,
                  double *h_c_hist, to_simp_info *info) {
  if (!c) return fail(nullptr, TO_E_INVALID, "ctx is NULL");
  if (!sp) return fail(c, TO_E_INVALID, "params are required");
  if (!d_x || !d_u || !d_work) return fail(c, TO_E_INVALID, "d_x, d_u and d_work are required");
  if (!(sp->vf > 0.0 && sp->vf <= 1.0)) return fail(c, TO_E_INVALID, "need 0 < vf <= 1");
  if (!(sp->rmin > 0.0 && sp->rmin <= MAX_RMIN)) return fail(c, TO_E_INVALID, "need 0 < rmin <= 6");
  if (!(sp->move > 0.0 && sp->move <= 1.0)) return fail(c, TO_E_INVALID, "need 0 < move <= 1");
  if (!(sp->eta > 0.0 && sp->eta <= 1.0)) return fail(c, TO_E_INVALID, "need 0 < eta <= 1");
  if (!(sp->change_tol >= 0.0)) return fail(c, TO_E_INVALID, "need change_tol >= 0");
  if (sp->max_iters < 1) return fail(c, TO_E_INVALID, "max_iters must be >= 1");
  const double t0 = now_ms();
  HIPCHK(hipSetDevice(c->device));
  const size_t nel = c->g.nel;
  double *dc = d_work, *dcf = d_work + nel;
  if (sp->init_uniform) HIPCHK(launch_set(d_x, nel, sp->vf, c->stream));
  int it = 0, converged = 0, inner = 0;
  double cval = 0.0, change = 0.0, volume = 0.0;
  to_status st = TO_OK;
  const char *step = "";
  while (it < sp->max_iters) {
    to_solve_info si{};
    step = "state solve";
    st = to_solve(c, d_x, it == 0 ? nullptr : d_u, d_u, &si);
    inner += si.inner_iters;
    if (st != TO_OK) break;
    step = "compliance and sensitivity";
    st = to_compliance_sensitivity(c, d_x, d_u, &cval, dc);
    if (st != TO_OK) break;
    step = "sensitivity filter";
    st = to_filter(c, sp->rmin, TO_FILTER_SENS, d_x, dc, dcf);
    if (st != TO_OK) break;
    step = "OC update";
    to_oc_info oi{};
    st = to_oc_update(c, d_x, dcf, sp->vf, sp->move, sp->eta, d_x, &oi);
    if (st != TO_OK) break;
    if (h_c_hist) h_c_hist[it] = cval;
    ++it;
    change = oi.change;
    volume = oi.volume;
    if (change <= sp->change_tol) {
      converged = 1;
      break;
    }
  }
  if (info) {
    info->iters = it;
    info->converged = converged;
    info->inner_iters = inner;
    info->reserved = 0;
    info->c = cval;
    info->change = change;
    info->volume = volume;
    info->ms = now_ms() - t0;
  }
  if (st != TO_OK)
    return fail(c, st, "SIMP iteration " + std::to_string(it + 1) + ", " + step + ": " + c->err);
  return TO_OK;
}

to_status to_matvec(to_ctx *c, const double *d_x, const double *d_u, double *d_y) {
  if (!c) return fail(nullptr, TO_E_INVALID, "ctx is NULL");
  if (!d_u || !d_y) return fail(c, TO_E_INVALID, "d_u and d_y are required");
  if (d_u == d_y) return fail(c, TO_E_INVALID, "d_y must not alias d_u");
  HIPCHK(hipSetDevice(c->device));
  if (d_x) {
    to_status st = prepare_moduli(c, d_x, false);
    if (st != TO_OK) return st;
  }
  MvArgs<double> a{};
  a.nelx = c->g.nelx;
  a.nely = c->g.nely;
  a.nelz = c->g.nelz;
  a.kz = c->kz;
  a.E = c->E64;
  a.in = d_u;
  a.out = d_y;
  a.mask = c->mask;
  a.k = c->k64;
  HIPCHK((launch_matvec<double, MV_APPLY>(a, nullptr, c->stream)));
  return TO_OK;
}

to_status to_matvec_f32(to_ctx *c, const double *d_x, const float *d_u, float *d_y) {
  if (!c) return fail(nullptr, TO_E_INVALID, "ctx is NULL");
  if (!d_u || !d_y) return fail(c, TO_E_INVALID, "d_u and d_y are required");
  if ((const void *)d_u == (const void *)d_y) return fail(c, TO_E_INVALID, "d_y must not alias d_u");
  HIPCHK(hipSetDevice(c->device));
  if (d_x) {
    to_status st = prepare_moduli(c, d_x, false);
    if (st != TO_OK) return st;
  }
  MvArgs<float> a{};
  a.nelx = c->g.nelx;
  a.nely = c->g.nely;
  a.nelz = c->g.nelz;
  a.kz = c->mA ? c->kz_mf : c->kz;
  a.E = c->E32;
  a.in = d_u;
  a.out = d_y;
  a.mask = c->mask;
  a.k = c->k32;
  a.mA = c->mA;
  a.mscale = c->mscale;
  if (c->mA) HIPCHK(launch_matvec_mfma(a, nullptr, c->stream));
  else HIPCHK((launch_matvec<float, MV_APPLY>(a, nullptr, c->stream)));
  return TO_OK;
}

to_status to_profile(to_ctx *c, int32_t enable, double *h_ms, int64_t *h_count) {
  if (!c) return fail(nullptr, TO_E_INVALID, "ctx is NULL");
  if (h_ms) *h_ms = c->prof_ms;
  if (h_count) *h_count = c->prof_count;
  c->prof = enable != 0;
  c->prof_ms = 0.0;
  c->prof_count = 0;
  c->ev_used = c->ev_done = 0;
  return TO_OK;
}

}  // extern "C"
