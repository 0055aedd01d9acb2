// Level-set evolution and reinitialisation on the node grid (Sec. 2.2.7,
// Eqs. 21-22; Sec. 2.2.8, Eqs. 23-24): forward Euler in time, first-order
// Godunov upwinding in space.
//
// With one-sided differences D-, D+ along each axis (the missing neighbour at
// a box face is the node itself, so the difference across the face is 0):
//   g+ = sqrt(sum over x, y, z of max(D-, 0)^2 + min(D+, 0)^2)   (speed > 0)
//   g- = sqrt(sum over x, y, z of min(D-, 0)^2 + max(D+, 0)^2)   (speed < 0)
//   evolution:        phi <- phi - dt (max(v, 0) g+ + min(v, 0) g-)
//   reinitialisation: phi <- phi - dtau (max(S, 0)(g+ - 1) + min(S, 0)(g- - 1)),
//                     S = phi / sqrt(phi^2 + h^2 |grad phi|^2), |grad phi|
//                     from central differences, S = 0 where that root is 0.
// Each update reads only the previous field, so a step is one launch that
// reads one buffer and writes the other.  Floating-point contraction is off
// and every expression keeps the order written above, so the result is the
// same number for number on any device that rounds IEEE operations
// correctly.
#include <algorithm>
#include <cmath>
#include <cstdint>

#include "common.h"
#include "device_common.h"

#pragma clang fp contract(off)

namespace topo {

constexpr int LS_BLOCK = 256;
// blocks per launch the plane chunks aim at (measured on the 257x129x129 node
// grid: the evolution step, light on arithmetic, gains from shorter chunks;
// the reinitialisation step, with two roots and a division per node, from
// fewer, longer ones)
constexpr long long LS_ADVECT_BLOCKS = 4096, LS_REINIT_BLOCKS = 2048;

struct Nb {
  double p, xm, xp, ym, yp, zm, zp;
};

// Walks planes k0 .. k1 - 1 of column (i, j), keeping the planes below, at and
// above the current node in registers; x and y neighbours come from the same
// plane (cache hits within the block's tile).  upd(neighbourhood, node index)
// returns the node's |change|; the largest is returned.
template <class F>
__device__ __forceinline__ double ls_march(const double *__restrict__ f, int i, int j, int k0,
                                           int k1, int NX, int NY, int NZ, F &&upd) {
  const size_t sy = (size_t)NX, sz = (size_t)NX * NY;
  size_t n = (size_t)i + sy * ((size_t)j + (size_t)NY * k0);
  double pc = f[n];
  double pm = k0 > 0 ? f[n - sz] : pc;
  double change = 0.0;
  for (int k = k0; k < k1; ++k, n += sz) {
    const double pn = k < NZ - 1 ? f[n + sz] : pc;
    Nb a;
    a.p = pc;
    a.zm = pm;
    a.zp = pn;
    a.xm = i > 0 ? f[n - 1] : pc;
    a.xp = i < NX - 1 ? f[n + 1] : pc;
    a.ym = j > 0 ? f[n - sy] : pc;
    a.yp = j < NY - 1 ? f[n + sy] : pc;
    change = fmax(change, upd(a, n));
    pm = pc;
    pc = pn;
  }
  return change;
}

// Difference quotient (a - b) / d.  When h is a power of two, P2 multiplies
// by the exact reciprocal instead, which gives the same number (scaling by a
// power of two is exact, or rounds the same exact value in the subnormal
// range) without a division sequence.
template <bool P2>
__device__ __forceinline__ double dq_over(double num, double d, double inv_d) {
  return P2 ? num * inv_d : num / d;
}

// Sums of squares of the upwind one-sided differences for a positive (sp)
// and a negative (sm) speed, taken x, then y, then z.  Only one of
// g+ = sqrt(sp) and g- = sqrt(sm) enters an update: for a speed w > 0,
// max(w, 0) g+ + min(w, 0) g- is w g+ plus an exact zero, and likewise for
// w < 0, so the callers take a single root.
template <bool P2>
__device__ __forceinline__ void godunov_sums(const Nb &a, double h, double inv_h, double &sp,
                                             double &sm) {
  double dm, dq, t;
  sp = 0.0;
  sm = 0.0;
  dm = dq_over<P2>(a.p - a.xm, h, inv_h);
  dq = dq_over<P2>(a.xp - a.p, h, inv_h);
  t = fmax(dm, 0.0); sp = sp + t * t; t = fmin(dq, 0.0); sp = sp + t * t;
  t = fmin(dm, 0.0); sm = sm + t * t; t = fmax(dq, 0.0); sm = sm + t * t;
  dm = dq_over<P2>(a.p - a.ym, h, inv_h);
  dq = dq_over<P2>(a.yp - a.p, h, inv_h);
  t = fmax(dm, 0.0); sp = sp + t * t; t = fmin(dq, 0.0); sp = sp + t * t;
  t = fmin(dm, 0.0); sm = sm + t * t; t = fmax(dq, 0.0); sm = sm + t * t;
  dm = dq_over<P2>(a.p - a.zm, h, inv_h);
  dq = dq_over<P2>(a.zp - a.p, h, inv_h);
  t = fmax(dm, 0.0); sp = sp + t * t; t = fmin(dq, 0.0); sp = sp + t * t;
  t = fmin(dm, 0.0); sm = sm + t * t; t = fmax(dq, 0.0); sm = sm + t * t;
}

__device__ __forceinline__ double wave_max_u(double v) {
  for (int o = 32; o > 0; o >>= 1) v = fmax(v, __shfl_xor(v, o));
  return v;
}

// one block max of a non-negative value into one word of a slot set (bit
// patterns of non-negative doubles order like the doubles)
__device__ __forceinline__ void block_max_to(double v, unsigned long long *set) {
  __shared__ double sh[LS_BLOCK / 64];
  const int t = threadIdx.x;
  v = wave_max_u(v);
  if ((t & 63) == 0) sh[t >> 6] = v;
  __syncthreads();
  if (t == 0) {
    double m = 0.0;
    for (int w = 0; w < LS_BLOCK / 64; ++w) m = fmax(m, sh[w]);
    if (m > 0.0)
      atomicMax(&set[(blockIdx.x % LS_SLOTS) * LS_SLOT_STRIDE],
                (unsigned long long)__double_as_longlong(m));
  }
}

// checks phi (and v) for NaN/Inf (flags[F_BADX] bit 1) and takes max|v|
__global__ __launch_bounds__(256) void k_ls_check(const double *__restrict__ phi,
                                                  const double *__restrict__ v, size_t n,
                                                  int *__restrict__ flags,
                                                  unsigned long long *__restrict__ vmax) {
  int bad = 0;
  double m = 0.0;
  for (size_t e = blockIdx.x * (size_t)blockDim.x + threadIdx.x; e < n;
       e += (size_t)gridDim.x * blockDim.x) {
    if (!isfinite(phi[e])) bad = 2;
    if (v) {
      const double ve = v[e];
      if (!isfinite(ve)) bad = 2;
      else m = fmax(m, fabs(ve));
    }
  }
  if (bad) atomicOr(&flags[F_BADX], bad);
  __shared__ double sh[4];
  m = wave_max_u(m);
  if ((threadIdx.x & 63) == 0) sh[threadIdx.x >> 6] = m;
  __syncthreads();
  if (threadIdx.x == 0) {
    double mm = 0.0;
    for (int w = 0; w < (int)(blockDim.x >> 6); ++w) mm = fmax(mm, sh[w]);
    if (mm > 0.0) atomicMax(vmax, (unsigned long long)__double_as_longlong(mm));
  }
}

// The grid is 1D over tiles: a run of LS_BLOCK consecutive nodes of one z
// plane (row-major, so a run may wrap from one y row to the next) by kz
// planes, ordered run, then z-chunk.  Every lane but those past a plane's
// last node holds a node, whatever NX is, and loads stay contiguous;
// xcd_local gives every XCD one contiguous range of tiles, so the rows and
// planes beside a run were mostly brought into the same L2 by its
// neighbours.
struct Tile {
  int i, j, k0, k1;
  bool valid;
};
__device__ __forceinline__ Tile ls_tile(int NX, int NY, int NZ, int kz) {
  const int plane = NX * NY;
  const int nseg = (plane + LS_BLOCK - 1) / LS_BLOCK;
  const int nkz = (NZ + kz - 1) / kz;
  const int lb = xcd_local((int)blockIdx.x, nseg * nkz);
  const int seg = lb % nseg, tz = lb / nseg;
  const int p = seg * LS_BLOCK + (int)threadIdx.x;
  Tile t;
  t.valid = p < plane;
  t.j = p / NX;
  t.i = p - t.j * NX;
  t.k0 = tz * kz;
  t.k1 = min(t.k0 + kz, NZ);
  return t;
}

template <bool P2>
__global__ __launch_bounds__(LS_BLOCK) void k_ls_advect(int NX, int NY, int NZ, int kz,
                                                         double h, double inv_h, double dt,
                                                         const double *__restrict__ in,
                                                         const double *__restrict__ v,
                                                         double *__restrict__ out) {
  const Tile tl = ls_tile(NX, NY, NZ, kz);
  const int i = tl.i, j = tl.j, k0 = tl.k0, k1 = tl.k1;
  if (!tl.valid) return;
  ls_march(in, i, j, k0, k1, NX, NY, NZ, [&](const Nb &a, size_t n) {
    double sp, sm;
    godunov_sums<P2>(a, h, inv_h, sp, sm);
    const double ve = v[n];
    const double g = sqrt(ve > 0.0 ? sp : sm);
    out[n] = ve == 0.0 ? a.p : a.p - dt * (ve * g);
    return 0.0;
  });
}

// Launch k computes pseudo-step k + 1 from `in` into `out`, with its largest
// |change| spread over slot set k % 3 (LS_SLOTS words).  It first takes the
// previous step's largest change from set (k - 1) % 3 (first wave: one word
// per lane, then a wave max): below tol the loop has converged; at
// k == max_steps without that it is capped.  state[0]: 0 running,
// 1 converged, 2 capped; state[1]: steps computed; state[2]: the last step's
// largest |change|; while running, state[3]: the previous step's largest
// |change| (written by every launch).  Only block 0 writes the state, and its
// first wave also clears set (k + 1) % 3 for the next launch (that set was
// last read by launch k - 1).
template <bool P2>
__global__ __launch_bounds__(LS_BLOCK) void k_ls_reinit(
    int NX, int NY, int NZ, int kz, double h, double inv_h, double dtau, double tol, int max_steps,
    int k_launch, const double *__restrict__ in, double *__restrict__ out,
    unsigned long long *__restrict__ slots, double *__restrict__ state) {
  __shared__ double prev_sh;
  const int t = threadIdx.x;
  const bool block0 = blockIdx.x == 0;
  const size_t set = (size_t)LS_SLOTS * LS_SLOT_STRIDE;
  if (t < 64) {
    double m = 0.0;
    if (k_launch > 0)
      m = __longlong_as_double(
          (long long)slots[((k_launch - 1) % 3) * set + (size_t)t * LS_SLOT_STRIDE]);
    m = wave_max_u(m);
    if (t == 0) prev_sh = k_launch > 0 ? m : INFINITY;
    if (block0) slots[((k_launch + 1) % 3) * set + (size_t)t * LS_SLOT_STRIDE] = 0ull;
  }
  __syncthreads();
  const double st = state[0];
  const double prev = prev_sh;
  const bool conv = prev < tol;
  const bool capped = !conv && k_launch >= max_steps;
  if (block0 && t == 0 && st == 0.0) {
    if (conv || capped) {
      state[0] = conv ? 1.0 : 2.0;
      state[1] = (double)k_launch;
      state[2] = prev;
    } else {
      state[3] = prev;  // progress, for the host's choice of batch
    }
  }
  if (st != 0.0 || conv || capped) return;
  const Tile tl = ls_tile(NX, NY, NZ, kz);
  const int i = tl.i, j = tl.j, k0 = tl.k0, k1 = tl.k1;
  double change = 0.0;
  if (tl.valid)
    change = ls_march(in, i, j, k0, k1, NX, NY, NZ, [&](const Nb &a, size_t n) {
      double sp, sm;
      godunov_sums<P2>(a, h, inv_h, sp, sm);
      const double h2 = 2.0 * h, inv_h2 = 0.5 * inv_h;
      const double cx = dq_over<P2>(a.xp - a.xm, h2, inv_h2),
                   cy = dq_over<P2>(a.yp - a.ym, h2, inv_h2),
                   cz = dq_over<P2>(a.zp - a.zm, h2, inv_h2);
      const double g2 = cx * cx + cy * cy + cz * cz;
      const double den = sqrt(a.p * a.p + (h * h) * g2);
      const double s = den > 0.0 ? a.p / den : 0.0;
      const double g = sqrt(s > 0.0 ? sp : sm);
      const double nv = s == 0.0 ? a.p : a.p - dtau * (s * (g - 1.0));
      out[n] = nv;
      return fabs(nv - a.p);
    });
  block_max_to(change, &slots[(k_launch % 3) * set]);
}

// planes per block: about `target` blocks (2048 of 4 waves fill the chip's
// 1024 SIMDs twice over), at most 16 planes
static int ls_kz(const Grid &g, long long target) {
  const long long runs = ((long long)(g.nelx + 1) * (g.nely + 1) + LS_BLOCK - 1) / LS_BLOCK;
  long long kz = (long long)(g.nelz + 1) * runs / target;
  return (int)std::max(1LL, std::min(16LL, kz));
}

static dim3 ls_grid(const Grid &g, int kz) {
  const long long runs = ((long long)(g.nelx + 1) * (g.nely + 1) + LS_BLOCK - 1) / LS_BLOCK;
  return dim3((unsigned)(runs * ((g.nelz + 1 + kz - 1) / kz)));
}

hipError_t launch_ls_check(const Grid &g, const double *phi, const double *v, int *flags,
                           unsigned long long *vmax, hipStream_t s) {
  size_t b = (g.nn + 255) / 256;
  if (b > 2048) b = 2048;
  hipLaunchKernelGGL(k_ls_check, dim3((unsigned)b), dim3(256), 0, s, phi, v, g.nn, flags, vmax);
  return hipGetLastError();
}

static bool pow2(double h) {
  int e = 0;
  return std::frexp(h, &e) == 0.5;
}

hipError_t launch_ls_advect(const Grid &g, double h, double dt, const double *in, const double *v,
                            double *out, hipStream_t s) {
  const int kz = ls_kz(g, LS_ADVECT_BLOCKS);
  if (pow2(h))
    hipLaunchKernelGGL(k_ls_advect<true>, ls_grid(g, kz), dim3(LS_BLOCK), 0, s, g.nelx + 1,
                       g.nely + 1, g.nelz + 1, kz, h, 1.0 / h, dt, in, v, out);
  else
    hipLaunchKernelGGL(k_ls_advect<false>, ls_grid(g, kz), dim3(LS_BLOCK), 0, s, g.nelx + 1,
                       g.nely + 1, g.nelz + 1, kz, h, 1.0 / h, dt, in, v, out);
  return hipGetLastError();
}

hipError_t launch_ls_reinit(const Grid &g, double h, double dtau, double tol, int max_steps,
                            int k, const double *in, double *out, unsigned long long *slots,
                            double *state, hipStream_t s) {
  const int kz = ls_kz(g, LS_REINIT_BLOCKS);
  if (pow2(h))
    hipLaunchKernelGGL(k_ls_reinit<true>, ls_grid(g, kz), dim3(LS_BLOCK), 0, s, g.nelx + 1,
                       g.nely + 1, g.nelz + 1, kz, h, 1.0 / h, dtau, tol, max_steps, k, in, out,
                       slots, state);
  else
    hipLaunchKernelGGL(k_ls_reinit<false>, ls_grid(g, kz), dim3(LS_BLOCK), 0, s, g.nelx + 1,
                       g.nely + 1, g.nelz + 1, kz, h, 1.0 / h, dtau, tol, max_steps, k, in, out,
                       slots, state);
  return hipGetLastError();
}

}  // namespace topo
