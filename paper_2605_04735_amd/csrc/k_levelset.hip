// Level-set evolution and reinitialisation on the node grid (Sec. 2.2.4,
// Eqs. 21-22; Sec. 2.2.5, Eqs. 23-24): forward Euler in time, first-order
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
#include <cstdint>

#include "common.h"
#include "device_common.h"

#pragma clang fp contract(off)

namespace topo {

constexpr int LSX = 64, LSY = 4;

struct Nb {
  double p, xm, xp, ym, yp, zm, zp;
};

__device__ __forceinline__ Nb ls_load(const double *__restrict__ f, int i, int j, int k, int NX,
                                      int NY, int NZ) {
  const size_t sy = (size_t)NX, sz = (size_t)NX * NY;
  const size_t n = (size_t)i + sy * ((size_t)j + (size_t)NY * k);
  Nb r;
  r.p = f[n];
  r.xm = i > 0 ? f[n - 1] : r.p;
  r.xp = i < NX - 1 ? f[n + 1] : r.p;
  r.ym = j > 0 ? f[n - sy] : r.p;
  r.yp = j < NY - 1 ? f[n + sy] : r.p;
  r.zm = k > 0 ? f[n - sz] : r.p;
  r.zp = k < NZ - 1 ? f[n + sz] : r.p;
  return r;
}

// (g+, g-) with the sums taken x, then y, then z
__device__ __forceinline__ void godunov(const Nb &a, double h, double &gp, double &gm) {
  double sp = 0.0, sm = 0.0, dm, dq, t;
  dm = (a.p - a.xm) / h;
  dq = (a.xp - a.p) / h;
  t = fmax(dm, 0.0); sp = sp + t * t; t = fmin(dq, 0.0); sp = sp + t * t;
  t = fmin(dm, 0.0); sm = sm + t * t; t = fmax(dq, 0.0); sm = sm + t * t;
  dm = (a.p - a.ym) / h;
  dq = (a.yp - a.p) / h;
  t = fmax(dm, 0.0); sp = sp + t * t; t = fmin(dq, 0.0); sp = sp + t * t;
  t = fmin(dm, 0.0); sm = sm + t * t; t = fmax(dq, 0.0); sm = sm + t * t;
  dm = (a.p - a.zm) / h;
  dq = (a.zp - a.p) / h;
  t = fmax(dm, 0.0); sp = sp + t * t; t = fmin(dq, 0.0); sp = sp + t * t;
  t = fmin(dm, 0.0); sm = sm + t * t; t = fmax(dq, 0.0); sm = sm + t * t;
  gp = sqrt(sp);
  gm = sqrt(sm);
}

__device__ __forceinline__ double wave_max_u(double v) {
  for (int o = 32; o > 0; o >>= 1) v = fmax(v, __shfl_xor(v, o));
  return v;
}

// one block max of a non-negative value into *slot (bit patterns of
// non-negative doubles order like the doubles)
__device__ __forceinline__ void block_max_to(double v, unsigned long long *slot) {
  __shared__ double sh[LSX * LSY / 64];
  const int t = threadIdx.x + LSX * threadIdx.y;
  v = wave_max_u(v);
  if ((t & 63) == 0) sh[t >> 6] = v;
  __syncthreads();
  if (t == 0) {
    double m = 0.0;
    for (int w = 0; w < LSX * LSY / 64; ++w) m = fmax(m, sh[w]);
    if (m > 0.0) atomicMax(slot, (unsigned long long)__double_as_longlong(m));
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

__global__ __launch_bounds__(LSX * LSY) void k_ls_advect(int NX, int NY, int NZ, double h,
                                                         double dt,
                                                         const double *__restrict__ in,
                                                         const double *__restrict__ v,
                                                         double *__restrict__ out) {
  const int i = blockIdx.x * LSX + threadIdx.x, j = blockIdx.y * LSY + threadIdx.y,
            k = blockIdx.z;
  if (i >= NX || j >= NY) return;
  const Nb a = ls_load(in, i, j, k, NX, NY, NZ);
  double gp, gm;
  godunov(a, h, gp, gm);
  const size_t n = (size_t)i + (size_t)NX * ((size_t)j + (size_t)NY * k);
  const double ve = v[n];
  out[n] = a.p - dt * (fmax(ve, 0.0) * gp + fmin(ve, 0.0) * gm);
}

// Launch k computes pseudo-step k + 1 from `in` into `out`, with its largest
// |change| in slots[k % 3].  It first reads the previous step's slot: below
// tol the loop has converged; at k == max_steps without that it is capped.
// state[0]: 0 running, 1 converged, 2 capped; state[1]: steps computed;
// state[2]: the last step's largest |change|.  Only block 0 writes the state,
// and it also clears slots[(k + 1) % 3] for the next launch (that slot was
// last read by launch k - 1).
__global__ __launch_bounds__(LSX * LSY) void k_ls_reinit(
    int NX, int NY, int NZ, double h, double dtau, double tol, int max_steps, int k_launch,
    const double *__restrict__ in, double *__restrict__ out,
    unsigned long long *__restrict__ slots, double *__restrict__ state) {
  const bool lead = blockIdx.x == 0 && blockIdx.y == 0 && blockIdx.z == 0 && threadIdx.x == 0 &&
                    threadIdx.y == 0;
  const double st = state[0];
  const double prev =
      k_launch > 0 ? __longlong_as_double((long long)slots[(k_launch - 1) % 3]) : INFINITY;
  const bool conv = prev < tol;
  const bool capped = !conv && k_launch >= max_steps;
  if (lead) {
    if (st == 0.0 && (conv || capped)) {
      state[0] = conv ? 1.0 : 2.0;
      state[1] = (double)k_launch;
      state[2] = prev;
    }
    slots[(k_launch + 1) % 3] = 0ull;
  }
  if (st != 0.0 || conv || capped) return;
  const int i = blockIdx.x * LSX + threadIdx.x, j = blockIdx.y * LSY + threadIdx.y,
            k = blockIdx.z;
  double change = 0.0;
  if (i < NX && j < NY) {
    const Nb a = ls_load(in, i, j, k, NX, NY, NZ);
    double gp, gm;
    godunov(a, h, gp, gm);
    const double cx = (a.xp - a.xm) / (2.0 * h), cy = (a.yp - a.ym) / (2.0 * h),
                 cz = (a.zp - a.zm) / (2.0 * h);
    const double g2 = cx * cx + cy * cy + cz * cz;
    const double den = sqrt(a.p * a.p + (h * h) * g2);
    const double s = den > 0.0 ? a.p / den : 0.0;
    const double nv = a.p - dtau * (fmax(s, 0.0) * (gp - 1.0) + fmin(s, 0.0) * (gm - 1.0));
    out[(size_t)i + (size_t)NX * ((size_t)j + (size_t)NY * k)] = nv;
    change = fabs(nv - a.p);
  }
  block_max_to(change, &slots[k_launch % 3]);
}

static dim3 ls_grid(const Grid &g) {
  return dim3((unsigned)((g.nelx + 1 + LSX - 1) / LSX), (unsigned)((g.nely + 1 + LSY - 1) / LSY),
              (unsigned)(g.nelz + 1));
}

hipError_t launch_ls_check(const Grid &g, const double *phi, const double *v, int *flags,
                           unsigned long long *vmax, hipStream_t s) {
  size_t b = (g.nn + 255) / 256;
  if (b > 2048) b = 2048;
  hipLaunchKernelGGL(k_ls_check, dim3((unsigned)b), dim3(256), 0, s, phi, v, g.nn, flags, vmax);
  return hipGetLastError();
}

hipError_t launch_ls_advect(const Grid &g, double h, double dt, const double *in, const double *v,
                            double *out, hipStream_t s) {
  hipLaunchKernelGGL(k_ls_advect, ls_grid(g), dim3(LSX, LSY), 0, s, g.nelx + 1, g.nely + 1,
                     g.nelz + 1, h, dt, in, v, out);
  return hipGetLastError();
}

hipError_t launch_ls_reinit(const Grid &g, double h, double dtau, double tol, int max_steps,
                            int k, const double *in, double *out, unsigned long long *slots,
                            double *state, hipStream_t s) {
  hipLaunchKernelGGL(k_ls_reinit, ls_grid(g), dim3(LSX, LSY), 0, s, g.nelx + 1, g.nely + 1,
                     g.nelz + 1, h, dtau, tol, max_steps, k, in, out, slots, state);
  return hipGetLastError();
}

}  // namespace topo
