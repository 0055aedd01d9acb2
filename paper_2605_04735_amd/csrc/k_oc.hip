// Optimality-criteria design update of the SIMP stage (Sec. 2.1, with the
// set-up of Sec. 4), in its textbook form.  For a multiplier lam every element
// takes
//   x_new = clamp(x (max(-dc, 0) / lam)^eta, [max(0, x - move), min(1, x + move)])
// (unit volume derivative: the voxels are equal), and lam is found by
// bisection on [0, l2_0]: the midpoint's design is evaluated, the lower end
// moves up when it holds more than V_f n of material, else the upper end moves
// down, until (l2 - l1) / (l1 + l2) <= tol.  The design of the last midpoint
// evaluated is the update.
//
// The bisection stays on the device, one launch per midpoint.  A launch first
// finishes the previous midpoint: every block sums the previous launch's
// per-block volume partials in one fixed order, so all blocks reach the same
// total and take the same decision.  Then it tests the bracket and, if the
// loop goes on, evaluates its own midpoint's partials.  The bracket state and
// the partials alternate between two buffers, so no launch writes what a
// block of the same launch may still read.  Launches after the loop ended
// return at once.
#include "common.h"
#include "device_common.h"

namespace topo {

__device__ __forceinline__ double oc_candidate(double x, double dc, double lam, double move,
                                               double eta) {
  const double b = fmax(-dc, 0.0) / lam;
  const double t = x * (eta == 0.5 ? sqrt(b) : pow(b, eta));
  return fmax(fmax(0.0, x - move), fmin(fmin(1.0, x + move), t));
}

__device__ __forceinline__ double wave_max_d(double v) {
  for (int o = 32; o > 0; o >>= 1) v = fmax(v, __shfl_xor(v, o));
  return v;
}

// Sums the previous midpoint's partials (same order in every block), updates
// the bracket, tests it, and evaluates the next midpoint.  The first launch
// starts from [0, l2_0] and also checks the inputs (flags[F_BADX] bits 0/1
// for x outside [0, 1] / non-finite, flags[F_BADG] for a non-finite dc).
__global__ __launch_bounds__(OC_THREADS) void k_oc_step(
    const double *__restrict__ x, const double *__restrict__ dc, size_t nel, double move,
    double eta, double target, double tol, double l2_0, int max_steps,
    const double *__restrict__ st_in, double *__restrict__ st_out,
    const double *__restrict__ part_in, double *__restrict__ part_out, int nb, int first,
    int *__restrict__ flags) {
  __shared__ double sh[OC_THREADS / 64];
  __shared__ double tot;
  double l1 = 0.0, l2 = l2_0, lam = 0.0, done = 0.0, steps = 0.0;
  if (!first) {
    l1 = st_in[OC_L1];
    l2 = st_in[OC_L2];
    lam = st_in[OC_LAM];
    done = st_in[OC_DONE];
    steps = st_in[OC_STEPS];
  }
  if (done == 0.0) {
    if (!first) {
      double v = 0.0;
      for (int i = threadIdx.x; i < nb; i += OC_THREADS) v += part_in[i];
      const double t = block_sum_d(v, sh);
      if (threadIdx.x == 0) tot = t;
      __syncthreads();
      if (tot > target) l1 = lam;
      else l2 = lam;
    }
    if (!((l2 - l1) / (l1 + l2) > tol)) {
      done = 1.0;
    } else if (steps >= (double)max_steps) {
      done = 2.0;
    } else {
      lam = 0.5 * (l2 + l1);
      steps += 1.0;
    }
  }
  if (blockIdx.x == 0 && threadIdx.x == 0) {
    st_out[OC_L1] = l1;
    st_out[OC_L2] = l2;
    st_out[OC_LAM] = lam;
    st_out[OC_DONE] = done;
    st_out[OC_STEPS] = steps;
  }
  if (done != 0.0) return;
  double s = 0.0;
  int bad = 0, badg = 0;
  for (size_t e = (size_t)blockIdx.x * OC_THREADS + threadIdx.x; e < nel;
       e += (size_t)gridDim.x * OC_THREADS) {
    const double xe = x[e], de = dc[e];
    if (first) {
      if (!isfinite(xe)) bad |= 2;
      else if (xe < 0.0 || xe > 1.0) bad |= 1;
      if (!isfinite(de)) badg = 1;
    }
    s += oc_candidate(xe, de, lam, move, eta);
  }
  if (bad) atomicOr(&flags[F_BADX], bad);
  if (badg) atomicOr(&flags[F_BADG], 1);
  const double t = block_sum_d(s, sh);
  if (threadIdx.x == 0) part_out[blockIdx.x] = t;
}

// Writes the design of the last midpoint, with per-block partials of its
// volume (part[b]) and of max |x_new - x| (part[OC_MAXB + b]).  x_new may
// alias x: each element is read and written by the same thread.
__global__ __launch_bounds__(OC_THREADS) void k_oc_apply(const double *x,
                                                         const double *__restrict__ dc,
                                                         double *xnew, size_t nel, double move,
                                                         double eta,
                                                         const double *__restrict__ st,
                                                         double *__restrict__ part) {
  __shared__ double sh[OC_THREADS / 64];
  __shared__ double shm[OC_THREADS / 64];
  const double lam = st[OC_LAM];
  double s = 0.0, m = 0.0;
  for (size_t e = (size_t)blockIdx.x * OC_THREADS + threadIdx.x; e < nel;
       e += (size_t)gridDim.x * OC_THREADS) {
    const double xe = x[e];
    const double v = oc_candidate(xe, dc[e], lam, move, eta);
    xnew[e] = v;
    s += v;
    m = fmax(m, fabs(v - xe));
  }
  m = wave_max_d(m);
  if ((threadIdx.x & 63) == 0) shm[threadIdx.x >> 6] = m;
  const double t = block_sum_d(s, sh);  // its barrier also publishes shm
  if (threadIdx.x == 0) {
    double mm = 0.0;
    for (int w = 0; w < OC_THREADS / 64; ++w) mm = fmax(mm, shm[w]);
    part[blockIdx.x] = t;
    part[OC_MAXB + blockIdx.x] = mm;
  }
}

// out: [0] lam, [1] max change, [2] volume sum, [3] midpoints, [4] done state
__global__ __launch_bounds__(OC_THREADS) void k_oc_finish(const double *__restrict__ st,
                                                          const double *__restrict__ part, int nb,
                                                          double *__restrict__ out) {
  __shared__ double sh[OC_THREADS / 64];
  __shared__ double shm[OC_THREADS / 64];
  double v = 0.0, m = 0.0;
  for (int i = threadIdx.x; i < nb; i += OC_THREADS) {
    v += part[i];
    m = fmax(m, part[OC_MAXB + i]);
  }
  m = wave_max_d(m);
  if ((threadIdx.x & 63) == 0) shm[threadIdx.x >> 6] = m;
  const double t = block_sum_d(v, sh);
  if (threadIdx.x == 0) {
    double mm = 0.0;
    for (int w = 0; w < OC_THREADS / 64; ++w) mm = fmax(mm, shm[w]);
    out[0] = st[OC_LAM];
    out[1] = mm;
    out[2] = t;
    out[3] = st[OC_STEPS];
    out[4] = st[OC_DONE];
  }
}

__global__ void k_set(double *__restrict__ p, size_t n, double v) {
  for (size_t i = blockIdx.x * (size_t)blockDim.x + threadIdx.x; i < n;
       i += (size_t)gridDim.x * blockDim.x)
    p[i] = v;
}

hipError_t launch_set(double *p, size_t n, double v, hipStream_t s) {
  size_t b = (n + 255) / 256;
  if (b > 4096) b = 4096;
  if (b < 1) b = 1;
  hipLaunchKernelGGL(k_set, dim3((unsigned)b), dim3(256), 0, s, p, n, v);
  return hipGetLastError();
}

int oc_blocks(size_t nel) {
  size_t b = (nel + 4 * OC_THREADS - 1) / (4 * OC_THREADS);
  if (b > (size_t)OC_MAXB) b = OC_MAXB;
  return b < 1 ? 1 : (int)b;
}

hipError_t launch_oc_steps(const double *x, const double *dc, size_t nel, double move, double eta,
                           double target, double tol, double l2_0, int max_steps, double *scratch,
                           int k0, int count, int *flags, hipStream_t s) {
  const int nb = oc_blocks(nel);
  for (int k = k0; k < k0 + count; ++k) {
    const int pi = k & 1, po = (k + 1) & 1;
    hipLaunchKernelGGL(k_oc_step, dim3(nb), dim3(OC_THREADS), 0, s, x, dc, nel, move, eta,
                       target, tol, l2_0, max_steps, scratch + OC_STATE_OFS + pi * OC_STATE,
                       scratch + OC_STATE_OFS + po * OC_STATE, scratch + pi * OC_MAXB,
                       scratch + po * OC_MAXB, nb, k == 0 ? 1 : 0, flags);
  }
  return hipGetLastError();
}

hipError_t launch_oc_apply(const double *x, const double *dc, double *xnew, size_t nel,
                           double move, double eta, double *scratch, int k, hipStream_t s) {
  const int nb = oc_blocks(nel);
  const double *st = scratch + OC_STATE_OFS + (k & 1) * OC_STATE;
  // the partials of the last midpoint are no longer needed: reuse both halves
  hipLaunchKernelGGL(k_oc_apply, dim3(nb), dim3(OC_THREADS), 0, s, x, dc, xnew, nel, move, eta,
                     st, scratch);
  hipLaunchKernelGGL(k_oc_finish, dim3(1), dim3(OC_THREADS), 0, s, st, scratch, nb,
                     scratch + OC_OUT_OFS);
  return hipGetLastError();
}

}  // namespace topo
