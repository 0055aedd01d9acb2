// Element/node set-up kernels (Eq. 1 moduli, Jacobi diagonal, boundary mask,
// load vector) and the streaming kernels of Jacobi-preconditioned CG with
// deterministic two-stage reductions.
#include <algorithm>

#include "common.h"
#include "device_common.h"

namespace topo {

__device__ __forceinline__ double block_sum(double v, double *sh) {
  v = wave_sum_d(v);
  const int lane = threadIdx.x & 63, w = threadIdx.x >> 6;
  if (lane == 0) sh[w] = v;
  __syncthreads();
  double r = 0.0;
  if (threadIdx.x == 0) {
    const int nw = (blockDim.x + 63) >> 6;
    for (int i = 0; i < nw; ++i) r += sh[i];
  }
  __syncthreads();
  return r;
}

// ---------------------------------------------------------------- Eq. 1
__global__ void k_modulus(size_t nel, const double *__restrict__ x, double E0, double Emin,
                          double penal, double *__restrict__ E64, float *__restrict__ E32,
                          int *__restrict__ flags) {
  int bad = 0;
  for (size_t e = blockIdx.x * (size_t)blockDim.x + threadIdx.x; e < nel;
       e += (size_t)gridDim.x * blockDim.x) {
    const double xe = x[e];
    if (!isfinite(xe)) bad |= 2;
    else if (xe < 0.0 || xe > 1.0) bad |= 1;
    const double E = Emin + pow(xe, penal) * (E0 - Emin);
    E64[e] = E;
    E32[e] = (float)E;
  }
  if (bad) atomicOr(&flags[F_BADX], bad);
}

hipError_t launch_modulus(const Grid &g, const double *x, double E0, double Emin, double penal,
                          double *E64, float *E32, int *flags, hipStream_t s) {
  int blocks = (int)((g.nel + 255) / 256);
  if (blocks > 4096) blocks = 4096;
  hipLaunchKernelGGL(k_modulus, dim3(blocks), dim3(256), 0, s, g.nel, x, E0, Emin, penal, E64,
                     E32, flags);
  return hipGetLastError();
}

// Jacobi diagonal: every diagonal entry of the unit-modulus k0 equals kd, so
// diag(K) at node n is kd * sum of the moduli of its (up to 8) elements.
__global__ void k_diag(int nelx, int nely, int nelz, const double *__restrict__ E64, double kd,
                       const uint8_t *__restrict__ mask, double *__restrict__ dinv64,
                       float *__restrict__ dinv32) {
  const int NX = nelx + 1, NY = nely + 1, NZ = nelz + 1;
  const size_t nn = (size_t)NX * NY * NZ;
  for (size_t n = blockIdx.x * (size_t)blockDim.x + threadIdx.x; n < nn;
       n += (size_t)gridDim.x * blockDim.x) {
    const int i = (int)(n % NX), j = (int)((n / NX) % NY), k = (int)(n / ((size_t)NX * NY));
    double s = 0.0;
    for (int bz = 0; bz < 2; ++bz)
      for (int by = 0; by < 2; ++by)
        for (int bx = 0; bx < 2; ++bx) {
          const int ei = i - 1 + bx, ej = j - 1 + by, ek = k - 1 + bz;
          if (ei >= 0 && ei < nelx && ej >= 0 && ej < nely && ek >= 0 && ek < nelz)
            s += E64[(size_t)ei + (size_t)nelx * ((size_t)ej + (size_t)nely * ek)];
        }
    const double d = (s > 0.0) ? 1.0 / (kd * s) : 0.0;
    dinv64[n] = d;
    dinv32[n] = (float)d;
  }
}

hipError_t launch_diag(const Grid &g, const double *E64, double kd, const uint8_t *mask,
                       double *dinv64, float *dinv32, hipStream_t s) {
  int blocks = (int)((g.nn + 255) / 256);
  if (blocks > 4096) blocks = 4096;
  hipLaunchKernelGGL(k_diag, dim3(blocks), dim3(256), 0, s, g.nelx, g.nely, g.nelz, E64, kd, mask,
                     dinv64, dinv32);
  return hipGetLastError();
}

// ---------------------------------------------------------------- BCs, load
__global__ void k_mask_builtin(int nelx, int nely, int nelz, int bc, uint8_t *__restrict__ mask) {
  const int NX = nelx + 1, NY = nely + 1, NZ = nelz + 1;
  const size_t nn = (size_t)NX * NY * NZ;
  for (size_t n = blockIdx.x * (size_t)blockDim.x + threadIdx.x; n < nn;
       n += (size_t)gridDim.x * blockDim.x) {
    const int i = (int)(n % NX), j = (int)((n / NX) % NY), k = (int)(n / ((size_t)NX * NY));
    unsigned m = 0;
    if (bc == 0) {         // cantilever: clamp x = 0
      if (i == 0) m = 7u;
    } else if (bc == 1) {  // MBB half beam
      if (i == 0) m |= 1u;
      if (i == nelx && k == 0) m |= 4u;
      if (i == 0 && j == 0 && k == 0) m |= 2u;
    } else if (bc == 3) {  // four corner squares 0.3 L x 0.3 L of x = 0
      const bool cy = 10 * j <= 3 * nely || 10 * j >= 7 * nely;
      const bool cz = 10 * k <= 3 * nelz || 10 * k >= 7 * nelz;
      if (i == 0 && cy && cz) m = 7u;
    } else {               // MBB with a one-element support strip
      if (i == 0) m |= 1u;
      if (i >= nelx - 1 && k == 0) m |= 4u;
      if (i == 0 && j == 0 && k == 0) m |= 2u;
    }
    mask[n] = (uint8_t)m;
  }
}

hipError_t launch_mask_builtin(const Grid &g, int bc, uint8_t *mask, hipStream_t s) {
  int blocks = (int)((g.nn + 255) / 256);
  if (blocks > 4096) blocks = 4096;
  hipLaunchKernelGGL(k_mask_builtin, dim3(blocks), dim3(256), 0, s, g.nelx, g.nely, g.nelz, bc,
                     mask);
  return hipGetLastError();
}

// Loaded quad of the corner-support cantilever (face x = Lx, quad (a, b) =
// (j, k)) or of the strip MBB (face z = Lz, quad (a, b) = (i, j)): tagged when
// 25 d2 <= thr, with 4 d2 the squared distance of its centroid to the region's
// centre in half-element units.
__device__ __forceinline__ bool quad_tagged(int bc, int a, int b, int nely, int nelz, long long thr) {
  long long d2;
  if (bc == 3) d2 = (long long)(2 * a + 1 - nely) * (2 * a + 1 - nely) +
                    (long long)(2 * b + 1 - nelz) * (2 * b + 1 - nelz);
  else d2 = (long long)(2 * a + 1) * (2 * a + 1) + (long long)(2 * b + 1 - nely) * (2 * b + 1 - nely);
  return 25 * d2 <= thr;
}

__global__ void k_load_builtin(int nelx, int nely, int nelz, int bc, double load_total,
                               long long thr, int nq, const uint8_t *__restrict__ mask,
                               double *__restrict__ f) {
  const int NX = nelx + 1, NY = nely + 1, NZ = nelz + 1;
  const size_t nn = (size_t)NX * NY * NZ;
  for (size_t n = blockIdx.x * (size_t)blockDim.x + threadIdx.x; n < nn;
       n += (size_t)gridDim.x * blockDim.x) {
    const int i = (int)(n % NX), j = (int)((n / NX) % NY), k = (int)(n / ((size_t)NX * NY));
    double fz = 0.0;
    if (bc == 0 || bc == 1) {
      const bool on_edge = (bc == 0) ? (i == nelx && k == 0) : (i == 0 && k == nelz);
      if (on_edge) {
        const double w = (j == 0 || j == nely) ? 0.5 : 1.0;
        fz = -(load_total * w) / (double)nely;
      }
    } else {
      // quarter shares of the tagged quads that touch the node
      const bool on_face = (bc == 3) ? (i == nelx) : (k == nelz);
      if (on_face) {
        const int a = (bc == 3) ? j : i, b = (bc == 3) ? k : j;
        const int na = (bc == 3) ? nely : nelx, nb = (bc == 3) ? nelz : nely;
        int c = 0;
        for (int da = -1; da <= 0; ++da)
          for (int db = -1; db <= 0; ++db) {
            const int qa = a + da, qb = b + db;
            if (qa >= 0 && qa < na && qb >= 0 && qb < nb &&
                quad_tagged(bc, qa, qb, nely, nelz, thr))
              ++c;
          }
        if (c) fz = -(load_total * (double)c) / (double)(4 * nq);
      }
    }
    const unsigned m = mask[n];
    f[3 * n + 0] = 0.0;
    f[3 * n + 1] = 0.0;
    f[3 * n + 2] = (m & 4u) ? 0.0 : fz;
  }
}

hipError_t launch_load_builtin(const Grid &g, int bc, double load_total, const uint8_t *mask,
                               double *f, hipStream_t s) {
  // the loaded region of bcs 3 and 4: threshold and quad count, by the same
  // integer test as the kernel (on grids too coarse for any centroid to fall
  // inside, the quads nearest the centre)
  long long thr = 0;
  int nq = 0;
  if (bc == 3 || bc == 4) {
    const long long m = std::min(g.nely, g.nelz);
    const int na = bc == 3 ? g.nely : g.nelx, nb = bc == 3 ? g.nelz : g.nely;
    long long dmin = -1;
    auto d2of = [&](int a, int b) -> long long {
      return bc == 3 ? (long long)(2 * a + 1 - g.nely) * (2 * a + 1 - g.nely) +
                           (long long)(2 * b + 1 - g.nelz) * (2 * b + 1 - g.nelz)
                     : (long long)(2 * a + 1) * (2 * a + 1) +
                           (long long)(2 * b + 1 - g.nely) * (2 * b + 1 - g.nely);
    };
    for (int b = 0; b < nb; ++b)
      for (int a = 0; a < na; ++a) {
        const long long d2 = d2of(a, b);
        if (dmin < 0 || d2 < dmin) dmin = d2;
      }
    thr = 25 * dmin <= m * m ? m * m : 25 * dmin;
    for (int b = 0; b < nb; ++b)
      for (int a = 0; a < na; ++a)
        if (25 * d2of(a, b) <= thr) ++nq;
  }
  int blocks = (int)((g.nn + 255) / 256);
  if (blocks > 4096) blocks = 4096;
  hipLaunchKernelGGL(k_load_builtin, dim3(blocks), dim3(256), 0, s, g.nelx, g.nely, g.nelz, bc,
                     load_total, thr, nq, mask, f);
  return hipGetLastError();
}

// CUSTOM: per-DOF byte mask (device copy) -> per-node bits; zero f on fixed DOFs
__global__ void k_mask_custom(size_t nn, const uint8_t *__restrict__ dof_mask,
                              uint8_t *__restrict__ mask, double *__restrict__ f) {
  for (size_t n = blockIdx.x * (size_t)blockDim.x + threadIdx.x; n < nn;
       n += (size_t)gridDim.x * blockDim.x) {
    unsigned m = 0;
    for (int c = 0; c < 3; ++c)
      if (dof_mask[3 * n + c]) {
        m |= 1u << c;
        f[3 * n + c] = 0.0;
      }
    mask[n] = (uint8_t)m;
  }
}

hipError_t launch_mask_custom(const Grid &g, const uint8_t *dof_mask, uint8_t *mask, double *f,
                              hipStream_t s) {
  int blocks = (int)((g.nn + 255) / 256);
  if (blocks > 4096) blocks = 4096;
  hipLaunchKernelGGL(k_mask_custom, dim3(blocks), dim3(256), 0, s, g.nn, dof_mask, mask, f);
  return hipGetLastError();
}

// ---------------------------------------------------------------- CG streams
// blocks of the batched update kernel for one design (grid-stride beyond)
int update_blocks(size_t nn) {
  size_t cap = 512;
  if (const char *e = getenv("TOPO_UPB")) cap = (size_t)atoi(e);
  if (cap < 1) cap = 1;
  if (cap > (size_t)MAXB) cap = MAXB;
  size_t b = (nn + 511) / 512;  // two nodes per thread: both loaded before the p^T q sum
  if (b < 64) b = 64;
  if (b > cap) b = cap;
  if (b > (nn + 255) / 256) b = (nn + 255) / 256;
  if (b < 1) b = 1;
  return (int)b;
}

int vec_blocks(size_t nn) {
  size_t b = (nn + 255) / 256;
  if (b > 2048) b = 2048;
  if (b < 1) b = 1;
  return (int)b;
}

template <typename T>
__global__ __launch_bounds__(256) void k_cg_init(size_t nn, const double *__restrict__ b,
                                                 const double *__restrict__ scal, T *__restrict__ x,
                                                 T *__restrict__ r, T *__restrict__ z,
                                                 T *__restrict__ p, T *__restrict__ p2,
                                                 T *__restrict__ p3, T *__restrict__ p4,
                                                 const T *__restrict__ dinv,
                                                 const uint8_t *__restrict__ mask,
                                                 double *__restrict__ rzp, double *__restrict__ rrp,
                                                 double *__restrict__ rpp, double *__restrict__ zqp,
                                                 int zbf) {
  __shared__ double sh[4];
  const double sc = scal[S_SCALE];
  double rz = 0.0, rr = 0.0;
  for (size_t n = blockIdx.x * (size_t)blockDim.x + threadIdx.x; n < nn;
       n += (size_t)gridDim.x * blockDim.x) {
    const unsigned m = mask[n];
    const T di = dinv[n];
#pragma unroll
    for (int c = 0; c < 3; ++c) {
      const size_t i = 3 * n + c;
      const T rv = ((m >> c) & 1u) ? T(0) : (T)(b[i] * sc);
      T zv = di * rv;
      x[i] = 0;
      r[i] = rv;
      bool zdone = false;
      if constexpr (sizeof(T) == 4) {
        if (zbf) {  // z in bfloat16 (the float32 buffer's first half), rounded once
          const __bf16 zb = (__bf16)zv;
          zv = (T)(float)zb;
          ((unsigned short *)z)[i] = __builtin_bit_cast(unsigned short, zb);
          zdone = true;
        }
      }
      if (!zdone) z[i] = zv;
      p[i] = 0;
      p2[i] = 0;
      if (p3) p3[i] = 0;
      if (p4) p4[i] = 0;
      rz += (double)rv * (double)zv;
      rr += (double)rv * (double)rv;
    }
  }
  const double s1 = block_sum(rz, sh);
  const double s2 = block_sum(rr, sh);
  if (threadIdx.x == 0) {
    rzp[blockIdx.x] = s1;
    rrp[blockIdx.x] = s2;
    rpp[blockIdx.x] = 0.0;  // r^T p_old and z^T q_old with p_old = 0
    zqp[blockIdx.x] = 0.0;
  }
}

template <typename T>
hipError_t launch_cg_init(const Grid &g, const double *b, const double *scal, T *x, T *r, T *z,
                          T *pA, T *pB, const T *dinv, const uint8_t *mask, double *cgp, int slot,
                          int nb_up, hipStream_t s, int zbf, T *pC, T *pD) {
  hipLaunchKernelGGL(k_cg_init<T>, dim3(nb_up), dim3(256), 0, s, g.nn, b, scal, x, r, z, pA, pB,
                     pC, pD, dinv, mask, cgp + CGP_RZ + slot * MAXB, cgp + CGP_RR + slot * MAXB,
                     cgp + CGP_RP + slot * MAXB, cgp + CGP_ZQ + slot * MAXB, zbf);
  return hipGetLastError();
}

template <typename T>
struct PSlots {
  const T *p[CG_NP_MAX];
};

// u += (x + pending steps) / scal[S_SCALE]  (float64 solution update of the
// outer refinement; the pending steps in the same order as a grouped update)
template <typename T>
__global__ void k_axpy_out(size_t ndof, double *__restrict__ u, const T *__restrict__ d,
                           const double *__restrict__ scal, int np, const PSlots<T> ps,
                           const int *__restrict__ flags) {
  const double a = 1.0 / scal[S_SCALE];
  const int npend = np > 0 ? (flags[F_SLOT0] + flags[F_ITERS] + 1) % np : 0;
  T al[CG_NP_MAX];
#pragma unroll
  for (int j = 0; j < CG_NP_MAX; ++j) al[j] = j < npend ? (T)scal[S_AH + j] : T(0);
  for (size_t i = blockIdx.x * (size_t)blockDim.x + threadIdx.x; i < ndof;
       i += (size_t)gridDim.x * blockDim.x) {
    T x = d[i];
    for (int j = 0; j < npend; ++j) x = x + al[j] * ps.p[j][i];
    u[i] += a * (double)x;
  }
}

template <typename T>
hipError_t launch_axpy_out(const Grid &g, double *u, const T *d, const double *scal,
                           hipStream_t s, int np, int xgroup, T *const *p, const int *flags) {
  int blocks = (int)((g.ndof + 255) / 256);
  if (blocks > 4096) blocks = 4096;
  PSlots<T> ps{};
  if (xgroup)
    for (int j = 0; j < np; ++j) ps.p[j] = p[j];
  else
    np = 0;  // nothing pending
  hipLaunchKernelGGL(k_axpy_out<T>, dim3(blocks), dim3(256), 0, s, g.ndof, u, d, scal, np, ps,
                     flags);
  return hipGetLastError();
}

// ---------------------------------------------------------------- reductions
// One block sums nb partials in a fixed order (strided per thread, then a
// fixed tree), so every reduction is reproducible run to run.
__device__ double fixed_order_sum(const double *v, int nb) {
  __shared__ double sh[RED_THREADS];
  double s = 0.0;
  for (int i = threadIdx.x; i < nb; i += RED_THREADS) s += v[i];
  sh[threadIdx.x] = s;
  __syncthreads();
  for (int w = RED_THREADS / 2; w > 0; w >>= 1) {
    if (threadIdx.x < w) sh[threadIdx.x] += sh[threadIdx.x + w];
    __syncthreads();
  }
  const double r = sh[0];
  __syncthreads();
  return r;
}

__global__ __launch_bounds__(RED_THREADS) void k_finish_init(const double *cgp, int nb, int slot,
                                                             double tol2_rel, int cap,
                                                             double *scal, int *flags,
                                                             int slot0) {
  const double rz = fixed_order_sum(cgp + CGP_RZ + slot * MAXB, nb);
  const double rr = fixed_order_sum(cgp + CGP_RR + slot * MAXB, nb);
  if (threadIdx.x == 0) {
    scal[S_RZ] = rz;
    scal[S_RZ0] = rz;   // both generations: the first product's beta multiplies p = 0
    scal[S_RZ1] = rz;
    scal[S_RR] = rr;
    scal[S_BETA] = 0.0;
    scal[S_TOL2] = tol2_rel * rr;
    flags[F_ITERS] = 0;
    flags[F_STATUS] = 0;
    flags[F_CAP] = cap;
    flags[F_SLOT0] = slot0;
    for (int j = 0; j < CG_NP_MAX; ++j) scal[S_AH + j] = 0.0;
    int done = (rr == 0.0) ? 1 : 0;
    if (!isfinite(rr) || !isfinite(rz)) {
      flags[F_STATUS] = 2;
      done = 1;
    }
    flags[F_DONE] = done;
  }
}

__global__ __launch_bounds__(RED_THREADS) void k_finish_sum(const double *part, int nb, double *scal,
                                                            int idx) {
  const double s = fixed_order_sum(part, nb);
  if (threadIdx.x == 0) scal[idx] = s;
}

hipError_t launch_finish_init(const double *cgp, int nb_up, int slot, double tol2_rel, int cap,
                              double *scal, int *flags, hipStream_t s, int slot0) {
  hipLaunchKernelGGL(k_finish_init, dim3(1), dim3(RED_THREADS), 0, s, cgp, nb_up, slot, tol2_rel,
                     cap, scal, flags, slot0);
  return hipGetLastError();
}
hipError_t launch_finish_sum(const double *part, int nb, int comp, double *scal, int idx,
                             hipStream_t s) {
  hipLaunchKernelGGL(k_finish_sum, dim3(1), dim3(RED_THREADS), 0, s, part + (size_t)comp * MAXB,
                     nb, scal, idx);
  return hipGetLastError();
}

// After the outer residual: S_SCALE = 1/||r||.
__global__ void k_set_scale(double *scal) {
  if (threadIdx.x == 0) {
    const double n2 = scal[S_NORM2];
    scal[S_SCALE] = (n2 > 0.0) ? 1.0 / sqrt(n2) : 1.0;
  }
}

// Byte fill with zeros: a kernel rather than a memset so that a captured
// graph replays it faithfully.
__global__ void k_fill(uint32_t *p, size_t nwords) {
  for (size_t i = blockIdx.x * (size_t)blockDim.x + threadIdx.x; i < nwords;
       i += (size_t)gridDim.x * blockDim.x)
    p[i] = 0u;
}

hipError_t launch_fill(void *p, size_t bytes, hipStream_t s) {
  const size_t nw = bytes / 4;
  int blocks = (int)((nw + 255) / 256);
  if (blocks > 4096) blocks = 4096;
  if (blocks < 1) blocks = 1;
  hipLaunchKernelGGL(k_fill, dim3(blocks), dim3(256), 0, s, (uint32_t *)p, nw);
  return hipGetLastError();
}

// partial sums of a^T b
__global__ __launch_bounds__(256) void k_dot(const double *__restrict__ a,
                                             const double *__restrict__ b, size_t n,
                                             double *__restrict__ part) {
  __shared__ double sh[4];
  double s = 0.0;
  for (size_t i = blockIdx.x * (size_t)blockDim.x + threadIdx.x; i < n;
       i += (size_t)gridDim.x * blockDim.x)
    s += a[i] * b[i];
  const double t = block_sum(s, sh);
  if (threadIdx.x == 0) part[blockIdx.x] = t;
}

hipError_t launch_dot(const double *a, const double *b, size_t n, double *part, int *nb,
                      hipStream_t s) {
  int blocks = (int)((n + 255) / 256);
  if (blocks > 2048) blocks = 2048;
  if (blocks < 1) blocks = 1;
  *nb = blocks;
  hipLaunchKernelGGL(k_dot, dim3(blocks), dim3(256), 0, s, a, b, n, part);
  return hipGetLastError();
}

hipError_t launch_set_scale(double *scal, hipStream_t s) {
  hipLaunchKernelGGL(k_set_scale, dim3(1), dim3(64), 0, s, scal);
  return hipGetLastError();
}

template hipError_t launch_cg_init<double>(const Grid &, const double *, const double *, double *,
                                           double *, double *, double *, double *, const double *,
                                           const uint8_t *, double *, int, int, hipStream_t, int,
                                           double *, double *);
template hipError_t launch_cg_init<float>(const Grid &, const double *, const double *, float *,
                                          float *, float *, float *, float *, const float *,
                                          const uint8_t *, double *, int, int, hipStream_t, int,
                                          float *, float *);
template hipError_t launch_axpy_out<double>(const Grid &, double *, const double *,
                                            const double *, hipStream_t, int, int,
                                            double *const *, const int *);
template hipError_t launch_axpy_out<float>(const Grid &, double *, const float *, const double *,
                                           hipStream_t, int, int, float *const *, const int *);

}  // namespace topo
