// Matrix-free SIMP-weighted hex8 stiffness product y = sum_e E_e k0 u_e
// (paper Eq. 2 with Eq. 1 moduli), for float64 and float32.
//
// Element apply.  On a cube every trilinear displacement component is
// u = sum_m c_m m(xi, eta, zeta) over the monomials m in
// {1, xi, eta, zeta, xi eta, eta zeta, xi zeta, xi eta zeta} (reference cube
// [-1,1]^3); the unnormalised coefficients C_m = sum_a m(node a) u_a are an
// 8-point Walsh-Hadamard transform of the nodal values.  The displacement
// gradient is a sum of monomials that are mutually L2-orthogonal on the cube,
// so u^T k0 u splits into independent quadratic forms: the constant gradient
// (weight 8), the three groups linear in one coordinate (weight 8/3) and the
// three bilinear groups (weight 8/9).  Differentiating that energy gives per
// monomial "stress" coefficients D_m, and y = E h/32 * WHT(D) with D_1 = 0
// (rigid translations never enter).  About 180 additions and multiplications
// per element instead of 576 multiply-adds for the dense 24 x 24 product; it
// equals the Gauss-integrated k0 to rounding.
//
// Tiling.  A 256-thread block holds a 16 x 16 element tile of one z layer and
// owns the 15 x 15 nodes interior to it; it marches up a range of node planes.
// Per element layer L: node plane L+1 of the input (17 x 17 nodes) is staged
// in LDS next to plane L, every thread applies its element and writes its 24
// outputs to LDS, then every owned node sums, in a fixed order, the
// contributions of layer L-1 (kept in registers) and layer L.  No atomics: the
// result is deterministic.  Each element is computed by one block only in z
// and by up to four blocks in x/y (halo), 256/225 ~ 1.14x element work.
#include "common.h"

namespace topo {

template <typename T>
__device__ __forceinline__ void wht8(T v[8]) {
  // v[a] -> sum_a' prod_d (m_d ? s_d(a') : 1) v[a'], index bits d = 0,1,2
#pragma unroll
  for (int d = 0; d < 3; ++d) {
#pragma unroll
    for (int a = 0; a < 8; ++a) {
      if (!((a >> d) & 1)) {
        const int b = a | (1 << d);
        const T lo = v[a], hi = v[b];
        v[a] = hi + lo;
        v[b] = hi - lo;
      }
    }
  }
}

template <typename T>
__device__ __forceinline__ void iwht8(T v[8]) {
  // transpose of wht8 (the matrix is symmetric; butterflies in the same order)
#pragma unroll
  for (int d = 0; d < 3; ++d) {
#pragma unroll
    for (int a = 0; a < 8; ++a) {
      if (!((a >> d) & 1)) {
        const int b = a | (1 << d);
        const T lo = v[a], hi = v[b];
        v[a] = lo - hi;
        v[b] = lo + hi;
      }
    }
  }
}

// y[a][c] = E * (k0 u)[3a+c]; u, y: [3][8] component-major.
template <typename T>
__device__ __forceinline__ void hex8_apply(T u[3][8], T E, const Coef<T> &k) {
  const T L2 = E * k.L2, M4 = E * k.M4, M2 = E * k.M2;
  const T L2_3 = E * k.L2_3, M2_3 = E * k.M2_3, B9 = E * k.B9;
  wht8(u[0]);
  wht8(u[1]);
  wht8(u[2]);
  T(&cx)[8] = u[0];
  T(&cy)[8] = u[1];
  T(&cz)[8] = u[2];
  // monomial index m = mx + 2 my + 4 mz: 1 xi, 2 eta, 3 xi.eta, 4 zeta,
  // 5 xi.zeta, 6 eta.zeta, 7 xi.eta.zeta
  T D[3][8];
  // constant gradient
  const T t0 = L2 * (cx[1] + cy[2] + cz[4]);
  D[0][1] = t0 + M4 * cx[1];
  D[1][2] = t0 + M4 * cy[2];
  D[2][4] = t0 + M4 * cz[4];
  const T sxy = M2 * (cy[1] + cx[2]);
  const T sxz = M2 * (cz[1] + cx[4]);
  const T syz = M2 * (cz[2] + cy[4]);
  D[1][1] = sxy; D[0][2] = sxy;
  D[2][1] = sxz; D[0][4] = sxz;
  D[2][2] = syz; D[1][4] = syz;
  // linear groups
  const T txi = L2_3 * (cy[3] + cz[5]);
  const T teta = L2_3 * (cx[3] + cz[6]);
  const T tzeta = L2_3 * (cx[5] + cy[6]);
  D[0][3] = teta + M2 * cx[3];
  D[1][3] = txi + M2 * cy[3];
  D[1][6] = tzeta + M2 * cy[6];
  D[2][6] = teta + M2 * cz[6];
  D[0][5] = tzeta + M2 * cx[5];
  D[2][5] = txi + M2 * cz[5];
  const T S = cz[3] + cy[5] + cx[6];
  D[2][3] = M2_3 * (S + cz[3]);
  D[0][6] = M2_3 * (S + cx[6]);
  D[1][5] = M2_3 * (S + cy[5]);
  // bilinear groups
  D[0][7] = B9 * cx[7];
  D[1][7] = B9 * cy[7];
  D[2][7] = B9 * cz[7];
  D[0][0] = 0;
  D[1][0] = 0;
  D[2][0] = 0;
  iwht8(D[0]);
  iwht8(D[1]);
  iwht8(D[2]);
#pragma unroll
  for (int c = 0; c < 3; ++c)
#pragma unroll
    for (int a = 0; a < 8; ++a) u[c][a] = D[c][a];
}

__device__ __forceinline__ double block_sum_d(double v, double *sh) {
#pragma unroll
  for (int o = 32; o > 0; o >>= 1) v += __shfl_down(v, o, 64);
  const int lane = threadIdx.x & 63, w = threadIdx.x >> 6;
  if (lane == 0) sh[w] = v;
  __syncthreads();
  double r = 0.0;
  if (threadIdx.x == 0) {
    const int nw = (blockDim.x + 63) >> 6;
    for (int i = 0; i < nw; ++i) r += sh[i];
  }
  return r;
}

template <typename T, int MODE>
__global__ __launch_bounds__(MV_THREADS) void k_matvec(const MvArgs<T> a) {
  if (MODE == MV_CG && a.flags[F_DONE]) return;
  __shared__ T pl[2][3][TP * TP];
  __shared__ T eo[24][MV_THREADS];
  __shared__ double red[MV_THREADS / 64];

  const int tid = threadIdx.x;
  const int NX = a.nelx + 1, NY = a.nely + 1, NZ = a.nelz + 1;
  const int i0 = blockIdx.x * TN, j0 = blockIdx.y * TN;
  const int k0 = blockIdx.z * a.kz;
  const int k1 = min(k0 + a.kz, NZ);
  const T beta = (MODE == MV_CG) ? (T)a.scal[S_BETA] : T(0);

  const int ei = tid % TE, ej = tid / TE;
  const int gi = i0 - 1 + ei, gj = j0 - 1 + ej;
  const bool e_xy = gi >= 0 && gi < a.nelx && gj >= 0 && gj < a.nely;

  const int ni = tid % TN, nj = tid / TN;
  const int gni = i0 + ni, gnj = j0 + nj;
  const bool own = tid < TN * TN && gni < NX && gnj < NY;

  // Stage node plane kp (17 x 17 nodes around the tile) into pl[buf]; fixed
  // DOFs read as zero.  In CG mode the plane is the new direction
  // p = z + beta p_old, written back for the owned nodes.
  auto load_plane = [&](int kp, int buf) {
    for (int idx = tid; idx < TP * TP; idx += MV_THREADS) {
      const int li = idx % TP, lj = idx / TP;
      const int gx = i0 - 1 + li, gy = j0 - 1 + lj;
      T v0 = 0, v1 = 0, v2 = 0;
      if (kp >= 0 && kp < NZ && gx >= 0 && gx < NX && gy >= 0 && gy < NY) {
        const size_t n = (size_t)gx + (size_t)NX * ((size_t)gy + (size_t)NY * kp);
        const unsigned m = a.mask[n];
        v0 = (m & 1u) ? T(0) : a.in[3 * n + 0];
        v1 = (m & 2u) ? T(0) : a.in[3 * n + 1];
        v2 = (m & 4u) ? T(0) : a.in[3 * n + 2];
        if (MODE == MV_CG) {
          v0 = (m & 1u) ? T(0) : v0 + beta * a.pold[3 * n + 0];
          v1 = (m & 2u) ? T(0) : v1 + beta * a.pold[3 * n + 1];
          v2 = (m & 4u) ? T(0) : v2 + beta * a.pold[3 * n + 2];
          if (li >= 1 && li <= TN && lj >= 1 && lj <= TN && kp >= k0 && kp < k1) {
            a.pout[3 * n + 0] = v0;
            a.pout[3 * n + 1] = v1;
            a.pout[3 * n + 2] = v2;
          }
        }
      }
      pl[buf][0][idx] = v0;
      pl[buf][1][idx] = v1;
      pl[buf][2][idx] = v2;
    }
  };

  T carry0 = 0, carry1 = 0, carry2 = 0;
  double acc = 0.0;
  int buf = 0;
  load_plane(k0 - 1, 0);
  for (int L = k0 - 1; L < k1; ++L) {
    load_plane(L + 1, buf ^ 1);
    __syncthreads();
    // CG: the owned node's direction on plane L, read while pl[buf] is
    // stable (the next layer's load overwrites it before the node phase ends)
    T pn0 = 0, pn1 = 0, pn2 = 0;
    if (MODE == MV_CG && own) {
      const int idx = (ni + 1) + TP * (nj + 1);
      pn0 = pl[buf][0][idx];
      pn1 = pl[buf][1][idx];
      pn2 = pl[buf][2][idx];
    }
    // element phase: element (gi, gj, L)
    {
      T u[3][8];
      T E = 0;
      const bool valid = e_xy && L >= 0 && L < a.nelz;
      if (valid) E = a.E[(size_t)gi + (size_t)a.nelx * ((size_t)gj + (size_t)a.nely * L)];
#pragma unroll
      for (int an = 0; an < 8; ++an) {
        const int ax = an & 1, ay = (an >> 1) & 1, az = an >> 2;
        const int idx = (ei + ax) + TP * (ej + ay);
        const int b = az ? (buf ^ 1) : buf;
        u[0][an] = pl[b][0][idx];
        u[1][an] = pl[b][1][idx];
        u[2][an] = pl[b][2][idx];
      }
      hex8_apply(u, E, a.k);
#pragma unroll
      for (int an = 0; an < 8; ++an) {
        eo[3 * an + 0][tid] = u[0][an];
        eo[3 * an + 1][tid] = u[1][an];
        eo[3 * an + 2][tid] = u[2][an];
      }
    }
    __syncthreads();
    // node phase: owned node (gni, gnj) on plane L gets carry + bottom
    // corners of layer L; the top corners of layer L become the new carry.
    if (own) {
      T s0 = carry0, s1 = carry1, s2 = carry2;
      T t0 = 0, t1 = 0, t2 = 0;
#pragma unroll
      for (int dy = 0; dy < 2; ++dy)
#pragma unroll
        for (int dx = 0; dx < 2; ++dx) {
          const int e = (ni + dx) + TE * (nj + dy);
          const int cb = (1 - dx) + 2 * (1 - dy);  // corner a = ax + 2 ay (+ 4 az)
          s0 += eo[3 * cb + 0][e];
          s1 += eo[3 * cb + 1][e];
          s2 += eo[3 * cb + 2][e];
          t0 += eo[3 * (cb + 4) + 0][e];
          t1 += eo[3 * (cb + 4) + 1][e];
          t2 += eo[3 * (cb + 4) + 2][e];
        }
      carry0 = t0;
      carry1 = t1;
      carry2 = t2;
      if (L >= k0) {
        const size_t n = (size_t)gni + (size_t)NX * ((size_t)gnj + (size_t)NY * L);
        const unsigned m = a.mask[n];
        if (MODE == MV_APPLY) {
          a.out[3 * n + 0] = (m & 1u) ? a.in[3 * n + 0] : s0;
          a.out[3 * n + 1] = (m & 2u) ? a.in[3 * n + 1] : s1;
          a.out[3 * n + 2] = (m & 4u) ? a.in[3 * n + 2] : s2;
        } else if (MODE == MV_CG) {
          s0 = (m & 1u) ? T(0) : s0;
          s1 = (m & 2u) ? T(0) : s1;
          s2 = (m & 4u) ? T(0) : s2;
          a.out[3 * n + 0] = s0;
          a.out[3 * n + 1] = s1;
          a.out[3 * n + 2] = s2;
          acc += (double)pn0 * (double)s0 + (double)pn1 * (double)s1 + (double)pn2 * (double)s2;
        } else {  // MV_RESID
          const double r0 = (m & 1u) ? 0.0 : a.f[3 * n + 0] - (double)s0;
          const double r1 = (m & 2u) ? 0.0 : a.f[3 * n + 1] - (double)s1;
          const double r2 = (m & 4u) ? 0.0 : a.f[3 * n + 2] - (double)s2;
          a.out[3 * n + 0] = (T)r0;
          a.out[3 * n + 1] = (T)r1;
          a.out[3 * n + 2] = (T)r2;
          acc += r0 * r0 + r1 * r1 + r2 * r2;
        }
      }
    }
    buf ^= 1;
  }
  if (MODE != MV_APPLY) {
    const double s = block_sum_d(acc, red);
    if (tid == 0) a.part[blockIdx.x + gridDim.x * (blockIdx.y + gridDim.y * blockIdx.z)] = s;
  }
}

int matvec_kz(const Grid &g) {
  const int NX = g.nelx + 1, NY = g.nely + 1, NZ = g.nelz + 1;
  const int tiles = ((NX + TN - 1) / TN) * ((NY + TN - 1) / TN);
  // aim for >= ~2048 blocks (8 per CU) while keeping the z-halo recompute
  // (kz + 1)/kz modest
  int chunks = (2048 + tiles - 1) / tiles;
  int kz = (NZ + chunks - 1) / chunks;
  if (kz < 4) kz = 4;
  if (kz > 64) kz = 64;
  return kz;
}

int matvec_blocks(const Grid &g, int kz) {
  const int NX = g.nelx + 1, NY = g.nely + 1, NZ = g.nelz + 1;
  return ((NX + TN - 1) / TN) * ((NY + TN - 1) / TN) * ((NZ + kz - 1) / kz);
}

template <typename T, int MODE>
hipError_t launch_matvec(const MvArgs<T> &a, int *nblocks, hipStream_t s) {
  const int NX = a.nelx + 1, NY = a.nely + 1, NZ = a.nelz + 1;
  dim3 grid((NX + TN - 1) / TN, (NY + TN - 1) / TN, (NZ + a.kz - 1) / a.kz);
  const int nb = grid.x * grid.y * grid.z;
  if (nblocks) *nblocks = nb;
  if (MODE != MV_APPLY && nb > MAXB) return hipErrorInvalidConfiguration;
  hipLaunchKernelGGL((k_matvec<T, MODE>), grid, dim3(MV_THREADS), 0, s, a);
  return hipGetLastError();
}

template hipError_t launch_matvec<double, MV_APPLY>(const MvArgs<double> &, int *, hipStream_t);
template hipError_t launch_matvec<double, MV_CG>(const MvArgs<double> &, int *, hipStream_t);
template hipError_t launch_matvec<double, MV_RESID>(const MvArgs<double> &, int *, hipStream_t);
template hipError_t launch_matvec<float, MV_APPLY>(const MvArgs<float> &, int *, hipStream_t);
template hipError_t launch_matvec<float, MV_CG>(const MvArgs<float> &, int *, hipStream_t);

// ---------------------------------------------------------------- energies
// s_e = u_e^T k0 u_e (float64) with the same factored apply, dc_e of Eq. 3,
// and block partial sums of sum_e E_e s_e.
__global__ __launch_bounds__(256) void k_energy_sens(int nelx, int nely, int nelz,
                                                     const double *__restrict__ x,
                                                     const double *__restrict__ u,
                                                     const double *__restrict__ E64,
                                                     Coef<double> k, double E0, double Emin,
                                                     double penal, double *__restrict__ dc,
                                                     double *__restrict__ part) {
  __shared__ double red[4];
  const size_t nel = (size_t)nelx * nely * nelz;
  const int NX = nelx + 1, NY = nely + 1;
  double acc = 0.0;
  for (size_t e = blockIdx.x * (size_t)blockDim.x + threadIdx.x; e < nel;
       e += (size_t)gridDim.x * blockDim.x) {
    const int i = (int)(e % nelx);
    const int j = (int)((e / nelx) % nely);
    const int kk = (int)(e / ((size_t)nelx * nely));
    double ue[3][8], ve[3][8];
#pragma unroll
    for (int an = 0; an < 8; ++an) {
      const size_t n = (size_t)(i + (an & 1)) +
                       (size_t)NX * ((size_t)(j + ((an >> 1) & 1)) + (size_t)NY * (kk + (an >> 2)));
      ue[0][an] = ve[0][an] = u[3 * n + 0];
      ue[1][an] = ve[1][an] = u[3 * n + 1];
      ue[2][an] = ve[2][an] = u[3 * n + 2];
    }
    hex8_apply(ve, 1.0, k);
    double s = 0.0;
#pragma unroll
    for (int an = 0; an < 8; ++an)
      s += ue[0][an] * ve[0][an] + ue[1][an] * ve[1][an] + ue[2][an] * ve[2][an];
    if (dc) dc[e] = -penal * pow(x[e], penal - 1.0) * (E0 - Emin) * s;
    acc += E64[e] * s;
  }
  const double t = block_sum_d(acc, red);
  if (threadIdx.x == 0) part[blockIdx.x] = t;
}

hipError_t launch_energy_sens(const Grid &g, const double *x, const double *u, const double *E64,
                              Coef<double> k, double E0, double Emin, double penal, double *dc,
                              double *part, int *nb, hipStream_t s) {
  int blocks = (int)((g.nel + 255) / 256);
  if (blocks > 2048) blocks = 2048;
  if (blocks < 1) blocks = 1;
  *nb = blocks;
  hipLaunchKernelGGL(k_energy_sens, dim3(blocks), dim3(256), 0, s, g.nelx, g.nely, g.nelz, x, u,
                     E64, k, E0, Emin, penal, dc, part);
  return hipGetLastError();
}

}  // namespace topo
