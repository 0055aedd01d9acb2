// Device helpers shared by the product kernels: the factored hex8 element
// apply, lane shifts and fixed-order block reductions.
#pragma once

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

// Per-monomial stresses D from the transform coefficients C of the three
// displacement components (C[c][0], the constant monomial, is never used):
// D = d(E u^T k0 u / 2)/dC with the h/32 scaling folded into the
// coefficients.  D[c][0] = 0.
template <typename T>
__device__ __forceinline__ void modal_stress(const T (&C)[3][8], T E, const Coef<T> &k,
                                             T (&D)[3][8]) {
  const T L2 = E * k.L2, M4 = E * k.M4, M2 = E * k.M2;
  const T L2_3 = E * k.L2_3, M2_3 = E * k.M2_3, B9 = E * k.B9;
  const T(&cx)[8] = C[0];
  const T(&cy)[8] = C[1];
  const T(&cz)[8] = C[2];
  // monomial index m = mx + 2 my + 4 mz: 1 xi, 2 eta, 3 xi.eta, 4 zeta,
  // 5 xi.zeta, 6 eta.zeta, 7 xi.eta.zeta
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
}

// u[c][a] <- E (k0 u)[3a + c] for one element; u: [3][8] component-major.
template <typename T>
__device__ __forceinline__ void hex8_apply(T (&u)[3][8], T E, const Coef<T> &k) {
  wht8(u[0]);
  wht8(u[1]);
  wht8(u[2]);
  T D[3][8];
  modal_stress(u, E, k, D);
  iwht8(D[0]);
  iwht8(D[1]);
  iwht8(D[2]);
#pragma unroll
  for (int c = 0; c < 3; ++c)
#pragma unroll
    for (int a = 0; a < 8; ++a) u[c][a] = D[c][a];
}

// Forward transform of one element face (4 corners (ax, ay) of a node plane
// in LDS): F[m], m = mx + 2 my, the x and y butterflies of the 8-point
// transform.
template <typename T>
__device__ __forceinline__ void face_forward(const T (*P)[TPX * TPY], int idx, T (&F)[3][4]) {
#pragma unroll
  for (int c = 0; c < 3; ++c) {
    const T v00 = P[c][idx], v10 = P[c][idx + 1], v01 = P[c][idx + TPX], v11 = P[c][idx + TPX + 1];
    const T s0 = v10 + v00, d0 = v10 - v00, s1 = v11 + v01, d1 = v11 - v01;
    F[c][0] = s1 + s0;
    F[c][1] = d1 + d0;
    F[c][2] = s1 - s0;
    F[c][3] = d1 - d0;
  }
}

// Sum over the 64 lanes of a wave, in a fixed order, returned in every lane:
// DPP row shifts 1, 2, 4, 8 leave each row's sum in its lane 15, the row
// broadcasts 15 and 31 carry those into lane 63, which is then read out.
// (A few cycles per step, against an LDS round trip per step for shuffles.)
template <int CTRL, int ROWMASK>
__device__ __forceinline__ double dpp_take(double v) {
  const int lo = __builtin_amdgcn_update_dpp(0, __double2loint(v), CTRL, ROWMASK, 0xF, true);
  const int hi = __builtin_amdgcn_update_dpp(0, __double2hiint(v), CTRL, ROWMASK, 0xF, true);
  return __hiloint2double(hi, lo);
}
__device__ __forceinline__ double wave_sum_d(double v) {
  v += dpp_take<0x111, 0xF>(v);  // row_shr:1
  v += dpp_take<0x112, 0xF>(v);  // row_shr:2
  v += dpp_take<0x114, 0xF>(v);  // row_shr:4
  v += dpp_take<0x118, 0xF>(v);  // row_shr:8
  v += dpp_take<0x142, 0xA>(v);  // row_bcast:15 into rows 1 and 3
  v += dpp_take<0x143, 0xC>(v);  // row_bcast:31 into rows 2 and 3
  const int lo = __builtin_amdgcn_readlane(__double2loint(v), 63);
  const int hi = __builtin_amdgcn_readlane(__double2hiint(v), 63);
  return __hiloint2double(hi, lo);
}

__device__ __forceinline__ double block_sum_d(double v, double *sh) {
  v = wave_sum_d(v);
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

// Two block sums in one pass (thread 0 holds both); sh: 8 doubles.
__device__ __forceinline__ void block_sum_d2(double a, double b, double *sh, double &sa,
                                             double &sb) {
  a = wave_sum_d(a);
  b = wave_sum_d(b);
  const int lane = threadIdx.x & 63, w = threadIdx.x >> 6;
  __syncthreads();
  if (lane == 0) {
    sh[w] = a;
    sh[w + 4] = b;
  }
  __syncthreads();
  sa = 0.0;
  sb = 0.0;
  if (threadIdx.x == 0) {
    const int nw = (blockDim.x + 63) >> 6;
    for (int i = 0; i < nw; ++i) {
      sa += sh[i];
      sb += sh[i + 4];
    }
  }
}

// Value of lane + 1 (0 for the last lane): a DPP shift, no LDS traffic.  With
// 16-element tile rows the shift stays within each row of 16 lanes
// (row_shl:1); wider rows span DPP rows and take the whole-wave shift
// (wave_shl:1).  Either way the last element of a tile row, which owns no
// node, is the only lane whose value is not its right neighbour's.
constexpr int DPP_NEXT_LANE = TEX == 16 ? 0x101 : 0x130;
__device__ __forceinline__ float from_next_lane(float v) {
  return __int_as_float(
      __builtin_amdgcn_update_dpp(0, __float_as_int(v), DPP_NEXT_LANE, 0xF, 0xF, true));
}
__device__ __forceinline__ double from_next_lane(double v) {
  const int lo = __builtin_amdgcn_update_dpp(0, __double2loint(v), DPP_NEXT_LANE, 0xF, 0xF, true);
  const int hi = __builtin_amdgcn_update_dpp(0, __double2hiint(v), DPP_NEXT_LANE, 0xF, 0xF, true);
  return __hiloint2double(hi, lo);
}

// ---- raw buffer access.  A buffer resource spans `bytes` bytes from p; a
// lane whose offset lies past the end loads 0 and its store is dropped, so
// lanes outside the grid take the offset OOB instead of a branch.  Offsets are
// 32-bit: voffset per lane, soffset uniform (an SGPR: the z plane).
using rsrc_t = __amdgpu_buffer_rsrc_t;
constexpr unsigned OOB = 0x80000000u;

__device__ __forceinline__ rsrc_t make_rsrc(const void *p, unsigned bytes) {
  // word 3 0x00020000: 32-bit raw data, range checked against `bytes`
  return __builtin_amdgcn_make_buffer_rsrc(const_cast<void *>(p), (short)0, (int)bytes, 0x00020000);
}

__device__ __forceinline__ void bload3(rsrc_t r, unsigned vo, unsigned so, float (&v)[3]) {
  const auto w = __builtin_amdgcn_raw_buffer_load_b96(r, (int)vo, (int)so, 0);
  v[0] = __uint_as_float(w[0]);
  v[1] = __uint_as_float(w[1]);
  v[2] = __uint_as_float(w[2]);
}
__device__ __forceinline__ void bload3(rsrc_t r, unsigned vo, unsigned so, double (&v)[3]) {
  const auto a = __builtin_amdgcn_raw_buffer_load_b128(r, (int)vo, (int)so, 0);
  const auto b = __builtin_amdgcn_raw_buffer_load_b64(r, (int)(vo + 16u), (int)so, 0);
  v[0] = __hiloint2double((int)a[1], (int)a[0]);
  v[1] = __hiloint2double((int)a[3], (int)a[2]);
  v[2] = __hiloint2double((int)b[1], (int)b[0]);
}
__device__ __forceinline__ void bstore3(rsrc_t r, unsigned vo, unsigned so, const float (&v)[3]) {
  typedef unsigned u3 __attribute__((ext_vector_type(3)));
  u3 w;
  w[0] = __float_as_uint(v[0]);
  w[1] = __float_as_uint(v[1]);
  w[2] = __float_as_uint(v[2]);
  // float32 CG streams: non-temporal (measured faster; float64 was not)
  __builtin_amdgcn_raw_buffer_store_b96(w, r, (int)vo, (int)so, 2);
}
__device__ __forceinline__ void bstore3(rsrc_t r, unsigned vo, unsigned so, const double (&v)[3]) {
  typedef unsigned u4 __attribute__((ext_vector_type(4)));
  typedef unsigned u2 __attribute__((ext_vector_type(2)));
  u4 a;
  a[0] = (unsigned)__double2loint(v[0]);
  a[1] = (unsigned)__double2hiint(v[0]);
  a[2] = (unsigned)__double2loint(v[1]);
  a[3] = (unsigned)__double2hiint(v[1]);
  u2 b;
  b[0] = (unsigned)__double2loint(v[2]);
  b[1] = (unsigned)__double2hiint(v[2]);
  __builtin_amdgcn_raw_buffer_store_b128(a, r, (int)vo, (int)so, 0);
  __builtin_amdgcn_raw_buffer_store_b64(b, r, (int)(vo + 16u), (int)so, 0);
}
__device__ __forceinline__ float bload1f(rsrc_t r, unsigned vo, unsigned so) {
  return __uint_as_float(__builtin_amdgcn_raw_buffer_load_b32(r, (int)vo, (int)so, 0));
}
__device__ __forceinline__ double bload1d(rsrc_t r, unsigned vo, unsigned so) {
  const auto w = __builtin_amdgcn_raw_buffer_load_b64(r, (int)vo, (int)so, 0);
  return __hiloint2double((int)w[1], (int)w[0]);
}
template <typename T>
__device__ __forceinline__ T bload1(rsrc_t r, unsigned vo, unsigned so) {
  if constexpr (sizeof(T) == 4) return bload1f(r, vo, so);
  else return bload1d(r, vo, so);
}
// Product rounded on its own, never fused into a following add: the CG
// product forms z = D r with exactly the value the update used for r^T z.
// (Fused into p = z + beta p_old, the unrounded z would make r^T z and the
// direction disagree by a rounding, which slowed the float32 CG by several
// percent in iterations.)
template <typename T>
__device__ __forceinline__ T mul_rn(T a, T b) {
#pragma clang fp contract(off)
  return a * b;
}

// bfloat16 storage of float32 vectors (3 components of 2 bytes per node):
// round to nearest even once, keep the rounded value in float32.
__device__ __forceinline__ float bf16_round(float v) {
  const __bf16 b = (__bf16)v;
  return __uint_as_float((unsigned)__builtin_bit_cast(unsigned short, b) << 16);
}
__device__ __forceinline__ void bload3_bf16(rsrc_t r, unsigned vo, unsigned so, float (&v)[3]) {
#pragma unroll
  for (int c = 0; c < 3; ++c)
    v[c] = __uint_as_float(
        (unsigned)__builtin_amdgcn_raw_buffer_load_b16(r, (int)(vo + 2u * c), (int)so, 0) << 16);
}
// v holds bfloat16-rounded values: the upper halves are exact
__device__ __forceinline__ void bstore3_bf16(rsrc_t r, unsigned vo, unsigned so, const float (&v)[3]) {
#pragma unroll
  for (int c = 0; c < 3; ++c)
    __builtin_amdgcn_raw_buffer_store_b16((unsigned short)(__float_as_uint(v[c]) >> 16), r,
                                          (int)(vo + 2u * c), (int)so, 2);
}
__device__ __forceinline__ unsigned bload_u8(rsrc_t r, unsigned vo, unsigned so) {
  return (unsigned)__builtin_amdgcn_raw_buffer_load_b8(r, (int)vo, (int)so, 0);
}

// Fixed-order sums of n block partials (NV arrays of the same length), split
// in two: load() issues this thread's first PK partials of each array (all of
// them when n <= PK BS; past n a buffer load returns 0, so there is
// no select) so that their round trip can start before other loads; sum()
// adds them in a fixed order (further batches only if n is larger), then a
// fixed shuffle/wave tree.  Every block gets the bit-identical values.
// sh: 4 NV doubles.
template <int PK, int NV, int BS = 256>  // BS: threads per block
struct Partials {
  double t[NV][PK];
  __device__ __forceinline__ void load(const double *const (&v)[NV], int n) {
#pragma unroll
    for (int a = 0; a < NV; ++a) {
      const rsrc_t r = make_rsrc(v[a], (unsigned)n * 8u);
#pragma unroll
      for (int k = 0; k < PK; ++k)
        t[a][k] = bload1d(r, 8u * (k * BS + threadIdx.x), 0);
    }
  }
  __device__ __forceinline__ void sum(const double *const (&v)[NV], int n, double *sh,
                                      double (&out)[NV]) {
    double s[NV];
#pragma unroll
    for (int a = 0; a < NV; ++a) {
      s[a] = 0.0;
#pragma unroll
      for (int k = 0; k < PK; ++k) s[a] += t[a][k];
    }
    if (n > PK * BS) {
      for (int base = PK * BS; base < n; base += BS) {
        const int i = base + (int)threadIdx.x;
#pragma unroll
        for (int a = 0; a < NV; ++a) s[a] += (i < n) ? v[a][i] : 0.0;
      }
    }
#pragma unroll
    for (int a = 0; a < NV; ++a) s[a] = wave_sum_d(s[a]);
    const int lane = threadIdx.x & 63, w = threadIdx.x >> 6;
    constexpr int nw = BS / 64;  // sh: nw * NV doubles
    __syncthreads();
    if (lane == 0)
#pragma unroll
      for (int a = 0; a < NV; ++a) sh[w + nw * a] = s[a];
    __syncthreads();
#pragma unroll
    for (int a = 0; a < NV; ++a) {
      out[a] = 0.0;
      for (int i = 0; i < nw; ++i) out[a] += sh[i + nw * a];
    }
    __syncthreads();
  }
};

}  // namespace topo
