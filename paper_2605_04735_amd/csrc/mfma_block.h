// Device part of the matrix-core float32 product (see k_mfma.hip for the
// derivation): LDS layout, exact bfloat16 splitting and the block routine,
// shared by the plain product and the inner-CG product kernels.
#pragma once

#include "common.h"
#include "device_common.h"

namespace topo {

typedef __bf16 bf16x8 __attribute__((ext_vector_type(8)));
typedef float floatx4 __attribute__((ext_vector_type(4)));

constexpr int MP = ME + 1;      // node plane edge (17)
constexpr int MPL = MP * MP;    // nodes per staged plane (289)

struct MfmaLds {
  uint2 sp[3][3][MPL];   // [plane % 3][part][node]: 4 bfloat16 (x, y, z, 0) per node
  float4 pf[3][MPL];     // [plane % 3][node]: the float32 values (x, y, z, 0)
  float xch[2][4][2][64];  // [layer parity][wave][az][lane]: a wave's last-row contributions
};

__device__ __forceinline__ unsigned bf16_bits(float v) {
  return (unsigned)__builtin_bit_cast(unsigned short, (__bf16)v);
}
__device__ __forceinline__ float bf16_value(unsigned bits) { return __uint_as_float(bits << 16); }

// v = hi + mid + lo, each part bfloat16 (exact: every difference is exact)
__device__ __forceinline__ void split3(float v, unsigned &hi, unsigned &mid, unsigned &lo) {
  hi = bf16_bits(v);
  const float r1 = v - bf16_value(hi);
  mid = bf16_bits(r1);
  lo = bf16_bits(r1 - bf16_value(mid));
}

__device__ __forceinline__ float shr1_row(float v) {
  // lane e of each 16-lane row gets lane e - 1's value; lane 0 of a row gets 0
  return __int_as_float(__builtin_amdgcn_update_dpp(0, __float_as_int(v), 0x111, 0xF, 0xF, true));
}

// One block of the matrix-core product (MODE: MV_APPLY or MV_CG), tile (bx, by)
// over node planes [bz kz, bz kz + kz).  Returns the block's p^T q partial in
// thread 0 (MV_CG).  pre/get_beta: as for the vector-ALU product.
template <int MODE, int ZF = ZF_READ, typename PreFn, typename BetaFn>
__device__ __forceinline__ double mfma_block(const MvArgs<float> &a, int bx, int by, int bz,
                                             PreFn &&pre, BetaFn &&get_beta, MfmaLds &S,
                                             double *red) {
  constexpr bool CG = MODE == MV_CG;
  constexpr bool MASKED = !CG;
  constexpr unsigned F4 = 4u;
  const int tid = threadIdx.x, lane = tid & 63, w = tid >> 6;
  const int g = lane >> 4, ei = lane & 15;  // B: corner pair (g & 1, g >> 1); D: component g
  const int NX = a.nelx + 1, NY = a.nely + 1, NZ = a.nelz + 1;
  const int i0 = bx * MN, j0 = by * MN;
  const int k0 = bz * a.kz;
  const int k1 = min(k0 + a.kz, NZ);
  const unsigned plane = (unsigned)NX * (unsigned)NY;
  const unsigned eplane = (unsigned)a.nelx * (unsigned)a.nely;
  const unsigned nn = plane * (unsigned)NZ;
  const rsrc_t rOut = make_rsrc(a.out, 3u * nn * F4);
  const rsrc_t rPn = make_rsrc(a.pout, CG ? 3u * nn * F4 : 0u);
  const rsrc_t rIn = make_rsrc(a.in, 3u * nn * F4);
  const rsrc_t rM = make_rsrc(a.mask, MASKED ? nn : 0u);
  // the input is r and z = D r is formed here (ZF_FORM, or ZF_DESC with zfuse)
  constexpr bool ZFC = CG && ZF != ZF_READ;
  const bool zf = ZFC && (ZF == ZF_FORM || a.zfuse);

  // the A operand (rows of M for az = 0 and az = 1), 16 bytes each
  bf16x8 A0, A1;
  {
    const uint4 *mA = (const uint4 *)a.mA;
    A0 = __builtin_bit_cast(bf16x8, mA[lane]);
    A1 = __builtin_bit_cast(bf16x8, mA[64 + lane]);
  }
  const float mscale = a.mscale;

  // staging slots: node idx = tid (+ 256 for tid < 33) of the 17 x 17 plane
  unsigned voN[2], voM[2], voP[2];
#pragma unroll
  for (int sl = 0; sl < 2; ++sl) {
    const int idx = tid + sl * MF_THREADS;
    const int li = idx % MP, lj = idx / MP;
    const int gx = i0 - 1 + li, gy = j0 - 1 + lj;
    const bool v = idx < MPL && gx >= 0 && gx < NX && gy >= 0 && gy < NY;
    const bool mine = li >= 1 && li <= MN && lj >= 1 && lj <= MN;
    const unsigned n = (unsigned)gx + (unsigned)NX * (unsigned)gy;
    voN[sl] = v ? 3u * F4 * n : OOB;
    voM[sl] = v ? n : OOB;
    voP[sl] = v && mine ? 3u * F4 * n : OOB;
  }
  // this lane's elements (one per set s: row 4w + s) and output nodes
  unsigned voE[4], voQ[4], nQ[4];
  const int gi = i0 - 1 + ei;
#pragma unroll
  for (int s = 0; s < 4; ++s) {
    const int ej = 4 * w + s;
    const int gj = j0 - 1 + ej;
    const bool ev = gi >= 0 && gi < a.nelx && gj >= 0 && gj < a.nely;
    voE[s] = ev ? ((unsigned)gi + (unsigned)a.nelx * (unsigned)gj) * F4 : OOB;
    // output node of row s: (ei, ej) in the plane, component g
    const bool own = g < 3 && ei >= 1 && ei <= MN && ej >= 1 && ej <= MN && gi < NX && gj < NY;
    const unsigned n = (unsigned)gi + (unsigned)NX * (unsigned)gj;
    nQ[s] = own ? n : OOB;
    voQ[s] = own ? F4 * (3u * n + (unsigned)g) : OOB;
  }

  struct Plane {
    float in[2][3], po[2][3];
    unsigned m[2];
    float e[4];
    float di[2];  // zf: Jacobi inverse diagonal
  };
  auto fetch = [&](Plane &R, int kp) {
    const bool inz = kp >= 0 && kp < NZ;  // uniform
    const unsigned kc = inz ? (unsigned)kp : 0u;
    const unsigned so = kc * plane * 3u * F4;
    const rsrc_t ri = make_rsrc(a.in, inz ? 3u * nn * F4 : 0u);
    const rsrc_t rp = make_rsrc(a.pold, CG && inz ? 3u * nn * F4 : 0u);
    const rsrc_t rm = make_rsrc(a.mask, MASKED && inz ? nn : 0u);
    const rsrc_t re = make_rsrc(a.E, kp >= 0 && kp < a.nelz ? eplane * (unsigned)a.nelz * F4 : 0u);
    const rsrc_t rd = make_rsrc(a.dinv, zf && inz ? nn * F4 : 0u);
#pragma unroll
    for (int sl = 0; sl < 2; ++sl) {
      bload3(ri, voN[sl], so, R.in[sl]);
      if constexpr (CG) {
        bload3(rp, voN[sl], so, R.po[sl]);
        if constexpr (ZFC)
          R.di[sl] = bload1f(rd, voM[sl] == OOB ? OOB : voM[sl] * F4, kc * plane * F4);
      }
      if constexpr (MASKED) R.m[sl] = bload_u8(rm, voM[sl], kc * plane);
    }
#pragma unroll
    for (int s = 0; s < 4; ++s) R.e[s] = bload1f(re, voE[s], kc * eplane * F4);
  };
  float beta = 0.f;
  // plane kp into LDS slot kp % 3 (split into bfloat16 parts); CG: p = z +
  // beta p_old (z = D r under zf), written out for the nodes this block owns
  auto stage = [&](Plane &R, int kp, float (&E)[4]) {
    const int slot = (kp + 3) % 3;
    const bool wr = CG && kp >= k0 && kp < k1;
#pragma unroll
    for (int sl = 0; sl < 2; ++sl) {
      const int idx = tid + sl * MF_THREADS;
      if (idx >= MPL) continue;
      float v[3];
#pragma unroll
      for (int c = 0; c < 3; ++c) {
        if constexpr (CG) {
          float z = R.in[sl][c];
          if constexpr (ZFC) {
            if (zf) z = mul_rn(R.di[sl], z);
          }
          v[c] = z + beta * R.po[sl][c];
        } else v[c] = ((R.m[sl] >> c) & 1u) ? 0.f : R.in[sl][c];
      }
      unsigned h[3], m[3], l[3];
#pragma unroll
      for (int c = 0; c < 3; ++c) split3(v[c], h[c], m[c], l[c]);
      S.sp[slot][0][idx] = make_uint2(h[0] | (h[1] << 16), h[2]);
      S.sp[slot][1][idx] = make_uint2(m[0] | (m[1] << 16), m[2]);
      S.sp[slot][2][idx] = make_uint2(l[0] | (l[1] << 16), l[2]);
      S.pf[slot][idx] = make_float4(v[0], v[1], v[2], 0.f);
      if (wr) bstore3(rPn, voP[sl], (unsigned)kp * plane * 3u * F4, v);
    }
#pragma unroll
    for (int s = 0; s < 4; ++s) E[s] = R.e[s];
  };

  float acc = 0.f;           // CG: this lane's p^T q terms
  float carry[4] = {0, 0, 0, 0};  // per row: az = 1 part of the layer below (the node's plane L)
  float row0[2] = {0, 0};    // row 0 of the last layer, az = 0 and 1, before the wave above adds
  float prow0 = 0.f;         // row 0's p (component g) on the last layer's lower plane
  // emits the node (row s, plane L): value + identity rows / CG dot
  auto emit = [&](int s, int L, float val, float pv) {
    if (L < k0) return;
    const unsigned so = (unsigned)L * plane * 3u * F4;
    if constexpr (CG) {
      __builtin_amdgcn_raw_buffer_store_b32(__float_as_uint(val), rOut, (int)voQ[s], (int)so, 2);
      if (voQ[s] != OOB) acc += pv * val;
    } else {
      const unsigned mb = bload_u8(rM, nQ[s], (unsigned)L * plane);
      const float u = bload1f(rIn, voQ[s], so);
      const float y = ((mb >> g) & 1u) ? u : val;
      __builtin_amdgcn_raw_buffer_store_b32(__float_as_uint(y), rOut, (int)voQ[s], (int)so, 2);
    }
  };
  // completes row 0 of layer L with the wave below's last row (layer parity L & 1)
  auto finish_row0 = [&](int L) {
    const float in0 = w > 0 ? S.xch[L & 1][w - 1][0][lane] : 0.f;
    const float in1 = w > 0 ? S.xch[L & 1][w - 1][1][lane] : 0.f;
    const float y0 = row0[0] + in0, y1 = row0[1] + in1;
    emit(0, L, y0 + carry[0], prow0);
    carry[0] = y1;
  };
  // element layer L (planes L and L + 1, LDS slots L % 3 and (L + 1) % 3)
  auto layer = [&](int L, const float (&E)[4]) {
    const int sl0 = (L + 3) % 3, sl1 = (L + 4) % 3;
    const int slB = (g >> 1) ? sl1 : sl0;  // this lane's B plane (az = g >> 1)
    float xprev[2] = {0, 0};
#pragma unroll
    for (int s = 0; s < 4; ++s) {
      const int ej = 4 * w + s;
      const int nb = (ej + (g & 1)) * MP + ei;  // corner pair's first node
      bf16x8 B[3];
#pragma unroll
      for (int part = 0; part < 3; ++part) {
        const uint2 lo = S.sp[slB][part][nb], hi = S.sp[slB][part][nb + 1];
        B[part] = __builtin_bit_cast(bf16x8, make_uint4(lo.x, lo.y, hi.x, hi.y));
      }
      floatx4 c0 = {0.f, 0.f, 0.f, 0.f}, c1 = {0.f, 0.f, 0.f, 0.f};
#pragma unroll
      for (int part = 0; part < 3; ++part) {
        c0 = __builtin_amdgcn_mfma_f32_16x16x32_bf16(A0, B[part], c0, 0, 0, 0);
        c1 = __builtin_amdgcn_mfma_f32_16x16x32_bf16(A1, B[part], c1, 0, 0, 0);
      }
      const float se = E[s] * mscale;
      // corner t = ax + 2 ay of this element, component g, az = 0 (c0) / 1 (c1);
      // x: node ei gets corner ax = 0 of element ei and ax = 1 of element ei - 1
      float X[2][2];  // [ay][az]
      X[0][0] = c0[0] * se + shr1_row(c0[1] * se);
      X[1][0] = c0[2] * se + shr1_row(c0[3] * se);
      X[0][1] = c1[0] * se + shr1_row(c1[1] * se);
      X[1][1] = c1[2] * se + shr1_row(c1[3] * se);
      const float pv = reinterpret_cast<const float *>(&S.pf[sl0][ej * MP + ei])[g];
      if (s == 0) {
        row0[0] = X[0][0];
        row0[1] = X[0][1];
        prow0 = pv;
      } else {
        // y: node row ej gets ay = 0 of element row ej and ay = 1 of row ej - 1
        const float y0 = X[0][0] + xprev[0], y1 = X[0][1] + xprev[1];
        emit(s, L, y0 + carry[s], pv);
        carry[s] = y1;
      }
      xprev[0] = X[1][0];
      xprev[1] = X[1][1];
    }
    S.xch[L & 1][w][0][lane] = xprev[0];
    S.xch[L & 1][w][1][lane] = xprev[1];
  };

  Plane R0, R1;
  float Ecur[4], Enext[4];
  pre();
  fetch(R0, k0 - 1);
  fetch(R1, k0);
  if (!get_beta(beta)) return 0.0;
  stage(R0, k0 - 1, Ecur);
  if (k0 + 1 <= k1) fetch(R0, k0 + 1);
  // layer L stages plane L + 1 from the ring and refills its set with plane
  // L + 3; unrolled by two so that ring sets alternate statically.  One
  // barrier per layer: planes rotate over three LDS slots, and the row
  // exchange alternates by layer parity.
  for (int L = k0 - 1;;) {
    {
      stage(R1, L + 1, Enext);
      if (L + 3 <= k1) fetch(R1, L + 3);
      __syncthreads();
      if (L > k0 - 1) finish_row0(L - 1);
      layer(L, Ecur);
#pragma unroll
      for (int s = 0; s < 4; ++s) Ecur[s] = Enext[s];
    }
    if (++L >= k1) break;
    {
      stage(R0, L + 1, Enext);
      if (L + 3 <= k1) fetch(R0, L + 3);
      __syncthreads();
      finish_row0(L - 1);
      layer(L, Ecur);
#pragma unroll
      for (int s = 0; s < 4; ++s) Ecur[s] = Enext[s];
    }
    if (++L >= k1) break;
  }
  __syncthreads();
  finish_row0(k1 - 1);
  if constexpr (CG) return block_sum_d((double)acc, red);
  return 0.0;
}

}  // namespace topo
