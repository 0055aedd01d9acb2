// Matrix-core form of the float32 SIMP-weighted hex8 product y = sum_e E_e k0 u_e
// (paper Eq. 2 with Eq. 1 moduli): the 24 x 24 element contraction of every
// element runs on the MFMA units in bfloat16 with exact operands.
//
// Exact bfloat16 operands.  On the unit cube the trilinear element's weak
// form splits as k0 = (lambda A + mu B) / 72 with A and B integer matrices:
// A_ab^ik = 72 int d_i N_a d_k N_b and B_ab^ik = 72 (delta_ik int grad N_a .
// grad N_b + int d_k N_a d_i N_b), both products of 1D integrals of the
// linear shape functions (int phi phi = 1/3 or 1/6, int phi' phi' = +-1,
// int phi' phi = +-1/2).  So k0 = (mu/72) M with M = B + (lambda/mu) A.  For
// nu = 0.3 (lambda/mu = 3/2) every entry of M is a multiple of 1/2 below 50
// in magnitude, exact in bfloat16; the host checks exactness for the given
// nu and falls back to the vector-ALU product otherwise.  Each float32 input
// value v is split into three bfloat16 parts hi + mid + lo = v exactly (hi =
// bf16(v), mid = bf16(v - hi), lo = v - hi - mid, each difference exact), so
// M v_e is three bfloat16 MFMAs whose products are exact in float32 and whose
// sums accumulate in float32: the float32 product to float32 rounding.  Row
// sums of M vanish, so a rigid translation maps to exactly zero.
//
// Tiling.  A 256-thread block takes a 16 x 16 element tile of one z layer and
// owns the 15 x 15 nodes interior to it; it marches up a chunk of node
// planes like the vector-ALU product.  Wave w takes element rows 4w .. 4w+3,
// one v_mfma_f32_16x16x32_bf16 set (16 elements along x) per row.  In one
// set, lane l = 16 g + e (e: element along x) holds as its B operand the 8
// values [x, y, z, 0] of the element's corner pair (ax = 0, 1) at (ay, az) =
// (g & 1, g >> 1) of one bfloat16 part, read from the node plane staged in
// LDS; the A operand is M with its rows permuted so that the result lands as
// lane 16 c + e holding component c of the element's 8 corners (4 corners
// per row block: two row blocks for az = 0, 1; lanes with c = 3 hold zero
// rows).  Each lane then scales by its element's modulus, and the corner
// values combine into nodes in a fixed order: along x by a DPP lane shift,
// along y between consecutive rows of the wave in registers (and between
// waves through LDS), along z by a carry from the layer below.  No atomics:
// the result is deterministic.
#include <hip/hip_ext.h>

#include <algorithm>
#include <cmath>
#include <cstring>

#include "common.h"
#include "device_common.h"
#include "mfma_block.h"

namespace topo {

#pragma clang fp contract(off)

// ---------------------------------------------------------------- host table
namespace {

// 1D integrals on [0, 1] of the linear shape functions phi_0 = 1 - x,
// phi_1 = x: value (dv = 0) or derivative (dv = 1) of phi_a against phi_b.
double int1d(int a, int da, int b, int db) {
  if (!da && !db) return a == b ? 1.0 / 3.0 : 1.0 / 6.0;
  if (da && db) return a == b ? 1.0 : -1.0;
  const int s = da ? a : b;  // the differentiated one: phi_0' = -1, phi_1' = +1
  return (s ? 1.0 : -1.0) * 0.5;
}

// 72 int d_i N_a d_k N_b over the unit cube (a, b: corners ax + 2 ay + 4 az)
double grad_grad(int a, int i, int b, int k) {
  double v = 72.0;
  for (int d = 0; d < 3; ++d)
    v *= int1d((a >> d) & 1, d == i, (b >> d) & 1, d == k);
  return v;
}

}  // namespace

bool mfma_operand_table(double nu, uint16_t out[2][64][8], float *mscale_unit) {
  const double lam = nu / ((1.0 + nu) * (1.0 - 2.0 * nu));
  const double mu = 1.0 / (2.0 * (1.0 + nu));
  const double rho = lam / mu;
  double M[24][24];
  for (int a = 0; a < 8; ++a)
    for (int i = 0; i < 3; ++i)
      for (int b = 0; b < 8; ++b)
        for (int k = 0; k < 3; ++k) {
          double Bv = grad_grad(a, k, b, i);
          if (i == k)
            for (int j = 0; j < 3; ++j) Bv += grad_grad(a, j, b, j);
          M[3 * a + i][3 * b + k] = Bv + rho * grad_grad(a, i, b, k);
        }
  bool exact = true;
  for (int r = 0; r < 2; ++r)
    for (int lane = 0; lane < 64; ++lane)
      for (int j = 0; j < 8; ++j) {
        // output row (lane % 16): component c_o = row / 4, corner (t & 1, t >> 1, r)
        const int row = lane % 16, c_o = row / 4, t = row % 4;
        const int a_o = (t & 1) + 2 * (t >> 1) + 4 * r;
        // input k = 8 (lane / 16) + j: corner pair (ay, az) = (g & 1, g >> 1),
        // then [ax = 0: x y z 0][ax = 1: x y z 0]
        const int g = lane / 16, ax = j / 4, c_i = j % 4;
        const int a_i = ax + 2 * (g & 1) + 4 * (g >> 1);
        const double v = (c_o < 3 && c_i < 3) ? M[3 * a_o + c_o][3 * a_i + c_i] : 0.0;
        const float f = (float)v;
        uint32_t bits;
        std::memcpy(&bits, &f, 4);
        const uint16_t hb = (uint16_t)(bits >> 16);  // exact values only: truncation = the value
        uint32_t back = (uint32_t)hb << 16;
        float fb;
        std::memcpy(&fb, &back, 4);
        if ((double)fb != v) exact = false;
        out[r][lane][j] = hb;
      }
  *mscale_unit = (float)(mu / 72.0);  // k0 = (mu / 72) M on the unit cube; times h and E_e
  return exact;
}

template <int MODE>
__global__ __launch_bounds__(MF_THREADS) void k_matvec_mfma(const MvArgs<float> a, int tx, int ty) {
  __shared__ MfmaLds S;
  __shared__ double red[MF_THREADS / 64];
  const int NZ = a.nelz + 1, tz = (NZ + a.kz - 1) / a.kz;
  const int lb = mv_local((int)blockIdx.x, tx * ty, tz);
  if (lb < 0) return;  // padding of the last band
  mfma_block<MODE>(a, lb % tx, (lb / tx) % ty, lb / (tx * ty), [] {},
                   [](float &b) { b = 0.f; return true; }, S, red);
}

hipError_t launch_matvec_mfma(const MvArgs<float> &a, int *nblocks, hipStream_t s) {
  const int NX = a.nelx + 1, NY = a.nely + 1, NZ = a.nelz + 1;
  const int tx = (NX + MN - 1) / MN, ty = (NY + MN - 1) / MN, tz = (NZ + a.kz - 1) / a.kz;
  if (nblocks) *nblocks = tx * ty * tz;
  hipLaunchKernelGGL((k_matvec_mfma<MV_APPLY>), dim3(mv_grid(tx * ty, tz)), dim3(MF_THREADS), 0, s,
                     a, tx, ty);
  return hipGetLastError();
}

}  // namespace topo
