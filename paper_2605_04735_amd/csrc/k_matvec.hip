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
// Tiling.  A 256-thread block holds a 32 x 8 element tile of one z layer and
// owns the 31 x 7 nodes interior to it; it marches up a range of node planes.
// Per element layer L: node plane L+1 of the input (33 x 9 nodes) is staged
// in LDS next to plane L, every thread applies its element and writes its 24
// outputs to LDS, then every owned node sums, in a fixed order, the
// contributions of layer L-1 (kept in registers) and layer L.  No atomics: the
// result is deterministic.  Each element is computed by one block only in z
// and by up to four blocks in x/y (halo), 256/217 ~ 1.18x element work.  The
// tile is wide in x because the product is bound by its memory access pattern
// more than by its arithmetic: rows of 33 nodes (396 bytes of a float32
// vector) are fewer and longer segments per plane than rows of 17.
#include <hip/hip_ext.h>

#include <algorithm>

#include "common.h"
#include "device_common.h"
#include "mfma_block.h"

namespace topo {

// One block of the product: the TEX x TEY element tile (bx, by) marching over
// node planes [bz kz, bz kz + kz).  Returns the block's partial sum (CG:
// p^T q, RESID: ||r||^2) in thread 0.
//
// Each lane owns one element column of the tile and carries it up the z
// layers in transform space: the forward transform of the element's bottom
// face is the top face of the layer below (kept in registers), so per layer a
// lane reads only the 4 corners of node plane L+1 from LDS; the inverse
// transform's contributions to a node plane are accumulated as face
// transforms (top face of layer L-1 plus bottom face of layer L) and turned
// into corner values once per plane.  The owned node's value then combines
// the corners of the 4 elements around it: along x by a DPP lane shift (no
// LDS), along y through a 3-value LDS exchange with the next tile row.  Node
// plane L+2 is fetched into registers while layer L computes.  The
// summation order is fixed: the result is deterministic.
template <typename T, int MODE, bool ZBF = false, int ZF = ZF_READ, typename PreFn,
          typename BetaFn>
__device__ __forceinline__ double matvec_block(const MvArgs<T> &a, int bx, int by, int bz,
                                               PreFn &&pre, BetaFn &&get_beta,
                                               T (*pl)[3][TPX * TPY], T (*ex)[MV_THREADS],
                                               double *red) {
  // CG inputs (z, p) are zero on fixed DOFs by construction and q there is
  // never used (the update masks r), so only APPLY and RESID read the mask.
  // ZBF: the preconditioned residual z arrives in bfloat16 (float32 arithmetic,
  // float32 directions).
  constexpr bool CG = MODE == MV_CG;
  static_assert(!ZBF || (CG && sizeof(T) == 4), "bfloat16 z: float32 CG only");
  // CG without bfloat16 z under ZF_FORM (or ZF_DESC with the arguments'
  // zfuse set): the input is r and z = D r is formed here
  constexpr bool ZFC = CG && !ZBF && ZF != ZF_READ;  // z may be formed here
  const bool zf = ZFC && (ZF == ZF_FORM || a.zfuse);
  constexpr unsigned SZ = ZBF ? 2u : sizeof(T);  // bytes per component of the input vector
  constexpr bool MASKED = !CG;
  constexpr unsigned S = sizeof(T);
  const int tid = threadIdx.x;
  const int NX = a.nelx + 1, NY = a.nely + 1, NZ = a.nelz + 1;
  const int i0 = bx * TNX, j0 = by * TNY;
  const int k0 = bz * a.kz;
  const int k1 = min(k0 + a.kz, NZ);
  const unsigned plane = (unsigned)NX * (unsigned)NY;
  const unsigned eplane = (unsigned)a.nelx * (unsigned)a.nely;
  const unsigned nn = plane * (unsigned)NZ;
  const rsrc_t rIn = make_rsrc(a.in, 3u * nn * SZ);
  const rsrc_t rOut = make_rsrc(a.out, 3u * nn * S);
  const rsrc_t rE = make_rsrc(a.E, eplane * (unsigned)a.nelz * S);
  // (resources a mode does not use span 0 bytes and are never accessed)
  const rsrc_t rPo = make_rsrc(a.pold, CG ? 3u * nn * S : 0u);
  const rsrc_t rPn = make_rsrc(a.pout, CG ? 3u * nn * S : 0u);
  const rsrc_t rM = make_rsrc(a.mask, MASKED ? nn : 0u);
  const rsrc_t rF = make_rsrc(a.f, MODE == MV_RESID ? 3u * nn * 8u : 0u);

  const int ei = tid % TEX, ej = tid / TEX;
  const int gi = i0 - 1 + ei, gj = j0 - 1 + ej;
  const bool e_xy = gi >= 0 && gi < a.nelx && gj >= 0 && gj < a.nely;
  // the node owned by this lane: (i0 + ei, j0 + ej), interior of the tile
  const int gni = i0 + ei, gnj = j0 + ej;
  const bool own = ei < TNX && ej < TNY && gni < NX && gnj < NY;
  const unsigned nown = (unsigned)gni + (unsigned)NX * (unsigned)gnj;
  const unsigned voE = e_xy ? ((unsigned)gi + (unsigned)a.nelx * (unsigned)gj) * S : OOB;
  const unsigned voOwn = own ? 3u * S * nown : OOB;

  // per lane, two slots of the TPX x TPY node plane; their buffer offsets
  unsigned voN[2], voM[2], voP[2], voZ[2];  // voZ: the input vector (SZ bytes per component)
#pragma unroll
  for (int sl = 0; sl < 2; ++sl) {
    const int idx = tid + sl * MV_THREADS;
    const int li = idx % TPX, lj = idx / TPX;
    const int gx = i0 - 1 + li, gy = j0 - 1 + lj;
    const bool v = idx < TPX * TPY && gx >= 0 && gx < NX && gy >= 0 && gy < NY;
    const bool mine = li >= 1 && li <= TNX && lj >= 1 && lj <= TNY;
    const unsigned n = (unsigned)gx + (unsigned)NX * (unsigned)gy;
    voN[sl] = v ? 3u * S * n : OOB;
    voM[sl] = v ? n : OOB;
    voZ[sl] = v ? 3u * SZ * n : OOB;
    voP[sl] = v && mine ? 3u * S * n : OOB;
  }

  // register ring: two node planes (and the moduli of the element layer on
  // top of each) in flight while a layer computes
  struct Plane {
    T in[2][3], po[2][3];
    unsigned m[2];
    T e;
    T di[2];  // zf: Jacobi inverse diagonal
  };
  auto fetch = [&](Plane &R, int kp) {
    // a plane outside the grid reads through empty resources (all zeros):
    // no branch, so the waits on loads already in flight stay exact
    const bool inz = kp >= 0 && kp < NZ;  // uniform
    const unsigned kc = inz ? (unsigned)kp : 0u;
    const unsigned so = kc * plane * 3u * S;
    const unsigned sz = kc * plane * 3u * SZ;
    const rsrc_t ri = make_rsrc(a.in, inz ? 3u * nn * SZ : 0u);
    const rsrc_t rp = make_rsrc(a.pold, CG && inz ? 3u * nn * S : 0u);
    const rsrc_t rm = make_rsrc(a.mask, MASKED && inz ? nn : 0u);
    const rsrc_t re = make_rsrc(a.E, kp >= 0 && kp < a.nelz ? eplane * (unsigned)a.nelz * S : 0u);
    const rsrc_t rd = make_rsrc(a.dinv, zf && inz ? nn * S : 0u);
#pragma unroll
    for (int sl = 0; sl < 2; ++sl) {
      if constexpr (ZBF) bload3_bf16(ri, voZ[sl], sz, R.in[sl]);
      else bload3(ri, voZ[sl], sz, R.in[sl]);
      if constexpr (CG) bload3(rp, voN[sl], so, R.po[sl]);
      if constexpr (MASKED) R.m[sl] = bload_u8(rm, voM[sl], kc * plane);
      if constexpr (ZFC)
        R.di[sl] = bload1<T>(rd, voM[sl] == OOB ? OOB : voM[sl] * S, kc * plane * S);
    }
    R.e = bload1<T>(re, voE, kc * eplane * S);
  };
  T beta = 0;
  // plane kp into LDS (CG: p = z + beta p_old, and p written out for the
  // nodes this block owns); returns the moduli of element layer kp
  auto stage = [&](Plane &R, int kp) -> T {
    T(*dst)[TPX * TPY] = pl[kp & 1];
    const bool wr = CG && kp >= k0 && kp < k1;
#pragma unroll
    for (int sl = 0; sl < 2; ++sl) {
      const int idx = tid + sl * MV_THREADS;
      if (idx >= TPX * TPY) continue;
      T v[3];
#pragma unroll
      for (int c = 0; c < 3; ++c) {
        if constexpr (CG) {
          T z = R.in[sl][c];
          if constexpr (ZFC) {
            if (zf) z = mul_rn(R.di[sl], z);  // the z of the update's r^T z, bit for bit
          }
          v[c] = z + beta * R.po[sl][c];
        } else {
          v[c] = ((R.m[sl] >> c) & 1u) ? T(0) : R.in[sl][c];
        }
        dst[c][idx] = v[c];
      }
      if (wr) bstore3(rPn, voP[sl], (unsigned)kp * plane * 3u * S, v);
    }
    return R.e;
  };

  const int fidx = ei + TPX * ej;  // corner (0,0) of this lane's element face in a plane
  double acc = 0.0;
  T acc_t = 0;  // CG: this lane's p^T q terms (at most 3 kz), in the product's precision
  // one element layer L: faces Fb (plane L, transformed) -> Ft (plane L+1),
  // inverse-transform carry Gb (plane L so far) -> Gt (plane L+1 so far)
  auto layer = [&](int L, T E, T (&Fb)[3][4], T (&Ft)[3][4], T (&Gb)[3][4], T (&Gt)[3][4]) {
    T pn[3] = {0, 0, 0};
    if (CG && own) {
      const int idx = (ei + 1) + TPX * (ej + 1);
#pragma unroll
      for (int c = 0; c < 3; ++c) pn[c] = pl[L & 1][c][idx];
    }
    face_forward(pl[(L + 1) & 1], fidx, Ft);
    T C[3][8], D[3][8];
#pragma unroll
    for (int c = 0; c < 3; ++c)
#pragma unroll
      for (int m = 0; m < 4; ++m) {
        C[c][m] = Ft[c][m] + Fb[c][m];
        C[c][m + 4] = Ft[c][m] - Fb[c][m];
      }
    modal_stress(C, E, a.k, D);
    // inverse z butterfly: bottom (plane L) and top (plane L+1) face parts;
    // plane L is now complete in transform space
    T A[3][4];
#pragma unroll
    for (int c = 0; c < 3; ++c)
#pragma unroll
      for (int m = 0; m < 4; ++m) {
        A[c][m] = Gb[c][m] + (D[c][m] - D[c][m + 4]);
        Gt[c][m] = D[c][m] + D[c][m + 4];
      }
    // inverse x and y butterflies -> corner values y(ax, ay); then x combine
    T xc[3][2];
#pragma unroll
    for (int c = 0; c < 3; ++c) {
      const T e00 = A[c][0] - A[c][1], e10 = A[c][0] + A[c][1];  // my = 0
      const T e01 = A[c][2] - A[c][3], e11 = A[c][2] + A[c][3];  // my = 1
      const T y00 = e00 - e01, y01 = e00 + e01;                  // ax = 0
      const T y10 = e10 - e11, y11 = e10 + e11;                  // ax = 1
      xc[c][0] = y10 + from_next_lane(y00);
      xc[c][1] = y11 + from_next_lane(y01);
      ex[c][tid] = xc[c][0];
    }
    __syncthreads();
    if (own && L >= k0) {
      const unsigned so = (unsigned)L * plane * 3u * S;
      T val[3];
#pragma unroll
      for (int c = 0; c < 3; ++c) val[c] = xc[c][1] + ex[c][tid + TEX];
      if constexpr (MODE == MV_CG) {
        bstore3(rOut, voOwn, so, val);
#pragma unroll
        for (int c = 0; c < 3; ++c) acc_t += pn[c] * val[c];
      } else {
        const unsigned m = bload_u8(rM, nown, (unsigned)L * plane);
        if constexpr (MODE == MV_APPLY) {
          T u[3];
          bload3(rIn, voOwn, so, u);
#pragma unroll
          for (int c = 0; c < 3; ++c) val[c] = ((m >> c) & 1u) ? u[c] : val[c];
          bstore3(rOut, voOwn, so, val);
        } else {
          double f[3];
          bload3(rF, 3u * 8u * nown, (unsigned)L * plane * 24u, f);
          T r[3];
#pragma unroll
          for (int c = 0; c < 3; ++c) {
            const double rd = ((m >> c) & 1u) ? 0.0 : f[c] - (double)val[c];
            r[c] = (T)rd;
            acc += rd * rd;
          }
          bstore3(rOut, voOwn, so, r);
        }
      }
    }
  };

  Plane R0, R1;
  pre();  // loads of the step's scalars (CG: the previous reduction) first
  fetch(R0, k0 - 1);
  fetch(R1, k0);
  // the scalars complete while the first planes are in flight; false:
  // nothing to do for this design
  if (!get_beta(beta)) return 0.0;
  T E = stage(R0, k0 - 1);
  if (k0 + 1 <= k1) fetch(R0, k0 + 1);
  __syncthreads();
  T Fa[3][4], Fb[3][4], Ga[3][4], Gb[3][4];
  face_forward(pl[(k0 - 1) & 1], fidx, Fa);
#pragma unroll
  for (int c = 0; c < 3; ++c)
#pragma unroll
    for (int m = 0; m < 4; ++m) Ga[c][m] = 0;
  // layer L stages plane L + 1 from the ring and refills its set with plane
  // L + 3; unrolled by two so that ring sets and carries alternate statically
  for (int L = k0 - 1;;) {
    {
      const T En = stage(R1, L + 1);
      if (L + 3 <= k1) fetch(R1, L + 3);
      __syncthreads();
      layer(L, E, Fa, Fb, Ga, Gb);
      E = En;
    }
    if (++L >= k1) break;
    {
      const T En = stage(R0, L + 1);
      if (L + 3 <= k1) fetch(R0, L + 3);
      __syncthreads();
      layer(L, E, Fb, Fa, Gb, Ga);
      E = En;
    }
    if (++L >= k1) break;
  }
  if constexpr (MODE == MV_CG) acc = (double)acc_t;
  if (MODE != MV_APPLY) return block_sum_d(acc, red);
  return 0.0;
}

template <typename T, int MODE>
__global__ __launch_bounds__(MV_THREADS) __attribute__((amdgpu_waves_per_eu(3)))
void k_matvec(const MvArgs<T> a, int tx, int ty) {
  __shared__ T pl[2][3][TPX * TPY];
  __shared__ T ex[3][MV_THREADS];
  __shared__ double red[MV_THREADS / 64];
  const int NZ = a.nelz + 1, tz = (NZ + a.kz - 1) / a.kz;
  const int lb = mv_local((int)blockIdx.x, tx * ty, tz);
  if (lb < 0) return;  // padding of the last band
  const double s = matvec_block<T, MODE>(
      a, lb % tx, (lb / tx) % ty, lb / (tx * ty), [] {}, [](T &b) { b = T(0); return true; }, pl,
      ex, red);
  if (MODE != MV_APPLY && threadIdx.x == 0) a.part[lb] = s;
}

// Inner-CG product, local block lb of design d.  Every block first completes
// the reduction of the previous update (r^T z and ||r||^2, partial set
// parity^1): converged designs stop here; otherwise beta = (r^T z)_new /
// (r^T z)_old, p = z + beta p_old (z = D r formed here from r when the
// descriptor's zfuse is set, else read as the update stored it), q = K p, and
// the block's p^T q partial is written for the update kernel.
template <typename T, bool ZBF = false, bool MF = false, int ZF = ZF_DESC>
__device__ __forceinline__ void cg_matvec_block(const CgDesc<T> &d, double *scal, int *flags,
                                                double *cgp, int nparts, int lb_in, int slot) {
  const int parity = slot & 1;
  static_assert(!MF || (sizeof(T) == 4 && !ZBF), "matrix-core product: float32 CG, float32 z");
  constexpr int BT = MF ? MF_THREADS : MV_THREADS;  // threads of this block
  __shared__ double red[4 * (BT / 64)];
  bool run = false;
  // the r^T z and ||r||^2 partials are loaded before the first planes, the
  // flags and scalars in the same round trip; a finished design only costs
  // this block its loads
  constexpr int NP = ZBF ? 4 : 2;  // bfloat16 z: also r^T p_old, z^T q_old
  const double *parts[NP];
  parts[0] = cgp + CGP_RZ + (parity ^ 1) * MAXB;
  parts[1] = cgp + CGP_RR + (parity ^ 1) * MAXB;
  if constexpr (ZBF) {
    parts[2] = cgp + CGP_RP + (parity ^ 1) * MAXB;
    parts[3] = cgp + CGP_ZQ + (parity ^ 1) * MAXB;
  }
  Partials<2, NP, BT> P;
  int done = 0, iters = 0, cap = 0;
  double rz_old = 0.0, tol2 = 0.0, pq_old = 0.0;
  // first the loads that need nothing but the leading arguments
  P.load(parts, nparts);
  {  // buffer loads from the preloaded pointers, issued with the partials
    const rsrc_t rf = make_rsrc(flags, F_COUNT * 4u), rs = make_rsrc(scal, S_COUNT * 8u);
    done = (int)__builtin_amdgcn_raw_buffer_load_b32(rf, 4 * F_DONE, 0, 0);
    iters = (int)__builtin_amdgcn_raw_buffer_load_b32(rf, 4 * F_ITERS, 0, 0);
    cap = (int)__builtin_amdgcn_raw_buffer_load_b32(rf, 4 * F_CAP, 0, 0);
    rz_old = bload1d(rs, 8u * (S_RZ0 + parity), 0);
    tol2 = bload1d(rs, 8u * S_TOL2, 0);
    if constexpr (ZBF) pq_old = bload1d(rs, 8u * S_PQ, 0);
  }
  __builtin_amdgcn_sched_barrier(0);  // keep those loads first
  // then every descriptor field in one round trip (the empty asm makes the
  // values needed at once, so their loads issue together)
  MvArgs<T> a;
  a.nelx = d.nelx;
  a.nely = d.nely;
  a.nelz = d.nelz;
  a.kz = d.kz;
  a.E = d.E;
  a.zfuse = ZBF || ZF == ZF_READ ? 0 : ZF == ZF_FORM ? 1 : d.zfuse;
  a.in = a.zfuse ? d.r : d.z;
  a.dinv = d.dinv;
  // the previous direction in slot s, the new one into slot s + 1 (mod np)
  const int np = d.np == 4 ? 4 : 2;
  T *const p0 = d.p[slot], *const p1 = d.p[slot + 1 == np ? 0 : slot + 1];
  a.pold = p0;
  a.pout = p1;
  a.out = d.q;
  a.mask = d.mask;
  a.k = d.k;
  a.mA = d.mA;
  a.mscale = d.mscale;
  const int tx = d.tx, ty = d.ty;
  // local block: from the table (batched), or this block's place (mv_local)
  const int lb = lb_in >= 0 ? lb_in : mv_local((int)blockIdx.x, tx * ty, d.nb_mv / (tx * ty));
  if (lb < 0) return;  // padding of the last band: nothing loaded is used
  asm volatile("" ::"s"(a.nelx), "s"(a.nely), "s"(a.nelz), "s"(a.kz), "s"(tx), "s"(ty), "s"(a.E),
               "s"(a.in), "s"(p0), "s"(p1), "s"(a.out), "s"(a.k.L2), "s"(a.k.M4), "s"(a.k.M2),
               "s"(a.k.L2_3), "s"(a.k.M2_3), "s"(a.k.B9), "s"(a.dinv), "s"(a.zfuse));
  const int bx = lb % tx, by = (lb / tx) % ty, bz = lb / (tx * ty);
  auto get_beta = [&](T &beta) -> bool {
    double sums[NP];
    P.sum(parts, nparts, red, sums);
    const double rz = sums[0], rr = sums[1];
    if (done) return false;
    const bool bad = !isfinite(rz) || !isfinite(rr);
    if (bad || rr <= tol2 || iters >= cap) {
      if (lb == 0 && threadIdx.x == 0) {
        if (bad) flags[F_STATUS] = 2;
        scal[S_RR] = rr;
        flags[F_DONE] = 1;
      }
      return false;
    }
    double b = rz / rz_old;
    if constexpr (ZBF) b = iters == 0 ? 0.0 : -sums[3] / pq_old;
    if (lb == 0 && threadIdx.x == 0) {
      scal[S_RZ0 + (parity ^ 1)] = rz;
      scal[S_RR] = rr;
      if constexpr (ZBF) {
        scal[S_BETA] = b;
        scal[S_RP] = sums[2];
      }
    }
    beta = (T)b;
    run = true;
    return true;
  };
  double s;
  if constexpr (MF) {
    __shared__ MfmaLds S;
    s = mfma_block<MV_CG, ZF>(a, bx, by, bz, [] {}, get_beta, S, red);
  } else {
    __shared__ T pl[2][3][TPX * TPY];
    __shared__ T ex[6][MV_THREADS];
    s = matvec_block<T, MV_CG, ZBF, ZF>(a, bx, by, bz, [] {}, get_beta, pl, ex, red);
  }
  if (run && threadIdx.x == 0) cgp[CGP_PQ + lb] = s;
}

// Batched form over a table of designs: blockmap[b] = (design, local block).
template <typename T>
__global__ __launch_bounds__(MV_THREADS) void k_cg_matvec(const CgDesc<T> *descs,
                                                          const BlockEntry *blockmap, int parity) {
  const BlockEntry be = blockmap[blockIdx.x];
  if (be.design < 0) return;  // padding entry
  cg_matvec_block<T>(descs[be.design], be.scal, be.flags, be.cgp, be.nparts, be.lb, parity);
}

// One design, its descriptor passed by value.  The scalars, flags, partial
// sums, parity and partial count lead the arguments (8 dwords) so that they
// arrive preloaded in SGPRs: the block's first loads (the previous reduction)
// need no argument load before them.
template <typename T, bool ZBF, bool MF = false, int ZF = ZF_READ>
__global__ __launch_bounds__(MF ? MF_THREADS : MV_THREADS) void k_cg_matvec1(double *scal, int *flags, double *cgp,
                                                           int slot, int nparts,
                                                           const CgDesc<T> d) {
  cg_matvec_block<T, ZBF, MF, ZF>(d, scal, flags, cgp, nparts, -1, slot);
}

// Batched CG vector update: every block completes the p^T q reduction of the
// product, alpha = (r^T z) / (p^T q), then x += alpha p; r -= alpha q
// (fixed DOFs 0); z = D r, stored unless the product forms it (zfuse), and
// the block's r^T z and ||r||^2 partials go to set `parity` for the next
// product.  A thread's first two nodes are loaded before the reduction, so
// their latency overlaps it.
template <typename T, bool ZBF = false, int XU = XU_EACH>
__device__ __forceinline__ void cg_update_block(const CgDesc<T> &d, double *scal, int *flags,
                                                double *cgp, int nparts, int lb, int slot) {
  static_assert(XU == XU_EACH || !ZBF, "grouped x: float32 or float64 z");
  constexpr bool FL = XU == XU_FLUSH2 || XU == XU_FLUSH4;  // the grouped x update
  constexpr int NG = XU == XU_FLUSH4 ? 4 : 2;               // its group size
  __shared__ double red[8];
  const int parity = slot & 1;
  constexpr unsigned S = sizeof(T);
  constexpr unsigned SZ = ZBF ? 2u : sizeof(T);  // stored z component
  // first the loads that need nothing but the leading arguments
  const double *const parts[1] = {cgp + CGP_PQ};
  Partials<4, 1> P;
  P.load(parts, nparts);
  const rsrc_t rf = make_rsrc(flags, F_COUNT * 4u), rs = make_rsrc(scal, S_COUNT * 8u);
  const int done = (int)__builtin_amdgcn_raw_buffer_load_b32(rf, 4 * F_DONE, 0, 0);
  double rz = bload1d(rs, 8u * (S_RZ0 + (parity ^ 1)), 0);
  // bfloat16 z (a preconditioner that varies with the rounding): the exact
  // line search along p, r^T p = r^T z + beta r^T p_old
  if constexpr (ZBF) rz += bload1d(rs, 8u * S_BETA, 0) * bload1d(rs, 8u * S_RP, 0);
  // grouped x (the update of slot np - 2): the step lengths of slots 0 ..
  // np - 2, kept by the updates before this one
  double ah[3] = {0.0, 0.0, 0.0};
  if constexpr (FL) {
#pragma unroll
    for (int j = 0; j < NG - 1; ++j) ah[j] = bload1d(rs, 8u * (S_AH + j), 0);
  }
  __builtin_amdgcn_sched_barrier(0);  // keep those loads first
  // then the descriptor fields in one round trip
  const unsigned nn = (unsigned)d.nn;
  T *const x = d.x, *const r = d.r, *const z = d.z, *const q = d.q;
  // the direction the product just wrote: slot s + 1 (mod np); the grouped
  // update reads all np slots
  T *const pn = d.p[slot ^ 1];  // np = 2: slot ^ 1 = slot + 1 (mod 2)
  T *const pf0 = d.p[0], *const pf1 = d.p[1], *const pf2 = d.p[2], *const pf3 = d.p[NG - 1];
  const T *const dinv = d.dinv;
  const uint8_t *const mask = d.mask;
  const int nb_up = d.nb_up, zfuse = d.zfuse;
  if constexpr (XU == XU_FLUSH4)
    asm volatile("" ::"s"(nn), "s"(x), "s"(r), "s"(z), "s"(q), "s"(pf0), "s"(pf1), "s"(pf2),
                 "s"(pf3), "s"(dinv), "s"(mask), "s"(nb_up), "s"(zfuse));
  else if constexpr (XU == XU_FLUSH2)
    asm volatile("" ::"s"(nn), "s"(x), "s"(r), "s"(z), "s"(q), "s"(pf0), "s"(pf3), "s"(dinv),
                 "s"(mask), "s"(nb_up), "s"(zfuse));
  else if constexpr (XU == XU_EACH)
    asm volatile("" ::"s"(nn), "s"(x), "s"(r), "s"(z), "s"(q), "s"(pn), "s"(dinv), "s"(mask),
                 "s"(nb_up), "s"(zfuse));
  else
    asm volatile("" ::"s"(nn), "s"(r), "s"(z), "s"(q), "s"(dinv), "s"(mask), "s"(nb_up),
                 "s"(zfuse));
  const bool zst = ZBF || !zfuse;  // z is stored for the product
  constexpr bool XA = XU != XU_SKIP;  // x advances in this launch
  const rsrc_t rX = make_rsrc(x, XA ? 3u * nn * S : 0u), rR = make_rsrc(r, 3u * nn * S);
  const rsrc_t rZ = make_rsrc(z, zst ? 3u * nn * SZ : 0u), rQ = make_rsrc(q, 3u * nn * S);
  // the last direction of a group is the one just written: slot NG - 1
  const rsrc_t rP = make_rsrc(FL ? pf3 : pn, XA ? 3u * nn * S : 0u);
  const rsrc_t rP0 = make_rsrc(pf0, FL ? 3u * nn * S : 0u);
  const rsrc_t rP1 = make_rsrc(pf1, XU == XU_FLUSH4 ? 3u * nn * S : 0u);
  const rsrc_t rP2 = make_rsrc(pf2, XU == XU_FLUSH4 ? 3u * nn * S : 0u);
  const rsrc_t rD = make_rsrc(dinv, nn * S), rM = make_rsrc(mask, nn);
  const unsigned stride = (unsigned)nb_up * 256u;
  struct Node {
    T x[3], p[3], r[3], q[3], di;
    T pg[3][3];  // grouped x: the directions of slots 0 .. NG - 2
    unsigned m, vo, vz;  // vz: offset of the node's z (SZ bytes per component)
  };
  auto load = [&](Node &v, unsigned n) {
    const bool in = n < nn;  // (n < nn + 4 stride: far below 2^32 for any accepted grid)
    v.vo = in ? 3u * S * n : OOB;
    v.vz = in ? 3u * SZ * n : OOB;
    if constexpr (XA) {
      bload3(rX, v.vo, 0, v.x);
      bload3(rP, v.vo, 0, v.p);
    }
    if constexpr (FL) bload3(rP0, v.vo, 0, v.pg[0]);
    if constexpr (XU == XU_FLUSH4) {
      bload3(rP1, v.vo, 0, v.pg[1]);
      bload3(rP2, v.vo, 0, v.pg[2]);
    }
    bload3(rR, v.vo, 0, v.r);
    bload3(rQ, v.vo, 0, v.q);
    v.di = bload1<T>(rD, in ? S * n : OOB, 0);
    v.m = bload_u8(rM, in ? n : OOB, 0);
  };
  const unsigned n0 = (unsigned)lb * 256u + threadIdx.x;
  Node A, B;
  load(A, n0);
  load(B, n0 + stride);
  double pqs[1];
  P.sum(parts, nparts, red, pqs);
  const double pq = pqs[0];
  if (done) return;
  if (!(pq > 0.0) || !isfinite(pq)) {
    if (lb == 0 && threadIdx.x == 0) {
      scal[S_PQ] = pq;
      flags[F_STATUS] = isfinite(pq) ? 1 : 2;
      flags[F_DONE] = 1;
    }
    return;
  }
  const T alpha = (T)(rz / pq);
  const T a0 = (T)ah[0], a1 = (T)ah[1], a2 = (T)ah[2];
  double rzs = 0.0, rrs = 0.0, rps = 0.0, zqs = 0.0;
  auto update = [&](const Node &v) {
    T xn[3], rn[3], zn[3];
#pragma unroll
    for (int c = 0; c < 3; ++c) {
      if constexpr (XU == XU_FLUSH4)  // the steps in the order they were taken
        xn[c] = v.x[c] + a0 * v.pg[0][c] + a1 * v.pg[1][c] + a2 * v.pg[2][c] + alpha * v.p[c];
      else if constexpr (XU == XU_FLUSH2)
        xn[c] = v.x[c] + a0 * v.pg[0][c] + alpha * v.p[c];
      else if constexpr (XU == XU_EACH)
        xn[c] = v.x[c] + alpha * v.p[c];
      rn[c] = ((v.m >> c) & 1u) ? T(0) : v.r[c] - alpha * v.q[c];
      zn[c] = mul_rn(v.di, rn[c]);
      if constexpr (ZBF) zn[c] = bf16_round(zn[c]);  // the z the next product reads
      rzs += (double)rn[c] * (double)zn[c];
      rrs += (double)rn[c] * (double)rn[c];
      if constexpr (ZBF) {
        rps += (double)rn[c] * (double)v.p[c];
        zqs += (double)zn[c] * (double)v.q[c];
      }
    }
    if constexpr (XA) bstore3(rX, v.vo, 0, xn);
    bstore3(rR, v.vo, 0, rn);
    if constexpr (ZBF) bstore3_bf16(rZ, v.vz, 0, zn);
    else bstore3(rZ, v.vz, 0, zn);  // (an empty resource drops it under zfuse)
  };
  // pairs of nodes, the next pair's loads in flight while a pair updates;
  // every thread runs the same number of pairs (nodes past nn load 0 and
  // their stores are dropped), so the loop has no divergent exit and its
  // waits stay exact
  const unsigned npair = (nn + 2u * stride - 1u) / (2u * stride);
  Node C, D;
  for (unsigned k = 0;; k += 2) {
    const unsigned n1 = n0 + (k + 1) * 2u * stride;
    load(C, n1);
    load(D, n1 + stride);
    update(A);
    update(B);
    if (k + 1 >= npair) break;
    const unsigned n2 = n0 + (k + 2) * 2u * stride;
    load(A, n2);
    load(B, n2 + stride);
    update(C);
    update(D);
    if (k + 2 >= npair) break;
  }
  double s1, s2, s3 = 0.0, s4 = 0.0;
  if constexpr (ZBF) {
    block_sum_d2(rzs, rrs, red, s1, s2);
    __syncthreads();
    block_sum_d2(rps, zqs, red, s3, s4);
  } else {
    block_sum_d2(rzs, rrs, red, s1, s2);
  }
  if (threadIdx.x == 0) {
    if constexpr (ZBF) {
      cgp[CGP_RP + parity * MAXB + lb] = s3;
      cgp[CGP_ZQ + parity * MAXB + lb] = s4;
    }
    cgp[CGP_RZ + parity * MAXB + lb] = s1;
    cgp[CGP_RR + parity * MAXB + lb] = s2;
    if (lb == 0) {
      scal[S_PQ] = pq;
      scal[S_ALPHA] = rz / pq;
      // grouped x: the step of the direction in slot s + 1, for the flush or
      // for the solution update if the CG stops before the flush
      if constexpr (XU != XU_EACH) scal[S_AH + (slot + 1 == (d.np == 4 ? 4 : 2) ? 0 : slot + 1)] = rz / pq;
      flags[F_ITERS] = flags[F_ITERS] + 1;
    }
  }
}

// (x grouped by two over the batch: every design of a batch has np = 2 and
// xgroup set, and the launch of parity 0 is the grouped x update)
template <typename T, int XU = XU_EACH>
__global__ __launch_bounds__(256) void k_cg_update(const CgDesc<T> *descs,
                                                   const BlockEntry *blockmap, int parity) {
  const BlockEntry be = blockmap[blockIdx.x];
  if (be.design < 0) return;  // padding entry
  cg_update_block<T, false, XU>(descs[be.design], be.scal, be.flags, be.cgp, be.nparts, be.lb,
                                parity);
}

template <typename T, bool ZBF, int XU = XU_EACH>
__global__ __launch_bounds__(256) void k_cg_update1(double *scal, int *flags, double *cgp,
                                                    int slot, int nparts, const CgDesc<T> d) {
  cg_update_block<T, ZBF, XU>(d, scal, flags, cgp, nparts, blockIdx.x, slot);
}

namespace {
// the kz whose equal-sized chunks give about `target` blocks, at least 2
int kz_for_target(int NZ, int tiles, int target) {
  int chunks = std::max(1, target / tiles);
  int kz = (NZ + chunks - 1) / chunks;
  if (kz < 2) kz = 2;
  if (kz > 32) kz = 32;
  chunks = (NZ + kz - 1) / kz;
  kz = (NZ + chunks - 1) / chunks;
  return kz < 2 ? 2 : kz;
}
}  // namespace

int matvec_kz(const Grid &g, bool fp64, bool mfma) {
  const int NX = g.nelx + 1, NY = g.nely + 1, NZ = g.nelz + 1;
  const int tnx = mfma ? MN : TNX, tny = mfma ? MN : TNY;
  const int tiles = ((NX + tnx - 1) / tnx) * ((NY + tny - 1) / tny);
  if (const char *e = getenv("TOPO_KZ")) {
    int v = atoi(e);
    if (v >= 1) {
      while (v < NZ && tiles * ((NZ + v - 1) / v) > MAXB) ++v;
      return v;
    }
  }
  // About 8 blocks per CU on large grids, with the node planes split into
  // chunks of (nearly) equal size: a short last chunk leaves its blocks idle
  // for most of the launch.  A chunk of kz planes recomputes (kz + 1)/kz
  // element layers, so small grids trade blocks for longer chunks:
  // - float32 (five blocks of the product resident per CU): kz = 3 while that
  //   still leaves about 2.5 blocks per CU;
  // - float64 (two resident per CU): about 512 blocks, one round of the
  //   resident blocks, with kz at most 12 (the large-grid optimum).
  const int sc = mfma ? 1 : MV_BLOCK_SCALE;  // the targets are for 256-thread blocks
  int kz = kz_for_target(NZ, tiles, 2048 / sc);
  if (!fp64 && kz < 3 && tiles * ((NZ + 2) / 3) >= 640 / sc) kz = 3;
  if (fp64) kz = std::max(kz, std::min(kz_for_target(NZ, tiles, 512 / sc), 12));
  // partial sums must fit (a grid whose tiles alone exceed the bound is
  // rejected before this is reached)
  while (kz < NZ && tiles * ((NZ + kz - 1) / kz) > MAXB) ++kz;
  return kz;
}

int matvec_blocks(const Grid &g, int kz, bool mfma) {
  const int NX = g.nelx + 1, NY = g.nely + 1, NZ = g.nelz + 1;
  const int tnx = mfma ? MN : TNX, tny = mfma ? MN : TNY;
  return ((NX + tnx - 1) / tnx) * ((NY + tny - 1) / tny) * ((NZ + kz - 1) / kz);
}

template <typename T, int MODE>
hipError_t launch_matvec(const MvArgs<T> &a, int *nblocks, hipStream_t s) {
  const int NX = a.nelx + 1, NY = a.nely + 1, NZ = a.nelz + 1;
  const int tx = (NX + TNX - 1) / TNX, ty = (NY + TNY - 1) / TNY, tz = (NZ + a.kz - 1) / a.kz;
  const int nb = tx * ty * tz;
  if (nblocks) *nblocks = nb;
  if (MODE != MV_APPLY && nb > MAXB) return hipErrorInvalidConfiguration;
  hipLaunchKernelGGL((k_matvec<T, MODE>), dim3(mv_grid(tx * ty, tz)), dim3(MV_THREADS), 0, s, a,
                     tx, ty);
  return hipGetLastError();
}

template <typename T>
hipError_t launch_cg_matvec(const CgDesc<T> *descs, const BlockEntry *bmap_mv, int nb_mv, int parity,
                            hipStream_t s, hipEvent_t start, hipEvent_t stop) {
  if (start && stop)  // timestamps taken by the dispatch itself
    hipExtLaunchKernelGGL(k_cg_matvec<T>, dim3(nb_mv), dim3(MV_THREADS), 0, s, start, stop, 0,
                          descs, bmap_mv, parity);
  else
    hipLaunchKernelGGL(k_cg_matvec<T>, dim3(nb_mv), dim3(MV_THREADS), 0, s, descs, bmap_mv, parity);
  return hipGetLastError();
}

template <typename T>
hipError_t launch_cg_update(const CgDesc<T> *descs, const BlockEntry *bmap_up, int nb_up, int parity,
                            hipStream_t s) {
  if (parity == 0)
    hipLaunchKernelGGL((k_cg_update<T, XU_FLUSH2>), dim3(nb_up), dim3(256), 0, s, descs, bmap_up,
                       parity);
  else
    hipLaunchKernelGGL((k_cg_update<T, XU_SKIP>), dim3(nb_up), dim3(256), 0, s, descs, bmap_up,
                       parity);
  return hipGetLastError();
}

template hipError_t launch_matvec<double, MV_APPLY>(const MvArgs<double> &, int *, hipStream_t);
template hipError_t launch_matvec<double, MV_RESID>(const MvArgs<double> &, int *, hipStream_t);
template hipError_t launch_matvec<float, MV_APPLY>(const MvArgs<float> &, int *, hipStream_t);
// the single-design product kernel for descriptor d: bfloat16 z, matrix-core
// or vector-ALU product, z formed inside or read
template <typename T>
void *cg_matvec1_kernel(const CgDesc<T> &d) {
  if constexpr (sizeof(T) == 4) {
    if (d.zbf16) return (void *)k_cg_matvec1<T, true>;
    if (d.mA)
      return d.zfuse ? (void *)k_cg_matvec1<T, false, true, ZF_FORM>
                     : (void *)k_cg_matvec1<T, false, true, ZF_READ>;
  }
  return d.zfuse ? (void *)k_cg_matvec1<T, false, false, ZF_FORM>
                 : (void *)k_cg_matvec1<T, false, false, ZF_READ>;
}

template <typename T>
hipError_t launch_cg_matvec1(const CgDesc<T> &d, int slot, hipStream_t s, hipEvent_t start,
                             hipEvent_t stop) {
  const dim3 grid(mv_grid(d.tx * d.ty, d.nb_mv / (d.tx * d.ty)));
  double *scal = d.scal, *cgp = d.cgp;
  int *flags = d.flags, nparts = d.nb_up;
  CgDesc<T> dd = d;
  void *args[] = {&scal, &flags, &cgp, &slot, &nparts, &dd};
  // timestamps taken by the dispatch itself when events are given
  return hipExtLaunchKernel(cg_matvec1_kernel(d), grid, dim3(d.mA ? MF_THREADS : MV_THREADS), args, 0, s, start, stop,
                            0);
}

// the single-design update kernel for descriptor d at direction slot `slot`
template <typename T>
void *cg_update1_kernel(const CgDesc<T> &d, int slot) {
  if constexpr (sizeof(T) == 4) {
    if (d.zbf16) return (void *)k_cg_update1<T, true>;
  }
  if (!d.xgroup) return (void *)k_cg_update1<T, false, XU_EACH>;
  const int np = d.np == 4 ? 4 : 2;
  if (slot != np - 2) return (void *)k_cg_update1<T, false, XU_SKIP>;
  return np == 4 ? (void *)k_cg_update1<T, false, XU_FLUSH4>
                 : (void *)k_cg_update1<T, false, XU_FLUSH2>;
}

template <typename T>
hipError_t launch_cg_update1(const CgDesc<T> &d, int slot, hipStream_t s) {
  double *scal = d.scal, *cgp = d.cgp;
  int *flags = d.flags, nparts = d.nb_mv;
  CgDesc<T> dd = d;
  void *args[] = {&scal, &flags, &cgp, &slot, &nparts, &dd};
  return hipLaunchKernel(cg_update1_kernel(d, slot), dim3(d.nb_up), dim3(256), args, 0, s);
}

// A graph of `iters` CG iterations (product then update, direction slots from
// slot0 on) for one design: the same launches as launch_cg_matvec1 /
// launch_cg_update1, built as explicit kernel nodes in a chain.
template <typename T>
hipError_t build_cg_graph(const CgDesc<T> &d, int slot0, int iters, hipGraphExec_t *out) {
  *out = nullptr;
  hipGraph_t g = nullptr;
  hipError_t e = hipGraphCreate(&g, 0);
  if (e != hipSuccess) return e;
  void *fmv = cg_matvec1_kernel(d);
  const int np = d.np == 4 ? 4 : 2;
  hipGraphNode_t prev = nullptr;
  for (int i = 0; i < 2 * iters && e == hipSuccess; ++i) {
    int slot = (slot0 + (i >> 1)) % np;
    const bool mv = (i & 1) == 0;
    int nparts = mv ? d.nb_up : d.nb_mv;
    double *scal = d.scal, *cgp = d.cgp;
    int *flags = d.flags;
    CgDesc<T> dd = d;
    void *args[] = {&scal, &flags, &cgp, &slot, &nparts, &dd};
    hipKernelNodeParams kp{};
    kp.func = mv ? fmv : cg_update1_kernel(d, slot);
    kp.gridDim = dim3(mv ? mv_grid(d.tx * d.ty, d.nb_mv / (d.tx * d.ty)) : d.nb_up);
    kp.blockDim = dim3(mv ? (d.mA ? MF_THREADS : MV_THREADS) : 256);
    kp.sharedMemBytes = 0;
    kp.kernelParams = args;
    kp.extra = nullptr;
    hipGraphNode_t node = nullptr;
    e = hipGraphAddKernelNode(&node, g, prev ? &prev : nullptr, prev ? 1 : 0, &kp);
    prev = node;
  }
  if (e == hipSuccess) e = hipGraphInstantiate(out, g, nullptr, nullptr, 0);
  hipGraphDestroy(g);
  return e;
}
template hipError_t build_cg_graph<double>(const CgDesc<double> &, int, int, hipGraphExec_t *);

// The same for the batched kernels over device tables (their contents may
// change between replays only while no replay is queued).
template <typename T>
hipError_t build_cg_graph_batched(const CgDesc<T> *descs, const BlockEntry *bmv, int nb_mv,
                                  const BlockEntry *bup, int nb_up, int parity0, int iters,
                                  hipGraphExec_t *out) {
  *out = nullptr;
  hipGraph_t g = nullptr;
  hipError_t e = hipGraphCreate(&g, 0);
  if (e != hipSuccess) return e;
  hipGraphNode_t prev = nullptr;
  for (int i = 0; i < 2 * iters && e == hipSuccess; ++i) {
    int parity = parity0 ^ ((i >> 1) & 1);
    const bool mv = (i & 1) == 0;
    const CgDesc<T> *dp = descs;
    const BlockEntry *bp = mv ? bmv : bup;
    void *args[] = {&dp, &bp, &parity};
    hipKernelNodeParams kp{};
    kp.func = mv ? (void *)k_cg_matvec<T>
                 : parity == 0 ? (void *)k_cg_update<T, XU_FLUSH2> : (void *)k_cg_update<T, XU_SKIP>;
    kp.gridDim = dim3(mv ? nb_mv : nb_up);
    kp.blockDim = dim3(mv ? MV_THREADS : 256);
    kp.sharedMemBytes = 0;
    kp.kernelParams = args;
    kp.extra = nullptr;
    hipGraphNode_t node = nullptr;
    e = hipGraphAddKernelNode(&node, g, prev ? &prev : nullptr, prev ? 1 : 0, &kp);
    prev = node;
  }
  if (e == hipSuccess) e = hipGraphInstantiate(out, g, nullptr, nullptr, 0);
  hipGraphDestroy(g);
  return e;
}
template hipError_t build_cg_graph_batched<float>(const CgDesc<float> *, const BlockEntry *, int,
                                                  const BlockEntry *, int, int, int,
                                                  hipGraphExec_t *);
template hipError_t build_cg_graph<float>(const CgDesc<float> &, int, int, hipGraphExec_t *);

template hipError_t launch_cg_matvec1<double>(const CgDesc<double> &, int, hipStream_t, hipEvent_t,
                                              hipEvent_t);
template hipError_t launch_cg_matvec1<float>(const CgDesc<float> &, int, hipStream_t, hipEvent_t,
                                             hipEvent_t);
template hipError_t launch_cg_update1<double>(const CgDesc<double> &, int, hipStream_t);
template hipError_t launch_cg_update1<float>(const CgDesc<float> &, int, hipStream_t);
template hipError_t launch_cg_matvec<double>(const CgDesc<double> *, const BlockEntry *, int, int,
                                             hipStream_t, hipEvent_t, hipEvent_t);
template hipError_t launch_cg_matvec<float>(const CgDesc<float> *, const BlockEntry *, int, int,
                                            hipStream_t, hipEvent_t, hipEvent_t);
template hipError_t launch_cg_update<double>(const CgDesc<double> *, const BlockEntry *, int, int,
                                             hipStream_t);
template hipError_t launch_cg_update<float>(const CgDesc<float> *, const BlockEntry *, int, int,
                                            hipStream_t);

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
