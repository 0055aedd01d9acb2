// Relaxed shape derivative (Sec. 2.2.5, Eqs. 15-18) and Hilbertian
// extension-regularisation (Sec. 2.2.6, Eqs. 19-20) on the voxel grid.
//
// Nodal shape-derivative vector: with trilinear phi and u on each voxel and
// a 2x2x2 Gauss rule,
//   g_a = sum_e sum_q w_q h^3 N_a(q) (c_s s(q) + c_0) H'_eta(phi(q)) |grad phi(q)|,
//   s = sigma:eps = lambda (tr eps)^2 + 2 mu eps:eps with the solid's E0,
//   H'_eta(t) = (1 + cos(pi t / eta)) / (2 eta) for |t| <= eta, else 0.
// Two passes: each element whose nodal phi range meets [-eta, eta] (the band)
// evaluates its Gauss-point factors once and stores its eight nodal
// contributions; then every node sums those of its (up to 8) band elements in
// a fixed order, so the vector is the same run to run.
//
// Extension: A_H = ell^2 K + M (Q1 Laplacian and mass).  On equal voxels both
// are sums of Kronecker products of the 1D assembled stiffness
// (1/h)[-1 2 -1] and mass (h/6)[1 4 1] (halved at the two end nodes), so the
// product is a 27-point stencil whose coefficients are products of 1D
// entries.  Nodes of Gamma_N (the loaded nodes) are identity rows.  It is
// solved by Jacobi-preconditioned CG in float64; every kernel sums the
// previous kernel's per-block partials itself, in one fixed order.
#include <algorithm>

#include "common.h"
#include "device_common.h"

namespace topo {

constexpr double GA = 0.21132486540518711775;  // (1 - 1/sqrt(3)) / 2
constexpr double GB = 0.78867513459481288225;  // (1 + 1/sqrt(3)) / 2

__device__ __forceinline__ double hprime(double t, double eta) {
  return fabs(t) <= eta ? (1.0 + cos(M_PI * t / eta)) / (2.0 * eta) : 0.0;
}

// Gauss factors F(q) = w_q h^3 (c_s s + c_0) H' |grad phi| of element
// (ei, ej, ek); returns false when no Gauss point lies in the band.
__device__ bool shape_elem_factors(int ei, int ej, int ek, int NX, int NY,
                                   const double *__restrict__ u, const double *__restrict__ phi,
                                   double h, double lam, double mu, double eta, double c_s,
                                   double c_0, double F[8]) {
  const size_t n0 = (size_t)ei + (size_t)NX * ((size_t)ej + (size_t)NY * ek);
  size_t nd[8];
  double ph[8];
  for (int a = 0; a < 8; ++a) {
    nd[a] = n0 + (size_t)(a & 1) + (size_t)NX * ((size_t)((a >> 1) & 1) + (size_t)NY * (a >> 2));
    ph[a] = phi[nd[a]];
  }
  // quick reject: phi is trilinear, so it lies between its nodal extremes
  double lo = ph[0], hi = ph[0];
  for (int a = 1; a < 8; ++a) {
    lo = fmin(lo, ph[a]);
    hi = fmax(hi, ph[a]);
  }
  if (lo > eta || hi < -eta) return false;
  double ue[8][3];
  if (c_s != 0.0)
    for (int a = 0; a < 8; ++a)
      for (int c = 0; c < 3; ++c) ue[a][c] = u[3 * nd[a] + c];
  const double w = 0.125 * h * h * h, ih = 1.0 / h;
  bool any = false;
  for (int q = 0; q < 8; ++q) {
    const double r[3] = {(q & 1) ? GB : GA, ((q >> 1) & 1) ? GB : GA, (q >> 2) ? GB : GA};
    double p = 0.0, gp[3] = {0.0, 0.0, 0.0};
    double gu[3][3] = {{0.0, 0.0, 0.0}, {0.0, 0.0, 0.0}, {0.0, 0.0, 0.0}};
    for (int a = 0; a < 8; ++a) {
      const int bx = a & 1, by = (a >> 1) & 1, bz = a >> 2;
      const double fx = bx ? r[0] : 1.0 - r[0], fy = by ? r[1] : 1.0 - r[1],
                   fz = bz ? r[2] : 1.0 - r[2];
      const double dx = (bx ? 1.0 : -1.0) * fy * fz * ih, dy = fx * (by ? 1.0 : -1.0) * fz * ih,
                   dz = fx * fy * (bz ? 1.0 : -1.0) * ih;
      p += fx * fy * fz * ph[a];
      gp[0] += dx * ph[a];
      gp[1] += dy * ph[a];
      gp[2] += dz * ph[a];
      if (c_s != 0.0)
        for (int c = 0; c < 3; ++c) {
          gu[c][0] += ue[a][c] * dx;
          gu[c][1] += ue[a][c] * dy;
          gu[c][2] += ue[a][c] * dz;
        }
    }
    const double hp = hprime(p, eta);
    if (hp == 0.0) {
      F[q] = 0.0;
      continue;
    }
    any = true;
    double dens = c_0;
    if (c_s != 0.0) {
      const double tr = gu[0][0] + gu[1][1] + gu[2][2];
      double ee = 0.0;
      for (int i = 0; i < 3; ++i)
        for (int j = 0; j < 3; ++j) {
          const double e = 0.5 * (gu[i][j] + gu[j][i]);
          ee += e * e;
        }
      dens = c_s * (lam * tr * tr + 2.0 * mu * ee) + c_0;
    }
    F[q] = w * dens * hp * sqrt(gp[0] * gp[0] + gp[1] * gp[1] + gp[2] * gp[2]);
  }
  return any;
}

// Node and element indices: grids hold fewer than 2^31 nodes, so 32-bit
// unsigned division recovers (i, j, k) (64-bit division is a long sequence).
__device__ __forceinline__ void split3(unsigned n, unsigned NX, unsigned NY, int &i, int &j,
                                       int &k) {
  const unsigned r = n / NX;
  i = (int)(n - r * NX);
  k = (int)(r / NY);
  j = (int)(r - (unsigned)k * NY);
}

// Element pass.  A block owns SH_RANGE consecutive elements (grid-stride over
// such ranges).  Its lanes first test their elements: band[e] = 1 when phi's
// nodal range on e meets [-eta, eta] (phi is trilinear, so it lies between
// its nodal extremes), and the band elements are appended to a list in LDS.
// The lanes then take the list densely, so a wave evaluates 64 band elements
// at once however thinly the band crosses the range.  Element e stores
// c_a = sum_q N_a(q) F(q) at contrib[a * nel + e], a = 0..7; the list order
// decides only which lane computes what.
constexpr int SH_THREADS = 256, SH_RANGE = 2048;

__global__ __launch_bounds__(SH_THREADS) void k_shape_elem(
    int nelx, int nely, int nelz, const double *__restrict__ u, const double *__restrict__ phi,
    double h, double lam, double mu, double eta, double c_s, double c_0,
    uint8_t *__restrict__ band, double *__restrict__ contrib) {
  __shared__ unsigned list[SH_RANGE];
  __shared__ unsigned count;
  const unsigned nel = (unsigned)nelx * nely * nelz;
  const int NX = nelx + 1, NY = nely + 1;
  for (unsigned base = blockIdx.x * (unsigned)SH_RANGE; base < nel;
       base += gridDim.x * (unsigned)SH_RANGE) {
    if (threadIdx.x == 0) count = 0;
    __syncthreads();
    // every lane loads the nodal phi of all its elements before testing any
    constexpr int PER = SH_RANGE / SH_THREADS;
    double lo[PER], hi[PER];
#pragma unroll
    for (int r = 0; r < PER; ++r) {
      const unsigned e = base + threadIdx.x + (unsigned)r * SH_THREADS;
      lo[r] = INFINITY;
      hi[r] = -INFINITY;
      if (e < nel) {
        int i, j, k;
        split3(e, nelx, nely, i, j, k);
        const size_t n0 = (size_t)i + (size_t)NX * ((size_t)j + (size_t)NY * k);
#pragma unroll
        for (int a = 0; a < 8; ++a) {
          const double v = phi[n0 + (size_t)(a & 1) +
                               (size_t)NX * ((size_t)((a >> 1) & 1) + (size_t)NY * (a >> 2))];
          lo[r] = fmin(lo[r], v);
          hi[r] = fmax(hi[r], v);
        }
      }
    }
#pragma unroll
    for (int r = 0; r < PER; ++r) {
      const unsigned e = base + threadIdx.x + (unsigned)r * SH_THREADS;
      if (e < nel) {
        const bool in = !(lo[r] > eta || hi[r] < -eta);
        band[e] = in ? 1 : 0;
        if (in) list[atomicAdd(&count, 1u)] = e;
      }
    }
    __syncthreads();
    const unsigned m = count;
    for (unsigned q = threadIdx.x; q < m; q += SH_THREADS) {
      const unsigned e = list[q];
      int i, j, k;
      split3(e, nelx, nely, i, j, k);
      double F[8];
      for (int r = 0; r < 8; ++r) F[r] = 0.0;
      shape_elem_factors(i, j, k, NX, NY, u, phi, h, lam, mu, eta, c_s, c_0, F);
      for (int a = 0; a < 8; ++a) {
        const int bx = a & 1, by = (a >> 1) & 1, bz = a >> 2;
        double c = 0.0;
        for (int r = 0; r < 8; ++r) {
          const double x = (r & 1) ? GB : GA, y = ((r >> 1) & 1) ? GB : GA, z = (r >> 2) ? GB : GA;
          c += (bx ? x : 1.0 - x) * (by ? y : 1.0 - y) * (bz ? z : 1.0 - z) * F[r];
        }
        contrib[(size_t)a * nel + e] = c;
      }
    }
    __syncthreads();
  }
}

// Node pass: g_n = sum over its elements in the order a = 0..7 (the node is
// local node a of element (i - ax, j - ay, k - az)) of their stored
// contributions; elements outside the band add nothing.
__global__ __launch_bounds__(256) void k_shape_gather(int nelx, int nely, int nelz,
                                                      const uint8_t *__restrict__ band,
                                                      const double *__restrict__ contrib,
                                                      double *__restrict__ g) {
  const int NX = nelx + 1, NY = nely + 1;
  const unsigned nn = (unsigned)NX * NY * (nelz + 1);
  const size_t nel = (size_t)nelx * nely * nelz;
  for (unsigned n = blockIdx.x * blockDim.x + threadIdx.x; n < nn; n += gridDim.x * blockDim.x) {
    int i, j, k;
    split3(n, NX, NY, i, j, k);
    // the eight band bytes first, then the stored contributions of the band
    // elements, then the sum in the order a = 0..7
    size_t e[8];
    bool in[8];
#pragma unroll
    for (int a = 0; a < 8; ++a) {
      const int ei = i - (a & 1), ej = j - ((a >> 1) & 1), ek = k - (a >> 2);
      const bool ok = ei >= 0 && ej >= 0 && ek >= 0 && ei < nelx && ej < nely && ek < nelz;
      e[a] = ok ? (size_t)ei + (size_t)nelx * ((size_t)ej + (size_t)nely * ek) : 0;
      in[a] = ok && band[e[a]] != 0;
    }
    double c[8];
#pragma unroll
    for (int a = 0; a < 8; ++a) c[a] = in[a] ? contrib[(size_t)a * nel + e[a]] : 0.0;
    double sum = 0.0;
#pragma unroll
    for (int a = 0; a < 8; ++a)
      if (in[a]) sum += c[a];
    g[n] = sum;
  }
}

hipError_t launch_shape_rhs(const Grid &g, const double *u, const double *phi, double h,
                            double lam, double mu, double eta, double c_s, double c_0,
                            uint8_t *band, double *contrib, double *out, hipStream_t s) {
  size_t b = (g.nel + SH_RANGE - 1) / SH_RANGE;
  if (b > 65535) b = 65535;
  hipLaunchKernelGGL(k_shape_elem, dim3((unsigned)b), dim3(SH_THREADS), 0, s, g.nelx, g.nely,
                     g.nelz, u, phi, h, lam, mu, eta, c_s, c_0, band, contrib);
  b = (g.nn + 255) / 256;
  if (b > 8192) b = 8192;
  hipLaunchKernelGGL(k_shape_gather, dim3((unsigned)b), dim3(256), 0, s, g.nelx, g.nely, g.nelz,
                     band, contrib, out);
  return hipGetLastError();
}

// ---------------------------------------------------------------- extension
// 1D assembled stiffness and mass entries (neighbour -1, self, +1) at node i
// of 0 .. N - 1; an end node has one element.  ih = 1/h, h6 = h/6 and
// h3 = h/3 come from the host, so an entry costs a multiplication.
struct Tri {
  double k[3], m[3];
};
__device__ __forceinline__ Tri tri1d(int i, int N, double ih, double h6, double h3) {
  const double lo = i > 0 ? 1.0 : 0.0, hi = i < N - 1 ? 1.0 : 0.0;
  Tri t;
  t.k[0] = -lo * ih;
  t.k[1] = (lo + hi) * ih;
  t.k[2] = -hi * ih;
  t.m[0] = lo * h6;
  t.m[1] = (lo + hi) * h3;
  t.m[2] = hi * h6;
  return t;
}

__device__ __forceinline__ double helm_diag(const Tri &x, const Tri &y, const Tri &z,
                                            double ell2) {
  return ell2 * (x.k[1] * y.m[1] * z.m[1] + x.m[1] * y.k[1] * z.m[1] + x.m[1] * y.m[1] * z.k[1]) +
         x.m[1] * y.m[1] * z.m[1];
}

// Gamma_N: nodes with a non-zero load component (f interleaved 3n + c)
__global__ void k_gamma_mask(size_t nn, const double *__restrict__ f, uint8_t *__restrict__ gm) {
  for (size_t n = blockIdx.x * (size_t)blockDim.x + threadIdx.x; n < nn;
       n += (size_t)gridDim.x * blockDim.x)
    gm[n] = (f[3 * n] != 0.0 || f[3 * n + 1] != 0.0 || f[3 * n + 2] != 0.0) ? 1 : 0;
}

struct HcgArgs {
  int NX, NY, NZ;
  double h, ell2;
  double ih, h6, h3;  // 1/h, h/6, h/3
  int max_iters;
  const uint8_t *gm;
  double *x, *r, *z, *p, *q;
  // block partials: [0, HCG_PQ_MAX) p^T q of the apply; from HCG_PQ_MAX,
  // HCG_MAXB each: [par] r^T z and [2 + par] r^T r of the update of
  // iteration parity par (the start counts as parity 1)
  double *part;
  double *scal;  // [0] stop threshold on r^T r, [1] last r^T r, [2] iterations, [3] b^T b
  int *flags;    // [0] 0 running, 1 converged, 2 iteration cap, 3 breakdown
  int nb;        // blocks of the streaming kernels
  int nb_pq;     // blocks of the apply
  int kz, ntile; // planes per tile and tiles of the apply
};
__device__ __forceinline__ Tri tri_x(const HcgArgs &A, int i) {
  return tri1d(i, A.NX, A.ih, A.h6, A.h3);
}
__device__ __forceinline__ Tri tri_y(const HcgArgs &A, int j) {
  return tri1d(j, A.NY, A.ih, A.h6, A.h3);
}
__device__ __forceinline__ Tri tri_z(const HcgArgs &A, int k) {
  return tri1d(k, A.NZ, A.ih, A.h6, A.h3);
}
// the diagonal of A_H at node (i, j, k)
__device__ __forceinline__ double node_diag(const HcgArgs &A, int i, int j, int k) {
  return helm_diag(tri_x(A, i), tri_y(A, j), tri_z(A, k), A.ell2);
}
__device__ __forceinline__ double *rz_part(const HcgArgs &A, int par) {
  return A.part + HCG_PQ_MAX + par * HCG_MAXB;
}
__device__ __forceinline__ double *rr_part(const HcgArgs &A, int par) {
  return A.part + HCG_PQ_MAX + (2 + par) * HCG_MAXB;
}

__device__ double block_total(const double *__restrict__ part, int nb, double *sh) {
  __shared__ double tot;
  double v = 0.0;
  for (int i = threadIdx.x; i < nb; i += blockDim.x) v += part[i];
  const double t = block_sum_d(v, sh);
  if (threadIdx.x == 0) tot = t;
  __syncthreads();
  return tot;
}

__device__ __forceinline__ void node_ijk(size_t n, int NX, int NY, int &i, int &j, int &k) {
  split3((unsigned)n, (unsigned)NX, (unsigned)NY, i, j, k);
}

// x = 0, r = b on free nodes, z = r / diag, p = z; partials of parity 1
__global__ __launch_bounds__(256) void k_hcg_init(HcgArgs A, const double *__restrict__ b) {
  __shared__ double sh[4];
  const size_t nn = (size_t)A.NX * A.NY * A.NZ;
  double rz = 0.0, rr = 0.0;
  for (size_t n = blockIdx.x * (size_t)blockDim.x + threadIdx.x; n < nn;
       n += (size_t)gridDim.x * blockDim.x) {
    int i, j, k;
    node_ijk(n, A.NX, A.NY, i, j, k);
    const double bn = A.gm[n] ? 0.0 : b[n];
    const double d = node_diag(A, i, j, k);
    const double zn = bn / d;
    A.x[n] = 0.0;
    A.r[n] = bn;
    A.z[n] = zn;
    A.p[n] = zn;
    rz += bn * zn;
    rr += bn * bn;
  }
  const double a = block_sum_d(rz, sh);
  __syncthreads();
  const double c = block_sum_d(rr, sh);
  if (threadIdx.x == 0) {
    rz_part(A, 1)[blockIdx.x] = a;
    rr_part(A, 1)[blockIdx.x] = c;
  }
}

__global__ __launch_bounds__(256) void k_hcg_init_finish(HcgArgs A, double tol2_rel) {
  __shared__ double sh[4];
  const double rr = block_total(rr_part(A, 1), A.nb, sh);
  if (threadIdx.x == 0) {
    A.scal[0] = tol2_rel * rr;
    A.scal[1] = rr;
    A.scal[2] = 0.0;
    A.scal[3] = rr;
    A.flags[0] = rr == 0.0 ? 1 : 0;
  }
}

// q = A_H p (masked), partials p^T q.  A_H groups by its z factor as
//   Mz (ell^2 (Kx My + Mx Ky) + Mx My) + ell^2 Kz (Mx My),
// so each plane k' contributes two 9-point plane sums at (i, j):
//   P1 = sum_dj [ell^2 my sum_di kx p + (ell^2 ky + my) sum_di mx p],
//   P2 = sum_dj my sum_di mx p,
// and q = sum_dk mz P1(k + dk) + ell^2 kz P2(k + dk).  A thread walks a z
// column keeping P1, P2 of three planes in registers: 9 loads per node.
// A tile is a run of HB consecutive nodes of one plane (row-major, so it may
// wrap from one y row to the next) by kz planes: every lane holds a node
// whatever NX is.  The tiles are ordered run, then z-chunk, and mapped by
// xcd_local.
constexpr int HB = 256;

// the 3 x 3 neighbourhood of node n in its plane.  A neighbour beyond a face
// is read as the node itself (ox, oy: the clamped offsets); its 1D
// coefficients are 0, and p is finite, so it adds exact zeros.  The loads
// and sums are then straight-line code.
struct Off {
  ptrdiff_t lo, hi;
};
__device__ __forceinline__ void plane_load(const double *__restrict__ p, size_t n, const Off &ox,
                                           const Off &oy, double (&v)[9]) {
  const ptrdiff_t dx[3] = {ox.lo, 0, ox.hi}, dy[3] = {oy.lo, 0, oy.hi};
#pragma unroll
  for (int a = 0; a < 3; ++a)
#pragma unroll
    for (int c = 0; c < 3; ++c) v[3 * a + c] = p[(ptrdiff_t)n + dy[a] + dx[c]];
}

__device__ __forceinline__ void plane_sums(const double (&v)[9], const Tri &tx, const Tri &ty,
                                           double ell2, double &P1, double &P2) {
  P1 = 0.0;
  P2 = 0.0;
#pragma unroll
  for (int a = 0; a < 3; ++a) {
    double sk = 0.0, sm = 0.0;
#pragma unroll
    for (int c = 0; c < 3; ++c) {
      const double x = v[3 * a + c];
      sk += tx.k[c] * x;
      sm += tx.m[c] * x;
    }
    P1 += ell2 * ty.m[a] * sk + (ell2 * ty.k[a] + ty.m[a]) * sm;
    P2 += ty.m[a] * sm;
  }
}

__global__ __launch_bounds__(HB, 4) void k_hcg_apply(HcgArgs A) {
  if (A.flags[0]) return;
  __shared__ double sh[HB / 64];
  const int plane = A.NX * A.NY;
  const int nseg = (plane + HB - 1) / HB;
  const int t = threadIdx.x;
  double pq = 0.0;
  for (int b = blockIdx.x; b < A.ntile; b += gridDim.x) {
    const int lb = xcd_local(b, A.ntile);
    const int pp = (lb % nseg) * HB + t, tz_ = lb / nseg;
    const int j = pp / A.NX, i = pp - j * A.NX;
    const int k0 = tz_ * A.kz, k1 = min(k0 + A.kz, A.NZ);
    if (pp < plane) {
      const size_t sy = (size_t)A.NX, sz = (size_t)A.NX * A.NY;
      const Tri tx = tri_x(A, i), ty = tri_y(A, j);
      const Off ox = {i > 0 ? -1 : 0, i < A.NX - 1 ? 1 : 0};
      const Off oy = {j > 0 ? -(ptrdiff_t)sy : 0, j < A.NY - 1 ? (ptrdiff_t)sy : 0};
      size_t n = (size_t)i + sy * ((size_t)j + (size_t)A.NY * k0);
      double m1 = 0.0, m2 = 0.0, c1, c2, n1 = 0.0, n2 = 0.0;
      double va[9], vb[9], vc[9];
      if (k0 > 0) {
        plane_load(A.p, n - sz, ox, oy, va);
        plane_sums(va, tx, ty, A.ell2, m1, m2);
      }
      plane_load(A.p, n, ox, oy, va);
      plane_sums(va, tx, ty, A.ell2, c1, c2);
      // the neighbourhoods of planes k + 1 and k + 2 are loaded ahead
      if (k0 + 1 < A.NZ) plane_load(A.p, n + sz, ox, oy, vb);
      if (k0 + 2 < A.NZ && k0 + 1 < k1) plane_load(A.p, n + 2 * sz, ox, oy, vc);
      for (int k = k0; k < k1; ++k, n += sz) {
        if (k + 1 < A.NZ) {
          for (int q = 0; q < 9; ++q) {
            va[q] = vb[q];
            vb[q] = vc[q];
          }
          if (k + 3 < A.NZ && k + 2 < k1) plane_load(A.p, n + 3 * sz, ox, oy, vc);
          plane_sums(va, tx, ty, A.ell2, n1, n2);
        } else {
          n1 = 0.0;
          n2 = 0.0;
        }
        const Tri tz = tri_z(A, k);
        const double pn = A.p[n];
        const double acc = A.gm[n] ? pn
                                   : tz.m[0] * m1 + tz.m[1] * c1 + tz.m[2] * n1 +
                                         A.ell2 * (tz.k[0] * m2 + tz.k[1] * c2 + tz.k[2] * n2);
        A.q[n] = acc;
        pq += pn * acc;
        m1 = c1;
        m2 = c2;
        c1 = n1;
        c2 = n2;
      }
    }
  }
  // block sum (fixed order) of p^T q
  double v = wave_sum_d(pq);
  if ((t & 63) == 0) sh[t >> 6] = v;
  __syncthreads();
  if (t == 0) {
    double s = 0.0;
    for (int w = 0; w < HB / 64; ++w) s += sh[w];
    A.part[blockIdx.x] = s;
  }
}

// iteration it: alpha = r^T z / p^T q; x += alpha p, r -= alpha q,
// z = r / diag; partials of parity it & 1
__global__ __launch_bounds__(256) void k_hcg_update(HcgArgs A, int it) {
  if (A.flags[0]) return;
  __shared__ double sh[4];
  const int cur = it & 1, old = cur ^ 1;
  const double pq = block_total(A.part, A.nb_pq, sh);
  __syncthreads();
  const double rz = block_total(rz_part(A, old), A.nb, sh);
  if (!(pq > 0.0)) {  // breakdown: every block sees the same pq
    if (blockIdx.x == 0 && threadIdx.x == 0) {
      A.flags[0] = 3;
      A.scal[2] = (double)it;
    }
    return;
  }
  const double alpha = rz / pq;
  const size_t nn = (size_t)A.NX * A.NY * A.NZ;
  double rzn = 0.0, rr = 0.0;
  for (size_t n = blockIdx.x * (size_t)blockDim.x + threadIdx.x; n < nn;
       n += (size_t)gridDim.x * blockDim.x) {
    int i, j, k;
    node_ijk(n, A.NX, A.NY, i, j, k);
    const double d = node_diag(A, i, j, k);
    A.x[n] += alpha * A.p[n];
    const double rn = A.gm[n] ? 0.0 : A.r[n] - alpha * A.q[n];
    const double zn = rn / d;
    A.r[n] = rn;
    A.z[n] = zn;
    rzn += rn * zn;
    rr += rn * rn;
  }
  const double a = block_sum_d(rzn, sh);
  __syncthreads();
  const double c = block_sum_d(rr, sh);
  if (threadIdx.x == 0) {
    rz_part(A, cur)[blockIdx.x] = a;
    rr_part(A, cur)[blockIdx.x] = c;
  }
}

// iteration it: stop test on r^T r, else beta = r^T z (it) / r^T z (it - 1)
// and p = z + beta p.  Every block takes the same decision; block 0 records
// it.
__global__ __launch_bounds__(256) void k_hcg_dir(HcgArgs A, int it) {
  if (A.flags[0]) return;
  __shared__ double sh[4];
  const int cur = it & 1, old = cur ^ 1;
  const double rzn = block_total(rz_part(A, cur), A.nb, sh);
  __syncthreads();
  const double rzo = block_total(rz_part(A, old), A.nb, sh);
  __syncthreads();
  const double rr = block_total(rr_part(A, cur), A.nb, sh);
  const bool conv = rr <= A.scal[0];
  const bool capped = !conv && it + 1 >= A.max_iters;
  if (conv || capped) {
    if (blockIdx.x == 0 && threadIdx.x == 0) {
      A.scal[1] = rr;
      A.scal[2] = (double)(it + 1);
      A.flags[0] = conv ? 1 : 2;
    }
    return;
  }
  if (blockIdx.x == 0 && threadIdx.x == 0) {  // progress, for the host's choice of chunk
    A.scal[1] = rr;
    A.scal[2] = (double)(it + 1);
  }
  const double beta = rzn / rzo;
  const size_t nn = (size_t)A.NX * A.NY * A.NZ;
  for (size_t n = blockIdx.x * (size_t)blockDim.x + threadIdx.x; n < nn;
       n += (size_t)gridDim.x * blockDim.x)
    A.p[n] = A.z[n] + beta * A.p[n];
}

hipError_t launch_hilbert(const Grid &g, double h, double ell, double rtol, int max_iters,
                          const double *f, const double *b, double *x, double *const vec[4],
                          uint8_t *gm, double *part, double *scal, int *flags, int it0, int count,
                          hipStream_t s) {
  HcgArgs A;
  A.NX = g.nelx + 1;
  A.NY = g.nely + 1;
  A.NZ = g.nelz + 1;
  A.h = h;
  A.ell2 = ell * ell;
  A.ih = 1.0 / h;
  A.h6 = h / 6.0;
  A.h3 = h / 3.0;
  A.max_iters = max_iters;
  A.gm = gm;
  A.x = x;
  A.r = vec[0];
  A.z = vec[1];
  A.p = vec[2];
  A.q = vec[3];
  A.part = part;
  A.scal = scal;
  A.flags = flags;
  // the apply runs over tiles of up to 16 planes (about 2048 of them where
  // the grid allows), at most HCG_PQ_MAX blocks that loop over the tiles; the
  // streaming kernels over at most HCG_MAXB blocks
  const long nseg = ((long)A.NX * A.NY + HB - 1) / HB;
  A.kz = (int)std::max(1L, std::min(16L, (long)A.NZ * nseg / 2048));
  A.ntile = (int)(nseg * ((A.NZ + A.kz - 1) / A.kz));
  A.nb_pq = std::min(A.ntile, HCG_PQ_MAX);
  size_t nb = (g.nn + 1023) / 1024;
  if (nb > (size_t)HCG_MAXB) nb = HCG_MAXB;
  if (nb < 1) nb = 1;
  A.nb = (int)nb;
  const dim3 grid((unsigned)nb), blk(256);
  if (it0 == 0) {
    size_t b1 = (g.nn + 255) / 256;
    if (b1 > 4096) b1 = 4096;
    hipLaunchKernelGGL(k_gamma_mask, dim3((unsigned)b1), dim3(256), 0, s, g.nn, f, gm);
    hipLaunchKernelGGL(k_hcg_init, grid, blk, 0, s, A, b);
    hipLaunchKernelGGL(k_hcg_init_finish, dim3(1), blk, 0, s, A, rtol * rtol);
  }
  for (int it = it0; it < it0 + count; ++it) {
    hipLaunchKernelGGL(k_hcg_apply, dim3((unsigned)A.nb_pq), dim3(HB), 0, s, A);
    hipLaunchKernelGGL(k_hcg_update, grid, blk, 0, s, A, it);
    hipLaunchKernelGGL(k_hcg_dir, grid, blk, 0, s, A, it);
  }
  return hipGetLastError();
}

}  // namespace topo
