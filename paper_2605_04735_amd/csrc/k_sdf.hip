// Density -> signed distance transfer on the voxel grid (paper Secs. 3.2-3.4,
// Eqs. 25-30) and the ersatz volume fraction.
//
//  node_mean  nodal density = mean of the adjacent elements (what the paper's
//             local LSQ map with its fallbacks gives on voxels), summed in
//             increasing element order, then times 1/m (m in {1,2,4,8}: exact)
//  mt_count   per voxel, triangles of marching tetrahedra on the six-tet Kuhn
//             split (tet p: corners 0, e_p0, e_p0 + e_p1, (1,1,1) for the axis
//             permutations p in lexicographic order); a node is inside when
//             rho >= rho_t
//  scan       exclusive prefix sum of the counts (triangle offsets)
//  mt_emit    triangle vertices, each voxel's triangles stored contiguously
//  udist      per node, the exact minimum distance to the triangles (Eq. 29):
//             every triangle lies in the voxel that produced it, so voxels
//             (and 4^3 coarse cells of them) can be skipped whenever their
//             box is farther than the best distance found so far; the search
//             grows outwards and stops when nothing unvisited can be closer
//  sign       Eq. 30: phi = -d if rho >= rho_t else +d
//  vf         per voxel, the volume fraction of {phi_lin < 0} over the same
//             six tets, in closed form from the edge crossing fractions
#include <climits>
#include <cstdlib>
#include <algorithm>

#include "common.h"

namespace topo {

#pragma clang fp contract(off)

// Kuhn tets as local corner numbers a = ax + 2 ay + 4 az
__constant__ int c_kuhn[6][4] = {
    {0, 1, 3, 7},  // (x, y, z)
    {0, 1, 5, 7},  // (x, z, y)
    {0, 2, 3, 7},  // (y, x, z)
    {0, 2, 6, 7},  // (y, z, x)
    {0, 4, 5, 7},  // (z, x, y)
    {0, 4, 6, 7},  // (z, y, x)
};

__device__ __forceinline__ size_t nidx(int NX, int NY, int i, int j, int k) {
  return (size_t)i + (size_t)NX * ((size_t)j + (size_t)NY * k);
}

__global__ void k_node_mean(int nelx, int nely, int nelz, const double *__restrict__ x,
                            double *__restrict__ rho) {
  const int NX = nelx + 1, NY = nely + 1, NZ = nelz + 1;
  const size_t nn = (size_t)NX * NY * NZ;
  for (size_t n = blockIdx.x * (size_t)blockDim.x + threadIdx.x; n < nn;
       n += (size_t)gridDim.x * blockDim.x) {
    const int i = (int)(n % NX), j = (int)((n / NX) % NY), k = (int)(n / ((size_t)NX * NY));
    double s = 0.0;
    int m = 0;
    for (int bz = 0; bz < 2; ++bz)
      for (int by = 0; by < 2; ++by)
        for (int bx = 0; bx < 2; ++bx) {
          const int ei = i - 1 + bx, ej = j - 1 + by, ek = k - 1 + bz;
          if (ei >= 0 && ei < nelx && ej >= 0 && ej < nely && ek >= 0 && ek < nelz) {
            s = s + x[(size_t)ei + (size_t)nelx * ((size_t)ej + (size_t)nely * ek)];
            ++m;
          }
        }
    rho[n] = s * (1.0 / (double)m);
  }
}

hipError_t launch_node_mean(const Grid &g, const double *x, double *rho, hipStream_t s) {
  int blocks = (int)((g.nn + 255) / 256);
  if (blocks > 8192) blocks = 8192;
  hipLaunchKernelGGL(k_node_mean, dim3(blocks), dim3(256), 0, s, g.nelx, g.nely, g.nelz, x, rho);
  return hipGetLastError();
}

__device__ __forceinline__ int tet_tris(int ninside) {
  return (ninside == 1 || ninside == 3) ? 1 : (ninside == 2 ? 2 : 0);
}

__global__ void k_mt_count(int nelx, int nely, int nelz, const double *__restrict__ rho,
                           double rho_t, int *__restrict__ count) {
  const int NX = nelx + 1, NY = nely + 1;
  const size_t nel = (size_t)nelx * nely * nelz;
  for (size_t e = blockIdx.x * (size_t)blockDim.x + threadIdx.x; e < nel;
       e += (size_t)gridDim.x * blockDim.x) {
    const int i = (int)(e % nelx), j = (int)((e / nelx) % nely), k = (int)(e / ((size_t)nelx * nely));
    unsigned in = 0;
    for (int a = 0; a < 8; ++a)
      if (rho[nidx(NX, NY, i + (a & 1), j + ((a >> 1) & 1), k + (a >> 2))] >= rho_t) in |= 1u << a;
    int c = 0;
    if (in != 0u && in != 0xFFu) {
      for (int t = 0; t < 6; ++t) {
        int ni = 0;
        for (int v = 0; v < 4; ++v) ni += (in >> c_kuhn[t][v]) & 1u;
        c += tet_tris(ni);
      }
    }
    count[e] = c;
  }
}

hipError_t launch_mt_count(const Grid &g, const double *rho, double rho_t, int *count,
                           hipStream_t s) {
  int blocks = (int)((g.nel + 255) / 256);
  if (blocks > 8192) blocks = 8192;
  hipLaunchKernelGGL(k_mt_count, dim3(blocks), dim3(256), 0, s, g.nelx, g.nely, g.nelz, rho, rho_t,
                     count);
  return hipGetLastError();
}

// ---------------------------------------------------------------- scan
constexpr int SCAN_THREADS = 256;
constexpr int SCAN_PER = 4;
constexpr int SCAN_TILE = SCAN_THREADS * SCAN_PER;

__device__ int block_exclusive_scan(int v, int *sh, int *total) {
  // Hillis-Steele on SCAN_THREADS values
  sh[threadIdx.x] = v;
  __syncthreads();
  for (int o = 1; o < SCAN_THREADS; o <<= 1) {
    const int t = (threadIdx.x >= (unsigned)o) ? sh[threadIdx.x - o] : 0;
    __syncthreads();
    sh[threadIdx.x] += t;
    __syncthreads();
  }
  const int incl = sh[threadIdx.x];
  *total = sh[SCAN_THREADS - 1];
  __syncthreads();
  return incl - v;
}

__global__ __launch_bounds__(SCAN_THREADS) void k_scan_tiles(const int *__restrict__ in,
                                                             int *__restrict__ out, size_t n,
                                                             int *__restrict__ tile_sums) {
  __shared__ int sh[SCAN_THREADS];
  const size_t base = (size_t)blockIdx.x * SCAN_TILE + (size_t)threadIdx.x * SCAN_PER;
  int v[SCAN_PER];
  int s = 0;
  for (int q = 0; q < SCAN_PER; ++q) {
    v[q] = (base + q < n) ? in[base + q] : 0;
    s += v[q];
  }
  int total;
  int ex = block_exclusive_scan(s, sh, &total);
  for (int q = 0; q < SCAN_PER; ++q) {
    if (base + q < n) out[base + q] = ex;
    ex += v[q];
  }
  if (threadIdx.x == 0) tile_sums[blockIdx.x] = total;
}

__global__ __launch_bounds__(SCAN_THREADS) void k_scan_sums(int *__restrict__ sums, int nt) {
  __shared__ int sh[SCAN_THREADS];
  int carry = 0;
  for (int base = 0; base < nt; base += SCAN_THREADS) {
    const int idx = base + threadIdx.x;
    const int v = (idx < nt) ? sums[idx] : 0;
    int total;
    const int ex = block_exclusive_scan(v, sh, &total);
    if (idx < nt) sums[idx] = carry + ex;
    carry += total;
    __syncthreads();
  }
  if (threadIdx.x == 0) sums[nt] = carry;
}

__global__ void k_scan_add(int *__restrict__ out, size_t n, const int *__restrict__ sums) {
  const size_t i = (size_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i < n) out[i] += sums[i / SCAN_TILE];
}

// out[0..n) exclusive scan of in; block_sums needs n/SCAN_TILE + 2 ints and
// receives the grand total at index ntiles.
hipError_t launch_scan(const int *in, int *out, size_t n, int *block_sums, hipStream_t s) {
  const int nt = (int)((n + SCAN_TILE - 1) / SCAN_TILE);
  hipLaunchKernelGGL(k_scan_tiles, dim3(nt), dim3(SCAN_THREADS), 0, s, in, out, n, block_sums);
  hipLaunchKernelGGL(k_scan_sums, dim3(1), dim3(SCAN_THREADS), 0, s, block_sums, nt);
  hipLaunchKernelGGL(k_scan_add, dim3((unsigned)((n + 255) / 256)), dim3(256), 0, s, out, n,
                     block_sums);
  return hipGetLastError();
}

// ---------------------------------------------------------------- emit
__device__ __forceinline__ void cut_point(const double pa[3], const double pb[3], double ra,
                                          double rb, double rho_t, double *o) {
  const double t = (rho_t - ra) / (rb - ra);
  o[0] = pa[0] + t * (pb[0] - pa[0]);
  o[1] = pa[1] + t * (pb[1] - pa[1]);
  o[2] = pa[2] + t * (pb[2] - pa[2]);
}

__global__ void k_mt_emit(int nelx, int nely, int nelz, const double *__restrict__ rho,
                          double rho_t, double h, const int *__restrict__ offset,
                          const int *__restrict__ count, double *__restrict__ tri) {
  const int NX = nelx + 1, NY = nely + 1;
  const size_t nel = (size_t)nelx * nely * nelz;
  for (size_t e = blockIdx.x * (size_t)blockDim.x + threadIdx.x; e < nel;
       e += (size_t)gridDim.x * blockDim.x) {
    if (count[e] == 0) continue;
    const int i = (int)(e % nelx), j = (int)((e / nelx) % nely), k = (int)(e / ((size_t)nelx * nely));
    double P[8][3], R[8];
    for (int a = 0; a < 8; ++a) {
      const int ii = i + (a & 1), jj = j + ((a >> 1) & 1), kk = k + (a >> 2);
      P[a][0] = (double)ii * h;
      P[a][1] = (double)jj * h;
      P[a][2] = (double)kk * h;
      R[a] = rho[nidx(NX, NY, ii, jj, kk)];
    }
    double *o = tri + 9 * (size_t)offset[e];
    for (int t = 0; t < 6; ++t) {
      int I[4], O[4], ni = 0, no = 0;
      for (int v = 0; v < 4; ++v) {
        const int c = c_kuhn[t][v];
        if (R[c] >= rho_t) I[ni++] = c;
        else O[no++] = c;
      }
      if (ni == 1) {
        for (int q = 0; q < 3; ++q) cut_point(P[I[0]], P[O[q]], R[I[0]], R[O[q]], rho_t, o + 3 * q);
        o += 9;
      } else if (ni == 3) {
        for (int q = 0; q < 3; ++q) cut_point(P[I[q]], P[O[0]], R[I[q]], R[O[0]], rho_t, o + 3 * q);
        o += 9;
      } else if (ni == 2) {
        double pac[3], pad[3], pbd[3], pbc[3];
        cut_point(P[I[0]], P[O[0]], R[I[0]], R[O[0]], rho_t, pac);
        cut_point(P[I[0]], P[O[1]], R[I[0]], R[O[1]], rho_t, pad);
        cut_point(P[I[1]], P[O[1]], R[I[1]], R[O[1]], rho_t, pbd);
        cut_point(P[I[1]], P[O[0]], R[I[1]], R[O[0]], rho_t, pbc);
        for (int q = 0; q < 3; ++q) {
          o[q] = pac[q];
          o[3 + q] = pad[q];
          o[6 + q] = pbd[q];
          o[9 + q] = pac[q];
          o[12 + q] = pbd[q];
          o[15 + q] = pbc[q];
        }
        o += 18;
      }
    }
  }
}

hipError_t launch_mt_emit(const Grid &g, const double *rho, double rho_t, double h,
                          const int *offset, const int *count, double *tri, hipStream_t s) {
  int blocks = (int)((g.nel + 255) / 256);
  if (blocks > 8192) blocks = 8192;
  hipLaunchKernelGGL(k_mt_emit, dim3(blocks), dim3(256), 0, s, g.nelx, g.nely, g.nelz, rho, rho_t,
                     h, offset, count, tri);
  return hipGetLastError();
}

// ---------------------------------------------------------------- distance
__device__ __forceinline__ double dot3(const double *a, const double *b) {
  return a[0] * b[0] + a[1] * b[1] + a[2] * b[2];
}

__device__ double seg_dist2(const double *p, const double *a, const double *b) {
  double ab[3] = {b[0] - a[0], b[1] - a[1], b[2] - a[2]};
  double ap[3] = {p[0] - a[0], p[1] - a[1], p[2] - a[2]};
  const double L = dot3(ab, ab);
  double t = (L > 0.0) ? dot3(ap, ab) / L : 0.0;
  t = fmin(1.0, fmax(0.0, t));
  double d[3] = {ap[0] - t * ab[0], ap[1] - t * ab[1], ap[2] - t * ab[2]};
  return dot3(d, d);
}

// Squared distance from p to triangle (a, b, c): the Voronoi-region case
// analysis named in the paper (vertex, edge and face regions from the signs of
// the projections of p - vertex on the edges); degenerate triangles (zero
// area) fall back to the nearest of the three edges.
__device__ double tri_dist2(const double *p, const double *a, const double *b, const double *c) {
  double ab[3] = {b[0] - a[0], b[1] - a[1], b[2] - a[2]};
  double ac[3] = {c[0] - a[0], c[1] - a[1], c[2] - a[2]};
  double ap[3] = {p[0] - a[0], p[1] - a[1], p[2] - a[2]};
  const double d1 = dot3(ab, ap), d2 = dot3(ac, ap);
  double q[3];
  if (d1 <= 0.0 && d2 <= 0.0) return dot3(ap, ap);  // vertex a
  double bp[3] = {p[0] - b[0], p[1] - b[1], p[2] - b[2]};
  const double d3 = dot3(ab, bp), d4 = dot3(ac, bp);
  if (d3 >= 0.0 && d4 <= d3) return dot3(bp, bp);  // vertex b
  const double vc = d1 * d4 - d3 * d2;
  if (vc <= 0.0 && d1 >= 0.0 && d3 <= 0.0) {  // edge ab
    const double v = d1 / (d1 - d3);
    for (int i = 0; i < 3; ++i) q[i] = ap[i] - v * ab[i];
    return dot3(q, q);
  }
  double cp[3] = {p[0] - c[0], p[1] - c[1], p[2] - c[2]};
  const double d5 = dot3(ab, cp), d6 = dot3(ac, cp);
  if (d6 >= 0.0 && d5 <= d6) return dot3(cp, cp);  // vertex c
  const double vb = d5 * d2 - d1 * d6;
  if (vb <= 0.0 && d2 >= 0.0 && d6 <= 0.0) {  // edge ac
    const double w = d2 / (d2 - d6);
    for (int i = 0; i < 3; ++i) q[i] = ap[i] - w * ac[i];
    return dot3(q, q);
  }
  const double va = d3 * d6 - d5 * d4;
  if (va <= 0.0 && (d4 - d3) >= 0.0 && (d5 - d6) >= 0.0) {  // edge bc
    const double w = (d4 - d3) / ((d4 - d3) + (d5 - d6));
    for (int i = 0; i < 3; ++i) q[i] = bp[i] - w * (c[i] - b[i]);
    return dot3(q, q);
  }
  const double den = va + vb + vc;
  if (!(den > 0.0)) {  // zero-area triangle
    return fmin(seg_dist2(p, a, b), fmin(seg_dist2(p, b, c), seg_dist2(p, c, a)));
  }
  const double v = vb / den, w = vc / den;  // face region
  for (int i = 0; i < 3; ++i) q[i] = ap[i] - v * ab[i] - w * ac[i];
  return dot3(q, q);
}

// Smallest squared distance from p to the c triangles stored from t on (9
// coordinates each).  When t is the same for the whole wave (UNIFORM), the
// triangles arrive as scalar loads, which complete in any order, so a test
// waits for every load in flight: they are taken two per round, both loads
// issued before the first test waits, so a pair costs one memory round trip.
// fmin is exact, so the order does not change the result.
template <bool UNIFORM>
__device__ __forceinline__ double voxel_dist2(const double *p, const double *t, int c) {
  double m = INFINITY;
  int q = 0;
  if constexpr (UNIFORM) {
    for (; q + 1 < c; q += 2, t += 18) {
      double a[18];
#pragma unroll
      for (int i = 0; i < 18; ++i) a[i] = t[i];
      // both triangles' values are needed here, so their loads issue together
      asm volatile("" ::"s"(a[0]), "s"(a[3]), "s"(a[6]), "s"(a[9]), "s"(a[12]), "s"(a[15]));
      m = fmin(m, fmin(tri_dist2(p, a, a + 3, a + 6), tri_dist2(p, a + 9, a + 12, a + 15)));
    }
  }
  for (; q < c; ++q, t += 9) m = fmin(m, tri_dist2(p, t, t + 3, t + 6));
  return m;
}

constexpr int CB = 4;  // coarse cell edge (voxels) of the occupancy grid

// occupancy of the CB^3 coarse cells as a bitmask: bit (c & 31) of word c / 32
// is 1 when any voxel of cell c has triangles.  One lane per cell; the wave's
// 64 bits (64-aligned cells) are written by lanes 0 and 1.
__global__ void k_occ(int nelx, int nely, int nelz, const int *__restrict__ count,
                      unsigned *__restrict__ occ) {
  const int cx = (nelx + CB - 1) / CB, cy = (nely + CB - 1) / CB, cz = (nelz + CB - 1) / CB;
  const size_t nc = (size_t)cx * cy * cz;
  const int lane = threadIdx.x & 63;
  const size_t stride = (size_t)gridDim.x * blockDim.x;
  for (size_t c0 = blockIdx.x * (size_t)blockDim.x + (threadIdx.x & ~63u); c0 < nc; c0 += stride) {
    const size_t c = c0 + lane;
    int any = 0;
    if (c < nc) {
      const int ci = (int)(c % cx), cj = (int)((c / cx) % cy), ck = (int)(c / ((size_t)cx * cy));
      for (int k = ck * CB; k < min((ck + 1) * CB, nelz) && !any; ++k)
        for (int j = cj * CB; j < min((cj + 1) * CB, nely) && !any; ++j)
          for (int i = ci * CB; i < min((ci + 1) * CB, nelx); ++i)
            if (count[(size_t)i + (size_t)nelx * ((size_t)j + (size_t)nely * k)]) {
              any = 1;
              break;
            }
    }
    const unsigned long long m = __ballot(any);
    const size_t w = c0 >> 5;
    if (lane == 0) occ[w] = (unsigned)m;
    if (lane == 1 && c0 + 32 < nc) occ[w + 1] = (unsigned)(m >> 32);
  }
}

// occupancy words held in LDS by the distance search (grids with more coarse
// cells read them from memory)
constexpr int OCC_LDS_WORDS = 4096;

__device__ __forceinline__ int axis_gap(int lo, int hi, int i) {  // voxels [lo, hi) vs node i
  return max(0, max(lo - i, i - hi));
}

__device__ __forceinline__ void scan_voxel(int vi, int vj, int vk, int nelx, int nely,
                                           const int *__restrict__ count,
                                           const int *__restrict__ offset,
                                           const double *__restrict__ tri, const double *p,
                                           double &best) {
  const size_t e = (size_t)vi + (size_t)nelx * ((size_t)vj + (size_t)nely * vk);
  const int c = count[e];
  if (c == 0) return;
  const double *t = tri + 9 * (size_t)offset[e];
  best = fmin(best, voxel_dist2<false>(p, t, c));
}

// whether the node (i, j, k) still needs voxel (vi, vj, vk) in phase 2: not
// stopped, not one of its phase-1 voxels, and the voxel's box is nearer than
// its best distance so far
__device__ __forceinline__ bool need_voxel(int vi, int vj, int vk, int i, int j, int k, double h,
                                           bool done, double best) {
  const int vx = axis_gap(vi, vi + 1, i), vy = axis_gap(vj, vj + 1, j), vz = axis_gap(vk, vk + 1, k);
  if (done || (vx <= 1 && vy <= 1 && vz <= 1)) return false;
  return ((double)vx * vx + (double)vy * vy + (double)vz * vz) * h * h < best;
}

// Exact Eq. 29 distance per node.  Phase 1 scans the voxels at Chebyshev gap
// 0 and 1 from the node (no point of a voxel at gap g is closer than g h, so
// a best distance <= 2 h is final).  Phase 2 scans rings of coarse cells
// around the node's cell, skipping empty cells and cells or voxels whose box
// is already farther than the best distance; after coarse ring R every
// unvisited cell lies beyond a face of the scanned box that the grid does not
// clip, so the distance to the nearest such face gives the stop rule.
//
// One 64-lane wave per CB^3 brick of nodes aligned with a coarse cell: the
// lanes share the ring centre, so phase 2 walks the rings and cells in step
// (a cell is entered when any unfinished lane may find a closer triangle in
// it) and a cell's 64 voxel counts and offsets arrive in one wave-wide load,
// one voxel per lane, read back voxel by voxel with readlane.  Each lane keeps
// its own best distance, its own voxel pruning and its own stop rule; the
// wave leaves the ring loop when every lane has stopped.
__global__ __launch_bounds__(128) void k_udist(
    int nelx, int nely, int nelz, double h, const int *__restrict__ count,
    const int *__restrict__ offset, const double *__restrict__ tri,
    const unsigned *__restrict__ occ, const double *__restrict__ rho, double rho_t,
    double *__restrict__ phi, int occ_lds_allowed) {
  const int NX = nelx + 1, NY = nely + 1, NZ = nelz + 1;
  const int cx = (nelx + CB - 1) / CB, cy = (nely + CB - 1) / CB, cz = (nelz + CB - 1) / CB;
  const int Rmax = max(cx, max(cy, cz));
  // the occupancy bitmask, staged in LDS when it fits
  __shared__ unsigned occ_lds[OCC_LDS_WORDS];
  const size_t nwords = ((size_t)cx * cy * cz + 31) / 32;
  const bool occ_in_lds = occ_lds_allowed && nwords <= (size_t)OCC_LDS_WORDS;
  if (occ_in_lds) {
    for (size_t w = threadIdx.x; w < nwords; w += blockDim.x) occ_lds[w] = occ[w];
    __syncthreads();
  }
  const int bx = (NX + CB - 1) / CB, by = (NY + CB - 1) / CB, bz = (NZ + CB - 1) / CB;
  const size_t nbr = (size_t)bx * by * bz;
  const int lane = threadIdx.x & 63;
  const int li = lane & 3, lj = (lane >> 2) & 3, lk = lane >> 4;
  // b is the same for the 64 lanes of a wave
  for (size_t b = (blockIdx.x * (size_t)blockDim.x + threadIdx.x) >> 6; b < nbr;
       b += ((size_t)gridDim.x * blockDim.x) >> 6) {
    const int ib = (int)(b % bx), jb = (int)((b / bx) % by), kb = (int)(b / ((size_t)bx * by));
    const int i = ib * CB + li, j = jb * CB + lj, k = kb * CB + lk;
    const bool valid = i < NX && j < NY && k < NZ;
    const double p[3] = {(double)i * h, (double)j * h, (double)k * h};
    double best = INFINITY;
    if (valid) {
      // phase 1: voxels i-2 .. i+1 (gaps 0 and 1) per axis
      for (int vk = max(k - 2, 0); vk <= min(k + 1, nelz - 1); ++vk)
        for (int vj = max(j - 2, 0); vj <= min(j + 1, nely - 1); ++vj)
          for (int vi = max(i - 2, 0); vi <= min(i + 1, nelx - 1); ++vi)
            scan_voxel(vi, vj, vk, nelx, nely, count, offset, tri, p, best);
    }
    bool done = !valid || best <= 4.0 * h * h;
    // the ring centre: the brick's own coarse cell (clamped for the nodes on
    // the grid's far faces), the same for every lane
    const int c0i = min(ib, cx - 1), c0j = min(jb, cy - 1), c0k = min(kb, cz - 1);
    for (int R = 0; R <= Rmax && __ballot(!done) != 0; ++R) {
      for (int ck = max(c0k - R, 0); ck <= min(c0k + R, cz - 1); ++ck) {
        const bool zs = (ck == c0k - R) || (ck == c0k + R);
        const int gz = axis_gap(ck * CB, min((ck + 1) * CB, nelz), k);
        for (int cj = max(c0j - R, 0); cj <= min(c0j + R, cy - 1); ++cj) {
          const bool ys = zs || (cj == c0j - R) || (cj == c0j + R);
          const int gy = axis_gap(cj * CB, min((cj + 1) * CB, nely), j);
          for (int ci = c0i - R; ci <= c0i + R; ci += (ys || ci == c0i + R) ? 1 : 2 * R) {
            if (ci < 0 || ci >= cx) continue;  // ring interior: only its two x faces
            const int gx = axis_gap(ci * CB, min((ci + 1) * CB, nelx), i);
            const double cd = ((double)gx * gx + (double)gy * gy + (double)gz * gz) * h * h;
            if (__ballot(!done && cd < best) == 0) continue;
            const size_t cell = (size_t)ci + (size_t)cx * ((size_t)cj + (size_t)cy * ck);
            const unsigned ow = occ_in_lds ? occ_lds[cell >> 5] : occ[cell >> 5];
            if (!((ow >> (cell & 31)) & 1u)) continue;
            // the cell's voxel counts and offsets, voxel (li, lj, lk) in lane
            const int ui = ci * CB + li, uj = cj * CB + lj, uk = ck * CB + lk;
            const bool uin = ui < nelx && uj < nely && uk < nelz;
            const size_t ue = uin ? (size_t)ui + (size_t)nelx * ((size_t)uj + (size_t)nely * uk) : 0;
            const int ucnt = uin ? count[ue] : 0;
            const int uoff = uin ? offset[ue] : 0;
            // only the cell's non-empty voxels (a wave-wide bit mask, lowest
            // first), and only those some unfinished lane may find closer
            unsigned long long live = __ballot(ucnt > 0);
            while (live) {
              const int v = __builtin_ctzll(live);  // the same for every lane
              live &= live - 1;
              const int c = __builtin_amdgcn_readlane(ucnt, v);
              const bool need = need_voxel(ci * CB + (v & 3), cj * CB + ((v >> 2) & 3),
                                           ck * CB + (v >> 4), i, j, k, h, done, best);
              if (__ballot(need) == 0) continue;
              if (need) {
                const double *t = tri + 9 * (size_t)__builtin_amdgcn_readlane(uoff, v);
                best = fmin(best, voxel_dist2<true>(p, t, c));
              }
            }
          }
        }
      }
      // unvisited voxels lie beyond a face of the scanned box that the grid
      // does not clip; the nearest such face bounds their distance
      int lim = INT_MAX;
      if (c0i - R > 0) lim = min(lim, i - (c0i - R) * CB);
      if (c0i + R < cx - 1) lim = min(lim, (c0i + R + 1) * CB - i);
      if (c0j - R > 0) lim = min(lim, j - (c0j - R) * CB);
      if (c0j + R < cy - 1) lim = min(lim, (c0j + R + 1) * CB - j);
      if (c0k - R > 0) lim = min(lim, k - (c0k - R) * CB);
      if (c0k + R < cz - 1) lim = min(lim, (c0k + R + 1) * CB - k);
      if (lim == INT_MAX || best <= (double)lim * lim * h * h) done = true;
    }
    if (valid) {
      const size_t n = (size_t)i + (size_t)NX * ((size_t)j + (size_t)NY * k);
      const double d = sqrt(best);
      phi[n] = (rho[n] >= rho_t) ? -d : d;
    }
  }
}

hipError_t launch_udist(const Grid &g, double h, const int *count, const int *offset,
                        const double *tri, int *occ, const double *rho, double rho_t, double *phi,
                        hipStream_t s) {
  const int cx = (g.nelx + CB - 1) / CB, cy = (g.nely + CB - 1) / CB, cz = (g.nelz + CB - 1) / CB;
  const size_t nc = (size_t)cx * cy * cz;
  hipLaunchKernelGGL(k_occ, dim3((unsigned)std::min<size_t>((nc + 255) / 256, 8192)), dim3(256), 0,
                     s, g.nelx, g.nely, g.nelz, count, (unsigned *)occ);
  static_assert(CB * CB * CB == 64, "one wave per node brick");
  const size_t nbr = (size_t)((g.nelx + CB) / CB) * ((g.nely + CB) / CB) * ((g.nelz + CB) / CB);
  // two bricks per block; at most 8192 blocks, so the occupancy staged per
  // block is reused over several bricks on large grids
  int blocks = (int)std::min<size_t>((nbr + 1) / 2, 8192);
  // TOPO_SDF_OCC_GLOBAL=1 reads the occupancy from memory at any size (the
  // path of grids whose bitmask exceeds the LDS copy), for testing
  const char *e = getenv("TOPO_SDF_OCC_GLOBAL");
  const int occ_lds_allowed = (e && atoi(e) != 0) ? 0 : 1;
  hipLaunchKernelGGL(k_udist, dim3(blocks), dim3(128), 0, s, g.nelx, g.nely, g.nelz, h, count,
                     offset, tri, (const unsigned *)occ, rho, rho_t, phi, occ_lds_allowed);
  return hipGetLastError();
}

// ---------------------------------------------------------------- vf
// Fraction of a tet where the linear interpolant of f is < 0, from the
// fractions s along the edges at which it crosses zero:
//   one negative vertex a:            s_ab s_ac s_ad
//   three negative (positive d):      1 - s_da s_db s_dc
//   two negative (a, b), two positive (c, d): the negative part is the prism
//   a p_ac p_ad | b p_bc p_bd; split in three tets its volume fraction is
//   s_ac s_ad + (1 - s_ac) s_ad s_bc + (1 - s_ad) s_bc s_bd.
__device__ double tet_neg_fraction(const double f[4]) {
  int neg[4], pos[4], nn = 0, np = 0;
  for (int v = 0; v < 4; ++v) {
    if (f[v] < 0.0) neg[nn++] = v;
    else pos[np++] = v;
  }
  if (nn == 0) return 0.0;
  if (nn == 4) return 1.0;
  if (nn == 1) {
    const double fa = f[neg[0]];
    double prod = 1.0;
    for (int q = 0; q < 3; ++q) prod *= fa / (fa - f[pos[q]]);
    return prod;
  }
  if (nn == 3) {
    const double fd = f[pos[0]];
    double prod = 1.0;
    for (int q = 0; q < 3; ++q) prod *= fd / (fd - f[neg[q]]);
    return 1.0 - prod;
  }
  const double fa = f[neg[0]], fb = f[neg[1]], fc = f[pos[0]], fd = f[pos[1]];
  const double s1 = fa / (fa - fc), s2 = fa / (fa - fd);
  const double s3 = fb / (fb - fc), s4 = fb / (fb - fd);
  return s1 * s2 + (1.0 - s1) * s2 * s3 + (1.0 - s2) * s3 * s4;
}

__global__ void k_vf(int nelx, int nely, int nelz, const double *__restrict__ phi,
                     double *__restrict__ vf) {
  const int NX = nelx + 1, NY = nely + 1;
  const size_t nel = (size_t)nelx * nely * nelz;
  for (size_t e = blockIdx.x * (size_t)blockDim.x + threadIdx.x; e < nel;
       e += (size_t)gridDim.x * blockDim.x) {
    const int i = (int)(e % nelx), j = (int)((e / nelx) % nely), k = (int)(e / ((size_t)nelx * nely));
    double F[8];
    int nneg = 0;
    for (int a = 0; a < 8; ++a) {
      F[a] = phi[nidx(NX, NY, i + (a & 1), j + ((a >> 1) & 1), k + (a >> 2))];
      nneg += F[a] < 0.0;
    }
    double v;
    if (nneg == 8) v = 1.0;
    else if (nneg == 0) v = 0.0;
    else {
      double acc = 0.0;
      for (int t = 0; t < 6; ++t) {
        const double f[4] = {F[c_kuhn[t][0]], F[c_kuhn[t][1]], F[c_kuhn[t][2]], F[c_kuhn[t][3]]};
        acc += tet_neg_fraction(f);
      }
      v = acc / 6.0;
    }
    vf[e] = v;
  }
}

hipError_t launch_vf(const Grid &g, const double *phi, double *vf, hipStream_t s) {
  int blocks = (int)((g.nel + 255) / 256);
  if (blocks > 8192) blocks = 8192;
  hipLaunchKernelGGL(k_vf, dim3(blocks), dim3(256), 0, s, g.nelx, g.nely, g.nelz, phi, vf);
  return hipGetLastError();
}

// empty iso-surface: the distance is infinite everywhere
__global__ void k_sign_inf(size_t nn, const double *__restrict__ rho, double rho_t,
                           double *__restrict__ phi) {
  for (size_t n = blockIdx.x * (size_t)blockDim.x + threadIdx.x; n < nn;
       n += (size_t)gridDim.x * blockDim.x)
    phi[n] = (rho[n] >= rho_t) ? -INFINITY : INFINITY;
}

hipError_t launch_sign_inf(const Grid &g, const double *rho, double rho_t, double *phi,
                           hipStream_t s) {
  int blocks = (int)((g.nn + 255) / 256);
  if (blocks > 8192) blocks = 8192;
  hipLaunchKernelGGL(k_sign_inf, dim3(blocks), dim3(256), 0, s, g.nn, rho, rho_t, phi);
  return hipGetLastError();
}

}  // namespace topo
