// Density filter, its adjoint and the sensitivity filter of paper Eq. 4 on the
// voxel grid.  The weights H = rmin - |d| of the integer offsets d with
// |d| < rmin come from a host-built table (float64, correctly rounded sqrt) in
// a fixed order; every element sums its in-bounds offsets in that order with
// no contraction, so the sums are reproducible bit for bit.
#include "common.h"

namespace topo {

#pragma clang fp contract(off)

// mode 0 DENS: out_e = sum (wV) x_i / sum wV
// mode 2 SENS: out_e = sum w (x_i/V) dc_i / ((max(x_e,g)/V) sum w)
// mode 1 DENS_T, pass 1: tmp_e = in_e / (V sum w)
__global__ __launch_bounds__(256) void k_filter_gather(int nelx, int nely, int nelz, int mode,
                                                       int nofs, const int *__restrict__ ofs,
                                                       const double *__restrict__ w, double V,
                                                       const double *__restrict__ x,
                                                       const double *__restrict__ in,
                                                       double *__restrict__ out) {
  const size_t nel = (size_t)nelx * nely * nelz;
  for (size_t e = blockIdx.x * (size_t)blockDim.x + threadIdx.x; e < nel;
       e += (size_t)gridDim.x * blockDim.x) {
    const int i = (int)(e % nelx), j = (int)((e / nelx) % nely), k = (int)(e / ((size_t)nelx * nely));
    double num = 0.0, den = 0.0;
    for (int o = 0; o < nofs; ++o) {
      const int ii = i + ofs[3 * o], jj = j + ofs[3 * o + 1], kk = k + ofs[3 * o + 2];
      if (ii < 0 || ii >= nelx || jj < 0 || jj >= nely || kk < 0 || kk >= nelz) continue;
      const size_t q = (size_t)ii + (size_t)nelx * ((size_t)jj + (size_t)nely * kk);
      if (mode == 0) {
        const double wv = w[o] * V;
        num = num + wv * in[q];
        den = den + wv;
      } else if (mode == 2) {
        num = num + w[o] * ((x[q] / V) * in[q]);
        den = den + w[o];
      } else {
        den = den + w[o];
      }
    }
    if (mode == 0) {
      out[e] = num / den;
    } else if (mode == 2) {
      const double xe = fmax(x[e], 1e-3) / V;
      out[e] = num / (xe * den);
    } else {
      out[e] = in[e] / (den * V);
    }
  }
}

// mode 1 DENS_T, pass 2: out_j = sum (wV) tmp_{j+d}
__global__ __launch_bounds__(256) void k_filter_scatter_t(int nelx, int nely, int nelz, int nofs,
                                                          const int *__restrict__ ofs,
                                                          const double *__restrict__ w, double V,
                                                          const double *__restrict__ tmp,
                                                          double *__restrict__ out) {
  const size_t nel = (size_t)nelx * nely * nelz;
  for (size_t e = blockIdx.x * (size_t)blockDim.x + threadIdx.x; e < nel;
       e += (size_t)gridDim.x * blockDim.x) {
    const int i = (int)(e % nelx), j = (int)((e / nelx) % nely), k = (int)(e / ((size_t)nelx * nely));
    double s = 0.0;
    for (int o = 0; o < nofs; ++o) {
      const int ii = i + ofs[3 * o], jj = j + ofs[3 * o + 1], kk = k + ofs[3 * o + 2];
      if (ii < 0 || ii >= nelx || jj < 0 || jj >= nely || kk < 0 || kk >= nelz) continue;
      const size_t q = (size_t)ii + (size_t)nelx * ((size_t)jj + (size_t)nely * kk);
      s = s + (w[o] * V) * tmp[q];
    }
    out[e] = s;
  }
}

hipError_t launch_filter(const Grid &g, int mode, int nofs, const int *ofs, const double *w,
                         double V, const double *x, const double *in, double *tmp, double *out,
                         hipStream_t s) {
  int blocks = (int)((g.nel + 255) / 256);
  if (blocks > 8192) blocks = 8192;
  if (blocks < 1) blocks = 1;
  if (mode == 1) {
    hipLaunchKernelGGL(k_filter_gather, dim3(blocks), dim3(256), 0, s, g.nelx, g.nely, g.nelz, 1,
                       nofs, ofs, w, V, x, in, tmp);
    hipLaunchKernelGGL(k_filter_scatter_t, dim3(blocks), dim3(256), 0, s, g.nelx, g.nely, g.nelz,
                       nofs, ofs, w, V, tmp, out);
  } else {
    hipLaunchKernelGGL(k_filter_gather, dim3(blocks), dim3(256), 0, s, g.nelx, g.nely, g.nelz,
                       mode, nofs, ofs, w, V, x, in, out);
  }
  return hipGetLastError();
}

}  // namespace topo
