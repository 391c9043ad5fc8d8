// Wall stresses in the local cylindrical frame and their ensemble bands
// (post-processing of the current state).
//
// Per element and sample: local strains from the element's shape-function
// derivatives and its nodal displacements in the local frame (Sec. 2.2.1),
// local stresses through the constitutive matrix with E = (E h) / h, and
// the components in the frame r = element normal, z = centreline tangent
// made orthogonal to r, theta = r x z (Sec. 2.3, fluid-structure coupling).
// The frame vectors are taken to local coordinates, so the global stress
// tensor is never formed: a . S_global . b = (R a) . S_local . (R b).
#include "internal.h"

#include <cmath>

namespace ensfem {
namespace {

__global__ __launch_bounds__(256) void k_stress(int64_t n_el, int32_t ld, const int32_t* __restrict__ tri,
                                                const double* __restrict__ frame, const double* __restrict__ u,
                                                const float* __restrict__ uh, const float* __restrict__ uc,
                                                const double* __restrict__ eh, const double* __restrict__ h,
                                                const double* __restrict__ axial, double nu, double shear_k,
                                                int comp, double* __restrict__ out, int32_t* __restrict__ bad) {
  const int64_t t = (int64_t)blockIdx.x * 256 + threadIdx.x;
  if (t >= n_el * ld) return;
  const int64_t e = t / ld;
  const int s = (int)(t % ld);
  const double* f = frame + (int64_t)kFrameWords * e;
  double R[3][3];
#pragma unroll
  for (int i = 0; i < 3; ++i)
#pragma unroll
    for (int c = 0; c < 3; ++c) R[i][c] = f[3 * i + c];
  // local displacements of the three nodes
  double ul[3][3];
#pragma unroll
  for (int v = 0; v < 3; ++v) {
    const int64_t node = tri[3 * e + v];
    double ug[3];
#pragma unroll
    for (int c = 0; c < 3; ++c) {
      const int64_t idx = (node * 3 + c) * ld + s;
      if (u) ug[c] = u[idx];
      else ug[c] = (double)uh[idx] - (uc ? (double)uc[idx] : 0.0);
    }
#pragma unroll
    for (int i = 0; i < 3; ++i) ul[v][i] = R[i][0] * ug[0] + R[i][1] * ug[1] + R[i][2] * ug[2];
  }
  double exx = 0.0, eyy = 0.0, gxy = 0.0, gxz = 0.0, gyz = 0.0;
#pragma unroll
  for (int v = 0; v < 3; ++v) {
    const double bx = f[9 + v], by = f[12 + v];
    exx += bx * ul[v][0];
    eyy += by * ul[v][1];
    gxy += by * ul[v][0] + bx * ul[v][1];
    gxz += bx * ul[v][2];
    gyz += by * ul[v][2];
  }
  const double E = eh[e * ld + s] / h[e * ld + s];
  const double cE = E / (1.0 - nu * nu);
  const double sxx = cE * (exx + nu * eyy);
  const double syy = cE * (nu * exx + eyy);
  const double txy = cE * 0.5 * (1.0 - nu) * gxy;
  const double txz = cE * 0.5 * shear_k * (1.0 - nu) * gxz;
  const double tyz = cE * 0.5 * shear_k * (1.0 - nu) * gyz;
  // cylindrical frame: r = e_z of the element, z the tangent without its
  // normal part, theta = r x z; all three in local coordinates
  const double a[3] = {axial[3 * e], axial[3 * e + 1], axial[3 * e + 2]};
  const double za[3] = {R[0][0] * a[0] + R[0][1] * a[1] + R[0][2] * a[2],
                        R[1][0] * a[0] + R[1][1] * a[1] + R[1][2] * a[2]};  // in-plane part
  const double zn = sqrt(za[0] * za[0] + za[1] * za[1]);
  const double an = sqrt(a[0] * a[0] + a[1] * a[1] + a[2] * a[2]);
  if (!(zn > 1e-9 * an)) {
    if (s == 0) atomicOr(bad, 1);
    out[t] = 0.0;
    return;
  }
  const double zx = za[0] / zn, zy = za[1] / zn;  // z = (zx, zy, 0)
  const double tx = -zy, ty = zx;                  // theta = (0,0,1) x z
  double v;
  switch (comp) {
    case 0: v = tx * (sxx * tx + txy * ty) + ty * (txy * tx + syy * ty); break;
    case 1: v = zx * (sxx * zx + txy * zy) + zy * (txy * zx + syy * zy); break;
    case 2: v = tx * (sxx * zx + txy * zy) + ty * (txy * zx + syy * zy); break;
    default: v = txz * zx + tyz * zy; break;
  }
  out[t] = v;
}

// One workgroup per row: bitonic sort of the row's S values (padded with
// +inf to a power of two) in LDS, then mean and interpolated quantiles.
__global__ __launch_bounds__(256) void k_bands(int64_t n_rows, int32_t ld, int32_t S, const double* __restrict__ vals,
                                               double p_lo, double p_hi, double* __restrict__ mean,
                                               double* __restrict__ lo, double* __restrict__ hi) {
  __shared__ double buf[kBandsMax];
  __shared__ double red[256];
  const int64_t row = blockIdx.x;
  if (row >= n_rows) return;
  int P = 1;
  while (P < S) P <<= 1;
  const double* r = vals + row * ld;
  double part = 0.0;
  for (int i = threadIdx.x; i < P; i += 256) {
    const double x = i < S ? r[i] : INFINITY;
    buf[i] = x;
    if (i < S) part += x;
  }
  red[threadIdx.x] = part;
  __syncthreads();
  for (int k = 2; k <= P; k <<= 1) {
    for (int j = k >> 1; j > 0; j >>= 1) {
      for (int i = threadIdx.x; i < P; i += 256) {
        const int l = i ^ j;
        if (l > i) {
          const bool up = (i & k) == 0;
          const double a = buf[i], b = buf[l];
          if ((a > b) == up) {
            buf[i] = b;
            buf[l] = a;
          }
        }
      }
      __syncthreads();
    }
  }
  for (int o = 128; o > 0; o >>= 1) {
    if (threadIdx.x < o) red[threadIdx.x] += red[threadIdx.x + o];
    __syncthreads();
  }
  if (threadIdx.x == 0) {
    mean[row] = red[0] / (double)S;
    const double pl = p_lo * (double)(S - 1), ph = p_hi * (double)(S - 1);
    const int il = (int)floor(pl), ih = (int)floor(ph);
    const double vl1 = buf[il < S - 1 ? il + 1 : il], vh1 = buf[ih < S - 1 ? ih + 1 : ih];
    lo[row] = buf[il] + (pl - (double)il) * (vl1 - buf[il]);
    hi[row] = buf[ih] + (ph - (double)ih) * (vh1 - buf[ih]);
  }
}

inline unsigned grid_for(int64_t n, int b) { return (unsigned)((n + b - 1) / b); }

}  // namespace

hipError_t launch_stress(int64_t n_el, int32_t ld, const int32_t* tri, const double* frame, const double* u,
                         const float* uh, const float* uc, const double* eh, const double* h,
                         const double* axial, double nu, double shear_k, int comp, double* out, int32_t* bad,
                         hipStream_t st) {
  const int64_t n = n_el * ld;
  if (n == 0) return hipSuccess;
  if (comp < 0 || comp > 3) return hipErrorInvalidValue;
  k_stress<<<grid_for(n, 256), 256, 0, st>>>(n_el, ld, tri, frame, u, uh, uc, eh, h, axial, nu, shear_k, comp,
                                              out, bad);
  return hipGetLastError();
}

hipError_t launch_bands(int64_t n_rows, int32_t ld, int32_t S, const double* vals, double p_lo, double p_hi,
                        double* mean, double* lo, double* hi, hipStream_t st) {
  if (n_rows == 0) return hipSuccess;
  if (S < 1 || S > kBandsMax || S > ld) return hipErrorInvalidValue;
  k_bands<<<(unsigned)n_rows, 256, 0, st>>>(n_rows, ld, S, vals, p_lo, p_hi, mean, lo, hi);
  return hipGetLastError();
}

}  // namespace ensfem
