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

// SPL consecutive samples per thread (one 8 * SPL-byte access per row).
// UNI: ld is a multiple of 64 * SPL, so a wave's 64 threads share one
// element and the element's connectivity, frame and tangent are
// wave-uniform (scalar loads).
template <int SPL, bool UNI>
__global__ __launch_bounds__(256) void k_stress(int64_t n_el, int32_t ld, const int32_t* __restrict__ tri,
                                                const double* __restrict__ frame, const double* __restrict__ u,
                                                const float* __restrict__ uh, const float* __restrict__ uc,
                                                const double* __restrict__ eh, const double* __restrict__ h,
                                                const double* __restrict__ axial, double nu, double shear_k,
                                                int comp, double* __restrict__ out, int32_t* __restrict__ bad) {
  typedef double D __attribute__((ext_vector_type(SPL)));
  typedef float F __attribute__((ext_vector_type(SPL)));
  const int64_t per = ld / SPL;  // threads per element
  const int64_t t = (int64_t)blockIdx.x * 256 + threadIdx.x;
  if (t >= n_el * per) return;
  const int64_t e = UNI ? (int64_t)__builtin_amdgcn_readfirstlane((int)(t / per)) : t / per;
  const int s = (int)(t % per) * SPL;
  const double* f = frame + (int64_t)kFrameWords * e;
  double R[3][3];
#pragma unroll
  for (int i = 0; i < 3; ++i)
#pragma unroll
    for (int c = 0; c < 3; ++c) R[i][c] = f[3 * i + c];
  // local displacements of the three nodes
  double ul[3][3][SPL];
#pragma unroll
  for (int v = 0; v < 3; ++v) {
    const int64_t node = tri[3 * e + v];
    double ug[3][SPL];
#pragma unroll
    for (int c = 0; c < 3; ++c) {
      const int64_t idx = (node * 3 + c) * ld + s;
      if (u) {
        const D x = *reinterpret_cast<const D*>(u + idx);
#pragma unroll
        for (int k = 0; k < SPL; ++k) ug[c][k] = x[k];
      } else {
        const F a = *reinterpret_cast<const F*>(uh + idx);
        F b = {};
        if (uc) b = *reinterpret_cast<const F*>(uc + idx);
#pragma unroll
        for (int k = 0; k < SPL; ++k) ug[c][k] = (double)a[k] - (uc ? (double)b[k] : 0.0);
      }
    }
#pragma unroll
    for (int i = 0; i < 3; ++i)
#pragma unroll
      for (int k = 0; k < SPL; ++k) ul[v][i][k] = R[i][0] * ug[0][k] + R[i][1] * ug[1][k] + R[i][2] * ug[2][k];
  }
  // cylindrical frame: r = e_z of the element, z the tangent without its
  // normal part, theta = r x z; all three in local coordinates
  const double a[3] = {axial[3 * e], axial[3 * e + 1], axial[3 * e + 2]};
  const double za[3] = {R[0][0] * a[0] + R[0][1] * a[1] + R[0][2] * a[2],
                        R[1][0] * a[0] + R[1][1] * a[1] + R[1][2] * a[2]};  // in-plane part
  const double zn = sqrt(za[0] * za[0] + za[1] * za[1]);
  const double an = sqrt(a[0] * a[0] + a[1] * a[1] + a[2] * a[2]);
  D res;
  if (!(zn > 1e-9 * an)) {
    if (s == 0) atomicOr(bad, 1);
    res = 0.0;
    *reinterpret_cast<D*>(out + e * ld + s) = res;
    return;
  }
  const double zx = za[0] / zn, zy = za[1] / zn;  // z = (zx, zy, 0)
  const double tx = -zy, ty = zx;                  // theta = (0,0,1) x z
  const D ehv = *reinterpret_cast<const D*>(eh + e * ld + s);
  const D hv = *reinterpret_cast<const D*>(h + e * ld + s);
#pragma unroll
  for (int k = 0; k < SPL; ++k) {
    double exx = 0.0, eyy = 0.0, gxy = 0.0, gxz = 0.0, gyz = 0.0;
#pragma unroll
    for (int v = 0; v < 3; ++v) {
      const double bx = f[9 + v], by = f[12 + v];
      exx += bx * ul[v][0][k];
      eyy += by * ul[v][1][k];
      gxy += by * ul[v][0][k] + bx * ul[v][1][k];
      gxz += bx * ul[v][2][k];
      gyz += by * ul[v][2][k];
    }
    const double E = ehv[k] / hv[k];
    const double cE = E / (1.0 - nu * nu);
    const double sxx = cE * (exx + nu * eyy);
    const double syy = cE * (nu * exx + eyy);
    const double txy = cE * 0.5 * (1.0 - nu) * gxy;
    const double txz = cE * 0.5 * shear_k * (1.0 - nu) * gxz;
    const double tyz = cE * 0.5 * shear_k * (1.0 - nu) * gyz;
    double v;
    switch (comp) {
      case 0: v = tx * (sxx * tx + txy * ty) + ty * (txy * tx + syy * ty); break;
      case 1: v = zx * (sxx * zx + txy * zy) + zy * (txy * zx + syy * zy); break;
      case 2: v = tx * (sxx * zx + txy * zy) + ty * (txy * zx + syy * zy); break;
      default: v = txz * zx + tyz * zy; break;
    }
    res[k] = v;
  }
  *reinterpret_cast<D*>(out + e * ld + s) = res;
}

// One workgroup per row (S > 512): bitonic sort of the row's S values
// (padded with +inf to a power of two) in LDS, then mean and interpolated
// quantiles.
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

// Value of lane (lane ^ M) for a compile-time lane mask M: DPP quad
// permutes for 1 and 2, ds_swizzle (bitmask mode, within 32 lanes) up to
// 16, ds_bpermute for 32.
template <int M>
__device__ __forceinline__ int xor_lane_b32(int x, int lane) {
  if constexpr (M == 1) return __builtin_amdgcn_mov_dpp(x, 0xB1, 0xF, 0xF, true);  // quad_perm(1,0,3,2)
  else if constexpr (M == 2) return __builtin_amdgcn_mov_dpp(x, 0x4E, 0xF, 0xF, true);  // quad_perm(2,3,0,1)
  else if constexpr (M < 32) return __builtin_amdgcn_ds_swizzle(x, (M << 10) | 0x1F);
  else return __builtin_amdgcn_ds_bpermute((lane ^ M) << 2, x);
}

template <int M>
__device__ __forceinline__ double xor_lane(double x, int lane) {
  const int lo = xor_lane_b32<M>(__double2loint(x), lane);
  const int hi = xor_lane_b32<M>(__double2hiint(x), lane);
  return __hiloint2double(hi, lo);
}

__device__ __forceinline__ double xor_lane(double x, int m, int lane) {
  switch (m) {
    case 1: return xor_lane<1>(x, lane);
    case 2: return xor_lane<2>(x, lane);
    case 4: return xor_lane<4>(x, lane);
    case 8: return xor_lane<8>(x, lane);
    case 16: return xor_lane<16>(x, lane);
    default: return xor_lane<32>(x, lane);
  }
}

// One wave per row for S <= 64 K: element e = K lane + k sits in register
// k of lane `lane` (+inf past S), so the bitonic network's exchanges at
// distance j < K stay inside a lane and the others are cross-lane
// exchanges at lane distance j / K; no LDS array and no barrier.  The
// mean sums each lane's K values in order, then the lanes by a butterfly.
template <int K>
__device__ __forceinline__ double pick(const double (&v)[K], int k) {
  double x = v[0];
#pragma unroll
  for (int t = 1; t < K; ++t)
    if (t == k) x = v[t];
  return x;
}

template <int K>
__global__ __launch_bounds__(256) void k_bands_wave(int64_t n_rows, int32_t ld, int32_t S,
                                                    const double* __restrict__ vals, double p_lo, double p_hi,
                                                    double* __restrict__ mean, double* __restrict__ lo,
                                                    double* __restrict__ hi) {
  constexpr int P = 64 * K;
  const int lane = threadIdx.x % 64;
  const int64_t row = (int64_t)blockIdx.x * 4 + threadIdx.x / 64;
  if (row >= n_rows) return;  // whole wave
  const double* r = vals + row * ld;
  double v[K];
  double part = 0.0;
#pragma unroll
  for (int k = 0; k < K; ++k) {
    const int e = K * lane + k;
    v[k] = e < S ? r[e] : INFINITY;
    if (e < S) part += v[k];
  }
#pragma unroll
  for (int size = 2; size <= P; size <<= 1) {
    // ascending block?  For size >= K the bit lies in the lane index.
    const bool up_lane = size >= K ? (lane & (size / K)) == 0 : true;
#pragma unroll
    for (int j = size >> 1; j > 0; j >>= 1) {
      if (j >= K) {
        const int m = j / K;
        const bool keep_min = ((lane & m) == 0) == up_lane;
#pragma unroll
        for (int k = 0; k < K; ++k) {
          const double b = xor_lane(v[k], m, lane);
          const double mn = fmin(v[k], b), mx = fmax(v[k], b);
          v[k] = keep_min ? mn : mx;
        }
      } else {
#pragma unroll
        for (int k = 0; k < K; ++k) {
          if (k & j) continue;
          const bool up = size >= K ? up_lane : (k & size) == 0;
          const double mn = fmin(v[k], v[k | j]), mx = fmax(v[k], v[k | j]);
          v[k] = up ? mn : mx;
          v[k | j] = up ? mx : mn;
        }
      }
    }
  }
#pragma unroll
  for (int o = 32; o > 0; o >>= 1) part += __shfl_xor(part, o);
  const double pl = p_lo * (double)(S - 1), ph = p_hi * (double)(S - 1);
  const int il = (int)floor(pl), ih = (int)floor(ph);
  const int il1 = il < S - 1 ? il + 1 : il, ih1 = ih < S - 1 ? ih + 1 : ih;
  const double a0 = __shfl(pick<K>(v, il % K), il / K), a1 = __shfl(pick<K>(v, il1 % K), il1 / K);
  const double b0 = __shfl(pick<K>(v, ih % K), ih / K), b1 = __shfl(pick<K>(v, ih1 % K), ih1 / K);
  if (lane == 0) {
    mean[row] = part / (double)S;
    lo[row] = a0 + (pl - (double)il) * (a1 - a0);
    hi[row] = b0 + (ph - (double)ih) * (b1 - b0);
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
  // two samples per thread when the padded width is even (it always is a
  // multiple of 8); a wave shares one element when ld is a multiple of 128
  if (ld % 2 == 0) {
    const int64_t nt = n / 2;
    if (ld % 128 == 0 && n_el <= INT32_MAX)
      k_stress<2, true><<<grid_for(nt, 256), 256, 0, st>>>(n_el, ld, tri, frame, u, uh, uc, eh, h, axial, nu, shear_k,
                                                          comp, out, bad);
    else
      k_stress<2, false><<<grid_for(nt, 256), 256, 0, st>>>(n_el, ld, tri, frame, u, uh, uc, eh, h, axial, nu,
                                                           shear_k, comp, out, bad);
  } else if (ld % 64 == 0 && n_el <= INT32_MAX) {
    k_stress<1, true><<<grid_for(n, 256), 256, 0, st>>>(n_el, ld, tri, frame, u, uh, uc, eh, h, axial, nu, shear_k,
                                                       comp, out, bad);
  } else {
    k_stress<1, false><<<grid_for(n, 256), 256, 0, st>>>(n_el, ld, tri, frame, u, uh, uc, eh, h, axial, nu, shear_k,
                                                        comp, out, bad);
  }
  return hipGetLastError();
}

hipError_t launch_bands(int64_t n_rows, int32_t ld, int32_t S, const double* vals, double p_lo, double p_hi,
                        double* mean, double* lo, double* hi, hipStream_t st) {
  if (n_rows == 0) return hipSuccess;
  if (S < 1 || S > kBandsMax || S > ld) return hipErrorInvalidValue;
  const unsigned g4 = grid_for(n_rows, 4);
  if (S <= 64)
    k_bands_wave<1><<<g4, 256, 0, st>>>(n_rows, ld, S, vals, p_lo, p_hi, mean, lo, hi);
  else if (S <= 128)
    k_bands_wave<2><<<g4, 256, 0, st>>>(n_rows, ld, S, vals, p_lo, p_hi, mean, lo, hi);
  else if (S <= 256)
    k_bands_wave<4><<<g4, 256, 0, st>>>(n_rows, ld, S, vals, p_lo, p_hi, mean, lo, hi);
  else if (S <= 512)
    k_bands_wave<8><<<g4, 256, 0, st>>>(n_rows, ld, S, vals, p_lo, p_hi, mean, lo, hi);
  else
    k_bands<<<(unsigned)n_rows, 256, 0, st>>>(n_rows, ld, S, vals, p_lo, p_hi, mean, lo, hi);
  return hipGetLastError();
}

}  // namespace ensfem
