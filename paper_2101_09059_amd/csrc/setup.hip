// Set-up kernels, run once per mesh / ensemble (FP64):
//   * reference element stiffness Khat_e (Sec. 2.2.1) in the global frame
//     and its largest eigenvalue (cyclic Jacobi on the 9x9);
//   * the per-adjacency 3x6 stiffness blocks used by the node-gather apply;
//   * the lumped mass per node and sample (Sec. 2.3);
//   * the element-eigenvalue stability bound.
#include "internal.h"

#include <cmath>

namespace ensfem {
namespace {

// Khat_e = A_e * B^T (C/E) B rotated to the global frame.  B is the 5x9
// strain matrix of the linear triangle with rows du_x/dx, du_y/dy, gamma_xy,
// du_z/dx, du_z/dy; C/E is block diagonal: [[1,nu],[nu,1]]/(1-nu^2),
// (1-nu)/2/(1-nu^2), k(1-nu)/2/(1-nu^2) twice.  With bx_p = dN_p/dx and
// by_p = dN_p/dy the product B^T C B couples node p and node q through
//   (x,x): c11 bx_p bx_q + c33 by_p by_q      (x,y): c12 bx_p by_q + c33 by_p bx_q
//   (y,x): c12 by_p bx_q + c33 bx_p by_q      (y,y): c11 by_p by_q + c33 bx_p bx_q
//   (z,z): c44 (bx_p bx_q + by_p by_q)        and zero between in-plane and z.
__global__ __launch_bounds__(64) void k_element_setup(int64_t n_el, const double* __restrict__ xyz,
                                                      const int32_t* __restrict__ tri, double nu,
                                                      double shear_k, double* __restrict__ khat,
                                                      double* __restrict__ area,
                                                      double* __restrict__ lam,
                                                      double* __restrict__ frame,
                                                      int32_t* __restrict__ bad) {
  const int64_t e = (int64_t)blockIdx.x * 64 + threadIdx.x;
  if (e >= n_el) return;
  double p[3][3];
#pragma unroll
  for (int v = 0; v < 3; ++v) {
    const int64_t nd = tri[3 * e + v];
#pragma unroll
    for (int c = 0; c < 3; ++c) p[v][c] = xyz[3 * nd + c];
  }
  double da[3], db[3];
#pragma unroll
  for (int c = 0; c < 3; ++c) {
    da[c] = p[1][c] - p[0][c];
    db[c] = p[2][c] - p[0][c];
  }
  const double la = sqrt(da[0] * da[0] + da[1] * da[1] + da[2] * da[2]);
  double nz[3] = {da[1] * db[2] - da[2] * db[1], da[2] * db[0] - da[0] * db[2],
                  da[0] * db[1] - da[1] * db[0]};
  const double ln = sqrt(nz[0] * nz[0] + nz[1] * nz[1] + nz[2] * nz[2]);
  double R[3][3];  // rows e_x, e_y, e_z
#pragma unroll
  for (int c = 0; c < 3; ++c) {
    R[0][c] = da[c] / la;
    R[2][c] = nz[c] / ln;
  }
  R[1][0] = R[2][1] * R[0][2] - R[2][2] * R[0][1];
  R[1][1] = R[2][2] * R[0][0] - R[2][0] * R[0][2];
  R[1][2] = R[2][0] * R[0][1] - R[2][1] * R[0][0];
  // local coordinates, node 1 at the origin
  const double x2 = da[0] * R[0][0] + da[1] * R[0][1] + da[2] * R[0][2];
  const double y2 = da[0] * R[1][0] + da[1] * R[1][1] + da[2] * R[1][2];
  const double x3 = db[0] * R[0][0] + db[1] * R[0][1] + db[2] * R[0][2];
  const double y3 = db[0] * R[1][0] + db[1] * R[1][1] + db[2] * R[1][2];
  const double A = 0.5 * (x2 * y3 - x3 * y2);
  area[e] = A;
  if (!(A > 0.0) || !(la > 0.0) || !(ln > 0.0)) {
    atomicOr(bad, 1);
    lam[e] = 0.0;
    for (int i = 0; i < 81; ++i) khat[81 * e + i] = 0.0;
    for (int i = 0; i < kFrameWords; ++i) frame[kFrameWords * e + i] = 0.0;
    return;
  }
  const double inv2A = 1.0 / (2.0 * A);
  // x_ij = x_i - x_j with x_1 = y_1 = 0
  const double bx[3] = {(y2 - y3) * inv2A, (y3 - 0.0) * inv2A, (0.0 - y2) * inv2A};
  const double by[3] = {(x3 - x2) * inv2A, (0.0 - x3) * inv2A, (x2 - 0.0) * inv2A};
  // frame rows and shape-function derivatives, for stress post-processing
#pragma unroll
  for (int i = 0; i < 3; ++i)
#pragma unroll
    for (int c = 0; c < 3; ++c) frame[kFrameWords * e + 3 * i + c] = R[i][c];
#pragma unroll
  for (int v = 0; v < 3; ++v) {
    frame[kFrameWords * e + 9 + v] = bx[v];
    frame[kFrameWords * e + 12 + v] = by[v];
  }
  frame[kFrameWords * e + 15] = 0.0;
  const double inv = 1.0 / (1.0 - nu * nu);
  const double c11 = inv, c12 = nu * inv, c33 = 0.5 * (1.0 - nu) * inv;
  const double c44 = 0.5 * shear_k * (1.0 - nu) * inv;

  double K[9][9];
#pragma unroll
  for (int pn = 0; pn < 3; ++pn) {
#pragma unroll
    for (int qn = 0; qn < 3; ++qn) {
      double kl[3][3];
      kl[0][0] = A * (c11 * bx[pn] * bx[qn] + c33 * by[pn] * by[qn]);
      kl[0][1] = A * (c12 * bx[pn] * by[qn] + c33 * by[pn] * bx[qn]);
      kl[1][0] = A * (c12 * by[pn] * bx[qn] + c33 * bx[pn] * by[qn]);
      kl[1][1] = A * (c11 * by[pn] * by[qn] + c33 * bx[pn] * bx[qn]);
      kl[0][2] = kl[1][2] = kl[2][0] = kl[2][1] = 0.0;
      kl[2][2] = A * c44 * (bx[pn] * bx[qn] + by[pn] * by[qn]);
      // global block = R^T kl R
#pragma unroll
      for (int i = 0; i < 3; ++i) {
#pragma unroll
        for (int j = 0; j < 3; ++j) {
          double s = 0.0;
#pragma unroll
          for (int k = 0; k < 3; ++k) {
#pragma unroll
            for (int l = 0; l < 3; ++l) s += R[k][i] * kl[k][l] * R[l][j];
          }
          K[3 * pn + i][3 * qn + j] = s;
        }
      }
    }
  }
  // exact symmetry (the two triangles of the product are rounded alike)
#pragma unroll
  for (int i = 0; i < 9; ++i) {
#pragma unroll
    for (int j = i + 1; j < 9; ++j) {
      const double s = 0.5 * (K[i][j] + K[j][i]);
      K[i][j] = s;
      K[j][i] = s;
    }
  }
#pragma unroll
  for (int i = 0; i < 9; ++i) {
#pragma unroll
    for (int j = 0; j < 9; ++j) khat[81 * e + 9 * i + j] = K[i][j];
  }

  // Largest eigenvalue: cyclic Jacobi rotations until the off-diagonal
  // mass is below 1e-30 of the Frobenius mass.
  double fro = 0.0;
#pragma unroll
  for (int i = 0; i < 9; ++i) {
#pragma unroll
    for (int j = 0; j < 9; ++j) fro += K[i][j] * K[i][j];
  }
  for (int sweep = 0; sweep < 40; ++sweep) {
    double off = 0.0;
#pragma unroll
    for (int i = 0; i < 9; ++i) {
#pragma unroll
      for (int j = i + 1; j < 9; ++j) off += K[i][j] * K[i][j];
    }
    if (off <= 1e-30 * fro) break;
#pragma unroll
    for (int pp = 0; pp < 8; ++pp) {
#pragma unroll
      for (int qq = pp + 1; qq < 9; ++qq) {
        const double apq = K[pp][qq];
        if (apq != 0.0) {
          const double th = (K[qq][qq] - K[pp][pp]) / (2.0 * apq);
          const double t = (th >= 0.0 ? 1.0 : -1.0) / (fabs(th) + sqrt(th * th + 1.0));
          const double c = 1.0 / sqrt(t * t + 1.0);
          const double s = t * c;
          K[pp][pp] -= t * apq;
          K[qq][qq] += t * apq;
          K[pp][qq] = 0.0;
          K[qq][pp] = 0.0;
#pragma unroll
          for (int r = 0; r < 9; ++r) {
            if (r != pp && r != qq) {
              const double arp = K[r][pp], arq = K[r][qq];
              const double np_ = c * arp - s * arq;
              const double nq_ = s * arp + c * arq;
              K[r][pp] = np_;
              K[pp][r] = np_;
              K[r][qq] = nq_;
              K[qq][r] = nq_;
            }
          }
        }
      }
    }
  }
  double lmax = K[0][0];
#pragma unroll
  for (int i = 1; i < 9; ++i) lmax = fmax(lmax, K[i][i]);
  lam[e] = lmax;
}

// 3x6 block [Khat_ab | Khat_ac] of each adjacency entry (node a = local
// index `loc`, b and c the next two nodes in cyclic order).
__global__ __launch_bounds__(256) void k_adjacency_blocks(int64_t n_adj,
                                                          const int32_t* __restrict__ adj_el,
                                                          const uint8_t* __restrict__ adj_loc,
                                                          const double* __restrict__ khat,
                                                          double* __restrict__ k64,
                                                          float* __restrict__ k32) {
  const int64_t t = (int64_t)blockIdx.x * 256 + threadIdx.x;
  if (t >= n_adj * 18) return;
  const int64_t k = t / 18;
  const int w = (int)(t % 18);
  const int i = w / 6, j = w % 6;
  const int a = adj_loc[k];
  const int other = (j < 3) ? (a + 1) % 3 : (a + 2) % 3;
  const double v = khat[81 * (int64_t)adj_el[k] + 9 * (3 * a + i) + 3 * other + (j % 3)];
  k64[t] = v;
  if (k32) k32[t] = (float)v;
}

// m_{i,s} = sum over incident elements of rho h_{e,s} A_e / 3; stores 1/m.
// Mass-scaling factor of an element and sample: max(1, omega^2 dt_t^2 / 4)
// for a target step dt_t > 0 (density raised just enough for the element's
// eigenvalue bound to allow dt_t), 1 without scaling.
__device__ __forceinline__ double mass_factor(double eh, double h, double lam, double area, double rho,
                                              double dt_t) {
  if (!(dt_t > 0.0)) return 1.0;
  const double w2 = 3.0 * (eh / h) * (lam / (rho * area));
  return fmax(1.0, w2 * (dt_t * dt_t / 4.0));
}

__global__ __launch_bounds__(256) void k_lumped_mass(int32_t n_nodes, int32_t ld,
                                                     const int32_t* __restrict__ adj_ptr,
                                                     const int32_t* __restrict__ adj_el,
                                                     const double* __restrict__ area,
                                                     const double* __restrict__ h, double rho,
                                                     const double* __restrict__ eh,
                                                     const double* __restrict__ lam, double dt_t,
                                                     double* __restrict__ minv64,
                                                     float* __restrict__ minv32) {
  const int64_t t = (int64_t)blockIdx.x * 256 + threadIdx.x;
  if (t >= (int64_t)n_nodes * ld) return;
  const int64_t node = t / ld;
  const int s = (int)(t % ld);
  double m = 0.0;
  for (int k = adj_ptr[node]; k < adj_ptr[node + 1]; ++k) {
    const int64_t e = adj_el[k];
    if (dt_t > 0.0) {
      const double f = mass_factor(eh[e * ld + s], h[e * ld + s], lam[e], area[e], rho, dt_t);
      m += rho * f * h[e * ld + s] * area[e] / 3.0;
    } else {
      m += rho * h[e * ld + s] * area[e] / 3.0;
    }
  }
  const double mi = 1.0 / m;
  minv64[t] = mi;
  if (minv32) minv32[t] = (float)mi;
}

// omega^2 bound per (element, sample): 3 E lambda_max / (rho A); global max.
__global__ __launch_bounds__(256) void k_cfl_max(int64_t n_el, int32_t ld, int32_t S,
                                                 const double* __restrict__ eh,
                                                 const double* __restrict__ h,
                                                 const double* __restrict__ lam,
                                                 const double* __restrict__ area, double rho, double dt_t,
                                                 unsigned long long* __restrict__ out_bits) {
  __shared__ double red[256];
  double w = 0.0;
  // grid-stride: one atomic per workgroup, not per element-sample
  for (int64_t t = (int64_t)blockIdx.x * 256 + threadIdx.x; t < n_el * S; t += (int64_t)gridDim.x * 256) {
    const int64_t e = t / S;
    const int s = (int)(t % S);
    const double E = eh[e * ld + s] / h[e * ld + s];
    double v = 3.0 * E * (lam[e] / (rho * area[e]));
    if (dt_t > 0.0) v = v / mass_factor(eh[e * ld + s], h[e * ld + s], lam[e], area[e], rho, dt_t);
    if (!(v >= 0.0)) v = INFINITY;  // NaN -> flagged as unbounded
    w = fmax(w, v);
  }
  red[threadIdx.x] = w;
  __syncthreads();
  for (int o = 128; o > 0; o >>= 1) {
    if (threadIdx.x < o) red[threadIdx.x] = fmax(red[threadIdx.x], red[threadIdx.x + o]);
    __syncthreads();
  }
  // non-negative doubles order like their bit patterns
  if (threadIdx.x == 0) atomicMax(out_bits, (unsigned long long)__double_as_longlong(red[0]));
}

// Shared-stiffness block rows: K_ij = sum over the elements e containing
// both i and j of (E h)_e Khat_e[i, j] (3x3), summed in adjacency order by
// the thread that owns row i.  adj_slot[k] = (block of b, block of c).
__global__ __launch_bounds__(256) void k_bsr_assemble(int32_t n_nodes, int32_t ld,
                                                      const int32_t* __restrict__ adj_ptr,
                                                      const int32_t* __restrict__ adj_el,
                                                      const uint8_t* __restrict__ adj_loc,
                                                      const int2* __restrict__ adj_slot,
                                                      const int32_t* __restrict__ bsr_ptr,
                                                      const double* __restrict__ khat,
                                                      const double* __restrict__ eh,
                                                      double* __restrict__ bsr) {
  const int node = blockIdx.x * 256 + threadIdx.x;
  if (node >= n_nodes) return;
  for (int64_t k = (int64_t)bsr_ptr[node] * 9; k < (int64_t)bsr_ptr[node + 1] * 9; ++k) bsr[k] = 0.0;
  for (int k = adj_ptr[node]; k < adj_ptr[node + 1]; ++k) {
    const int64_t e = adj_el[k];
    const int a = adj_loc[k];
    const double w = eh[e * ld];
    const int2 sl = adj_slot[k];
    const double* K = khat + 81 * e;
    for (int t = 0; t < 2; ++t) {
      const int other = (a + 1 + t) % 3;
      double* B = bsr + 9 * (int64_t)(t == 0 ? sl.x : sl.y);
      for (int r = 0; r < 3; ++r)
        for (int c = 0; c < 3; ++c) B[3 * r + c] += w * K[9 * (3 * a + r) + 3 * other + c];
    }
  }
}

__global__ __launch_bounds__(256) void k_cast_f32(int64_t n, const double* __restrict__ src,
                                                  float* __restrict__ dst) {
  const int64_t t = (int64_t)blockIdx.x * 256 + threadIdx.x;
  if (t < n) dst[t] = (float)src[t];
}

inline unsigned grid_for(int64_t n, int per) { return (unsigned)((n + per - 1) / per); }

}  // namespace

hipError_t launch_element_setup(int64_t n_el, const double* xyz, const int32_t* tri, double nu,
                                double shear_k, double* khat, double* area, double* lam,
                                double* frame, int32_t* bad, hipStream_t st) {
  if (n_el == 0) return hipSuccess;
  k_element_setup<<<grid_for(n_el, 64), 64, 0, st>>>(n_el, xyz, tri, nu, shear_k, khat, area, lam,
                                                      frame, bad);
  return hipGetLastError();
}

hipError_t launch_adjacency_blocks(int64_t n_adj, const int32_t* adj_el, const uint8_t* adj_loc,
                                   const double* khat, double* k64, float* k32, hipStream_t st) {
  if (n_adj == 0) return hipSuccess;
  k_adjacency_blocks<<<grid_for(n_adj * 18, 256), 256, 0, st>>>(n_adj, adj_el, adj_loc, khat, k64,
                                                                 k32);
  return hipGetLastError();
}

hipError_t launch_lumped_mass(int32_t n_nodes, int32_t ld, const int32_t* adj_ptr,
                              const int32_t* adj_el, const double* area, const double* h, double rho,
                              const double* eh, const double* lam, double dt_t, double* minv64, float* minv32,
                              hipStream_t st) {
  const int64_t n = (int64_t)n_nodes * ld;
  if (n == 0) return hipSuccess;
  k_lumped_mass<<<grid_for(n, 256), 256, 0, st>>>(n_nodes, ld, adj_ptr, adj_el, area, h, rho, eh, lam, dt_t,
                                                   minv64, minv32);
  return hipGetLastError();
}

hipError_t launch_cfl_max(int64_t n_el, int32_t ld, int32_t S, const double* eh, const double* h,
                          const double* lam, const double* area, double rho, double dt_t,
                          unsigned long long* out_bits, hipStream_t st) {
  const int64_t n = n_el * S;
  if (n == 0) return hipSuccess;
  const unsigned g = grid_for(n, 256) < 2048u ? grid_for(n, 256) : 2048u;
  k_cfl_max<<<g, 256, 0, st>>>(n_el, ld, S, eh, h, lam, area, rho, dt_t, out_bits);
  return hipGetLastError();
}

hipError_t launch_bsr_assemble(int32_t n_nodes, int32_t ld, const int32_t* adj_ptr,
                               const int32_t* adj_el, const uint8_t* adj_loc, const int2* adj_slot,
                               const int32_t* bsr_ptr, const double* khat, const double* eh,
                               double* bsr64, hipStream_t st) {
  if (n_nodes == 0) return hipSuccess;
  k_bsr_assemble<<<grid_for(n_nodes, 256), 256, 0, st>>>(n_nodes, ld, adj_ptr, adj_el, adj_loc, adj_slot,
                                                          bsr_ptr, khat, eh, bsr64);
  return hipGetLastError();
}

hipError_t launch_cast_f32(int64_t n, const double* src, float* dst, hipStream_t st) {
  if (n == 0) return hipSuccess;
  k_cast_f32<<<grid_for(n, 256), 256, 0, st>>>(n, src, dst);
  return hipGetLastError();
}

}  // namespace ensfem
