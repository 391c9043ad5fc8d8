// Time-stepping kernels of the ensemble wall solver.
//
// Fused step (node-gather): one thread per (node, sample), samples fastest
// so every load of an ensemble array is a contiguous run of `SB` samples.
// For node a with incident elements e (other nodes b, c):
//
//   R_a,s = sum_e (E h)_{e,s} ( Khat_ab (u_b - u_a) + Khat_ac (u_c - u_a) )
//
// which equals row-block a of sum_e (E h)_{e,s} Khat_e u_e because every
// row of Khat_e annihilates rigid translations (the diagonal block is minus
// the sum of the off-diagonal blocks); writing it on differences removes
// the diagonal blocks and cancels the rigid part before rounding.  Then the
// central-difference update (eq. dynamicsCD, lumped M, C = alpha M):
//
//   (1 + a) u_{n+1} = dt^2 m^-1 (g(t_n) F - R) + 2 u_n - (1 - a) u_{n-1}
//
// or, for the FP32 states, its velocity form
//   v_{n+1/2} = ((1 - a) v_{n-1/2} + dt m^-1 (g F - R)) / (1 + a),
//   u_{n+1}   = u_n + dt v_{n+1/2}   (Kahan-compensated in F32_KAHAN).
// Clamped dofs are written as zero.  Optional outputs in the same pass:
// running peak radial displacement and the per-sample discrete energy.
#include "internal.h"

#include <cmath>

namespace ensfem {
namespace {

template <int SB>
__device__ __forceinline__ bool wg_coords(const StepArgs& p, int& nb, int& sb) {
  // Workgroups are dealt round-robin to the 8 XCDs; give each XCD a
  // contiguous range of logical tiles so neighbouring node blocks share an L2.
  const unsigned G = gridDim.x;
  const unsigned per = G >> 3;
  const unsigned w = blockIdx.x;
  const unsigned L = (w & 7u) * per + (w >> 3);
  if (p.sb_inner) {
    sb = (int)(L % (unsigned)p.n_sb);
    nb = (int)(L / (unsigned)p.n_sb);
  } else {
    nb = (int)(L % (unsigned)p.n_nb);
    sb = (int)(L / (unsigned)p.n_nb);
  }
  return nb < p.n_nb && sb < p.n_sb;
}

template <typename AT, typename ST>
__device__ __forceinline__ void gather_apply(const StepArgs& p, int node, int64_t ld, int s,
                                             const ST* __restrict__ U, ST ua0, ST ua1, ST ua2,
                                             AT& r0, AT& r1, AT& r2) {
  const int kb = p.adj.ptr[node];
  const int ke = p.adj.ptr[node + 1];
  const AT* __restrict__ KB = static_cast<const AT*>(p.adj.k);
  const AT* __restrict__ EH = static_cast<const AT*>(p.eh);
  r0 = r1 = r2 = AT(0);
#pragma unroll 2
  for (int k = kb; k < ke; ++k) {
    const int64_t e = p.adj.el[k];
    const int2 bc = p.adj.nb[k];
    const AT* __restrict__ kk = KB + (int64_t)k * 18;
    const AT eh = EH[e * ld + s];
    const int64_t rb = (int64_t)bc.x * 3, rc = (int64_t)bc.y * 3;
    const AT d0 = (AT)(U[(rb + 0) * ld + s] - ua0);
    const AT d1 = (AT)(U[(rb + 1) * ld + s] - ua1);
    const AT d2 = (AT)(U[(rb + 2) * ld + s] - ua2);
    const AT d3 = (AT)(U[(rc + 0) * ld + s] - ua0);
    const AT d4 = (AT)(U[(rc + 1) * ld + s] - ua1);
    const AT d5 = (AT)(U[(rc + 2) * ld + s] - ua2);
    const AT f0 = kk[0] * d0 + kk[1] * d1 + kk[2] * d2 + kk[3] * d3 + kk[4] * d4 + kk[5] * d5;
    const AT f1 = kk[6] * d0 + kk[7] * d1 + kk[8] * d2 + kk[9] * d3 + kk[10] * d4 + kk[11] * d5;
    const AT f2 = kk[12] * d0 + kk[13] * d1 + kk[14] * d2 + kk[15] * d3 + kk[16] * d4 + kk[17] * d5;
    r0 += eh * f0;
    r1 += eh * f1;
    r2 += eh * f2;
  }
}

template <typename AT, int MODE, int SB, bool QOI, bool ENERGY>
__global__ __launch_bounds__(kBlock) void k_step(StepArgs p) {
  constexpr int NPB = kBlock / SB;
  int nb, sbk;
  if (!wg_coords<SB>(p, nb, sbk)) return;  // uniform over the workgroup
  const int ln = threadIdx.x / SB;
  const int ls = threadIdx.x % SB;
  int node = nb * NPB + ln;
  if (SB >= 64) node = __builtin_amdgcn_readfirstlane(node);
  const int s = sbk * SB + ls;
  const int64_t ld = p.ld;
  const bool active = node < p.n_nodes;
  double e_loc = 0.0;
  if (active) {
    using ST = typename std::conditional<MODE == kStateF64, double, float>::type;
    const ST* __restrict__ U = nullptr;
    if constexpr (MODE == kStateF64) U = p.u_cur; else U = p.uh_cur;
    const int64_t row = (int64_t)node * 3;
    const ST ua0 = U[(row + 0) * ld + s];
    const ST ua1 = U[(row + 1) * ld + s];
    const ST ua2 = U[(row + 2) * ld + s];
    AT r0, r1, r2;
    gather_apply<AT, ST>(p, node, ld, s, U, ua0, ua1, ua2, r0, r1, r2);

    const double g = p.gtab[p.j];
    const unsigned fx = p.fixed[node];
    const int64_t ms = (int64_t)node * ld + s;
    double un[3];
    if constexpr (MODE == kStateF64) {
      const double minv = std::is_same<AT, double>::value
                              ? static_cast<const double*>(p.minv)[ms]
                              : (double)static_cast<const float*>(p.minv)[ms];
      const double dt2m = p.dt * p.dt * minv;
      const double inv1pa = 1.0 / (1.0 + p.a);
      const double oma = 1.0 - p.a;
      const double ua[3] = {ua0, ua1, ua2};
      const double rr[3] = {(double)r0, (double)r1, (double)r2};
#pragma unroll
      for (int c = 0; c < 3; ++c) {
        const int64_t idx = (row + c) * ld + s;
        const double up = p.u_prev[idx];
        double v = (dt2m * (g * p.F[row + c] - rr[c]) + 2.0 * ua[c] - oma * up) * inv1pa;
        if (fx & (1u << c)) v = 0.0;
        p.u_next[idx] = v;
        un[c] = v;
      }
      if constexpr (ENERGY) {
        const double m = 1.0 / minv;
#pragma unroll
        for (int c = 0; c < 3; ++c) {
          const double vel = (un[c] - ua[c]) / p.dt;
          e_loc += 0.5 * m * vel * vel + 0.5 * un[c] * rr[c];
        }
      }
    } else {
      const float minv = static_cast<const float*>(p.minv)[ms];
      const float dtf = (float)p.dt;
      const float inv1pa = (float)(1.0 / (1.0 + p.a));
      const float oma = (float)(1.0 - p.a);
      const float ua[3] = {ua0, ua1, ua2};
      const float rr[3] = {(float)r0, (float)r1, (float)r2};
#pragma unroll
      for (int c = 0; c < 3; ++c) {
        const int64_t idx = (row + c) * ld + s;
        const float acc = minv * ((float)(g * p.F[row + c]) - rr[c]);
        float vel = (oma * p.v[idx] + dtf * acc) * inv1pa;
        float uh = ua[c];
        float cc = 0.0f;
        if constexpr (MODE == kStateF32Kahan) {
          cc = p.uc[idx];
          const float y = dtf * vel - cc;
          const float t = uh + y;
          cc = (t - uh) - y;
          uh = t;
        } else {
          uh = uh + dtf * vel;
        }
        if (fx & (1u << c)) {
          uh = 0.0f;
          cc = 0.0f;
          vel = 0.0f;
        }
        p.uh_next[idx] = uh;
        if constexpr (MODE == kStateF32Kahan) p.uc[idx] = cc;
        p.v[idx] = vel;
        un[c] = (double)uh - (double)cc;
        if constexpr (ENERGY) {
          e_loc += 0.5 / (double)minv * (double)vel * (double)vel + 0.5 * un[c] * (double)rr[c];
        }
      }
    }
    if constexpr (QOI) {
      const double qv = p.radial[row + 0] * un[0] + p.radial[row + 1] * un[1] +
                        p.radial[row + 2] * un[2];
      const double qo = p.q[ms];
      if (qv > qo) p.q[ms] = qv;
    }
  }
  if constexpr (ENERGY) {
    __shared__ double red[kBlock];
    red[threadIdx.x] = e_loc;
    __syncthreads();
    if (ln == 0) {
      double sum = 0.0;
      for (int i = 0; i < NPB; ++i) sum += red[i * SB + ls];
      p.energy_part[(int64_t)nb * ld + s] = sum;
    }
  }
}

template <typename AT, int SB>
__global__ __launch_bounds__(kBlock) void k_apply(StepArgs p, const AT* __restrict__ U,
                                                  AT* __restrict__ R) {
  constexpr int NPB = kBlock / SB;
  int nb, sbk;
  if (!wg_coords<SB>(p, nb, sbk)) return;
  int node = nb * NPB + (int)(threadIdx.x / SB);
  if (SB >= 64) node = __builtin_amdgcn_readfirstlane(node);
  if (node >= p.n_nodes) return;
  const int s = sbk * SB + (int)(threadIdx.x % SB);
  const int64_t ld = p.ld;
  const int64_t row = (int64_t)node * 3;
  AT r0, r1, r2;
  gather_apply<AT, AT>(p, node, ld, s, U, U[(row + 0) * ld + s], U[(row + 1) * ld + s],
                       U[(row + 2) * ld + s], r0, r1, r2);
  R[(row + 0) * ld + s] = r0;
  R[(row + 1) * ld + s] = r1;
  R[(row + 2) * ld + s] = r2;
}

__device__ double load_factor(const Schedule& sc, double t) {
  if (sc.kind == 0) return 1.0;
  const double ramp = (t < sc.t_ramp) ? sin(M_PI * t / (2.0 * sc.t_ramp)) : 1.0;
  if (sc.kind == 1) return ramp;
  return ramp * (1.0 + sc.amp * sin(2.0 * M_PI * t / sc.period));
}

__global__ __launch_bounds__(256) void k_schedule(double* __restrict__ gtab,
                                                  const int64_t* __restrict__ base, int32_t k,
                                                  double dt, Schedule sc) {
  const int64_t n0 = *base;
  for (int j = threadIdx.x; j < k; j += 256) gtab[j] = load_factor(sc, (double)(n0 + j) * dt);
}

__global__ void k_advance(int64_t* base, int32_t k) {
  if (threadIdx.x == 0 && blockIdx.x == 0) *base += k;
}

// Energy: partials [n_nb][ld] -> one row [S]; fixed summation order.
__global__ __launch_bounds__(64) void k_energy_reduce1(const double* __restrict__ part,
                                                       int32_t n_nb, int32_t ld, int32_t chunks,
                                                       double* __restrict__ tmp) {
  const int s = blockIdx.x * 64 + threadIdx.x;
  const int ch = blockIdx.y;
  if (s >= ld) return;
  const int per = (n_nb + chunks - 1) / chunks;
  const int b0 = ch * per, b1 = min(n_nb, b0 + per);
  double sum = 0.0;
  for (int b = b0; b < b1; ++b) sum += part[(int64_t)b * ld + s];
  tmp[(int64_t)ch * ld + s] = sum;
}

__global__ __launch_bounds__(64) void k_energy_reduce2(const double* __restrict__ tmp,
                                                       int32_t chunks, int32_t ld, int32_t S,
                                                       double* __restrict__ out) {
  const int s = blockIdx.x * 64 + threadIdx.x;
  if (s >= S) return;
  double sum = 0.0;
  for (int c = 0; c < chunks; ++c) sum += tmp[(int64_t)c * ld + s];
  out[s] = sum;
}

// Taylor starter, FP64 two-level state: on entry vprev_io holds v_0; on
// exit u_{-1} = u_0 - dt v_0 + dt^2/2 (m^-1 (g_0 F - K u_0) - alpha v_0).
__global__ __launch_bounds__(256) void k_starter_f64(int32_t n_nodes, int32_t ld,
                                                     const double* __restrict__ R,
                                                     const double* __restrict__ minv,
                                                     const double* __restrict__ F,
                                                     const uint8_t* __restrict__ fixed,
                                                     const double* __restrict__ u0,
                                                     double* __restrict__ vprev,
                                                     const double* __restrict__ gtab, double dt,
                                                     double alpha) {
  const int64_t t = (int64_t)blockIdx.x * 256 + threadIdx.x;
  if (t >= (int64_t)n_nodes * 3 * ld) return;
  const int64_t row = t / ld;
  const int s = (int)(t % ld);
  const int64_t node = row / 3;
  const int c = (int)(row % 3);
  const double v0 = vprev[t];
  const double acc = minv[node * ld + s] * (gtab[0] * F[row] - R[t]) - alpha * v0;
  double um = u0[t] - dt * v0 + 0.5 * dt * dt * acc;
  if (fixed[node] & (1u << c)) um = 0.0;
  vprev[t] = um;
}

// Starter in velocity form: v_{-1/2} = v_0 - dt/2 (m^-1 (g_0 F - K u_0) - alpha v_0).
__global__ __launch_bounds__(256) void k_starter_f32(int32_t n_nodes, int32_t ld,
                                                     const float* __restrict__ R,
                                                     const float* __restrict__ minv,
                                                     const double* __restrict__ F,
                                                     const uint8_t* __restrict__ fixed,
                                                     float* __restrict__ v,
                                                     const double* __restrict__ gtab, double dt,
                                                     double alpha) {
  const int64_t t = (int64_t)blockIdx.x * 256 + threadIdx.x;
  if (t >= (int64_t)n_nodes * 3 * ld) return;
  const int64_t row = t / ld;
  const int s = (int)(t % ld);
  const int64_t node = row / 3;
  const int c = (int)(row % 3);
  const double v0 = (double)v[t];
  const double acc = (double)minv[node * ld + s] * (gtab[0] * F[row] - (double)R[t]) - alpha * v0;
  float vm = (float)(v0 - 0.5 * dt * acc);
  if (fixed[node] & (1u << c)) vm = 0.0f;
  v[t] = vm;
}

__global__ __launch_bounds__(256) void k_split_f32(int64_t n, const double* __restrict__ u0,
                                                   float* __restrict__ uh, float* __restrict__ uc) {
  const int64_t t = (int64_t)blockIdx.x * 256 + threadIdx.x;
  if (t >= n) return;
  const float h = (float)u0[t];
  uh[t] = h;
  if (uc) uc[t] = (float)((double)h - u0[t]);  // Kahan convention: u = uh - uc
}

__global__ __launch_bounds__(256) void k_qoi_init(int32_t n_nodes, int32_t ld,
                                                  const double* __restrict__ radial,
                                                  const double* __restrict__ u,
                                                  const float* __restrict__ uh,
                                                  const float* __restrict__ uc,
                                                  double* __restrict__ q) {
  const int64_t t = (int64_t)blockIdx.x * 256 + threadIdx.x;
  if (t >= (int64_t)n_nodes * ld) return;
  const int64_t node = t / ld;
  const int s = (int)(t % ld);
  double acc = 0.0;
  for (int c = 0; c < 3; ++c) {
    const int64_t idx = (node * 3 + c) * ld + s;
    double x;
    if (u) x = u[idx];
    else x = (double)uh[idx] - (uc ? (double)uc[idx] : 0.0);
    acc += radial[node * 3 + c] * x;
  }
  q[t] = acc;
}

__global__ __launch_bounds__(256) void k_combine_f32(int64_t n, const float* __restrict__ uh,
                                                     const float* __restrict__ uc,
                                                     double* __restrict__ out) {
  const int64_t t = (int64_t)blockIdx.x * 256 + threadIdx.x;
  if (t >= n) return;
  out[t] = (double)uh[t] - (uc ? (double)uc[t] : 0.0);
}

// Per-node mean and unbiased variance over the S real samples: one 64-lane
// wave per node, fixed lane-strided order then a fixed butterfly.
__global__ __launch_bounds__(64) void k_moments(int32_t n_nodes, int32_t ld, int32_t S,
                                                const double* __restrict__ q,
                                                double* __restrict__ mean,
                                                double* __restrict__ var) {
  const int node = blockIdx.x;
  if (node >= n_nodes) return;
  const double* row = q + (int64_t)node * ld;
  double sum = 0.0;
  for (int s = threadIdx.x; s < S; s += 64) sum += row[s];
  for (int o = 32; o > 0; o >>= 1) sum += __shfl_xor(sum, o, 64);
  const double mu = sum / S;
  double ss = 0.0;
  for (int s = threadIdx.x; s < S; s += 64) {
    const double d = row[s] - mu;
    ss += d * d;
  }
  for (int o = 32; o > 0; o >>= 1) ss += __shfl_xor(ss, o, 64);
  if (threadIdx.x == 0) {
    mean[node] = mu;
    var[node] = S > 1 ? ss / (S - 1) : 0.0;
  }
}

__global__ __launch_bounds__(256) void k_check_finite(int64_t n, const void* __restrict__ x,
                                                      int is_f32, int32_t* __restrict__ flag) {
  int bad = 0;
  for (int64_t t = (int64_t)blockIdx.x * 256 + threadIdx.x; t < n;
       t += (int64_t)gridDim.x * 256) {
    const double v = is_f32 ? (double)static_cast<const float*>(x)[t]
                            : static_cast<const double*>(x)[t];
    if (!isfinite(v)) bad = 1;
  }
  if (bad) atomicOr(flag, 1);
}

inline unsigned grid_for(int64_t n, int per) { return (unsigned)((n + per - 1) / per); }

inline unsigned step_grid(const StepArgs& a) {
  const int64_t n = (int64_t)a.n_nb * a.n_sb;
  return (unsigned)(((n + 7) / 8) * 8);
}

template <typename AT, int MODE, int SB>
hipError_t dispatch_flags(const StepArgs& a, bool qoi, bool energy, hipStream_t st) {
  const unsigned g = step_grid(a);
  if (qoi && energy) k_step<AT, MODE, SB, true, true><<<g, kBlock, 0, st>>>(a);
  else if (qoi) k_step<AT, MODE, SB, true, false><<<g, kBlock, 0, st>>>(a);
  else if (energy) k_step<AT, MODE, SB, false, true><<<g, kBlock, 0, st>>>(a);
  else k_step<AT, MODE, SB, false, false><<<g, kBlock, 0, st>>>(a);
  return hipGetLastError();
}

template <typename AT, int MODE>
hipError_t dispatch_sb(const StepArgs& a, int sb, bool qoi, bool energy, hipStream_t st) {
  switch (sb) {
    case 8: return dispatch_flags<AT, MODE, 8>(a, qoi, energy, st);
    case 16: return dispatch_flags<AT, MODE, 16>(a, qoi, energy, st);
    case 32: return dispatch_flags<AT, MODE, 32>(a, qoi, energy, st);
    case 64: return dispatch_flags<AT, MODE, 64>(a, qoi, energy, st);
    default: return hipErrorInvalidValue;
  }
}

template <typename AT>
hipError_t dispatch_apply(const StepArgs& a, int sb, const void* U, void* R, hipStream_t st) {
  const unsigned g = step_grid(a);
  const AT* u = static_cast<const AT*>(U);
  AT* r = static_cast<AT*>(R);
  switch (sb) {
    case 8: k_apply<AT, 8><<<g, kBlock, 0, st>>>(a, u, r); break;
    case 16: k_apply<AT, 16><<<g, kBlock, 0, st>>>(a, u, r); break;
    case 32: k_apply<AT, 32><<<g, kBlock, 0, st>>>(a, u, r); break;
    case 64: k_apply<AT, 64><<<g, kBlock, 0, st>>>(a, u, r); break;
    default: return hipErrorInvalidValue;
  }
  return hipGetLastError();
}

}  // namespace

hipError_t launch_step(const StepArgs& a, bool apply_f32, int mode, int sample_block, bool qoi,
                       bool energy, hipStream_t st) {
  if (a.n_nb == 0 || a.n_sb == 0) return hipSuccess;
  if (!apply_f32) {
    if (mode != kStateF64) return hipErrorInvalidValue;
    return dispatch_sb<double, kStateF64>(a, sample_block, qoi, energy, st);
  }
  switch (mode) {
    case kStateF64: return dispatch_sb<float, kStateF64>(a, sample_block, qoi, energy, st);
    case kStateF32Kahan: return dispatch_sb<float, kStateF32Kahan>(a, sample_block, qoi, energy, st);
    case kStateF32: return dispatch_sb<float, kStateF32>(a, sample_block, qoi, energy, st);
    default: return hipErrorInvalidValue;
  }
}

hipError_t launch_apply(const StepArgs& a, bool f32, int sample_block, const void* U, void* R,
                        hipStream_t st) {
  if (a.n_nb == 0 || a.n_sb == 0) return hipSuccess;
  return f32 ? dispatch_apply<float>(a, sample_block, U, R, st)
             : dispatch_apply<double>(a, sample_block, U, R, st);
}

hipError_t launch_schedule(double* gtab, int64_t* base, int32_t k, double dt, Schedule s,
                           hipStream_t st) {
  k_schedule<<<1, 256, 0, st>>>(gtab, base, k, dt, s);
  return hipGetLastError();
}

hipError_t launch_advance(int64_t* base, int32_t k, hipStream_t st) {
  k_advance<<<1, 64, 0, st>>>(base, k);
  return hipGetLastError();
}

hipError_t launch_energy_reduce(const double* part, int32_t n_nb, int32_t ld, int32_t S,
                                double* out_row, hipStream_t st) {
  // second-level buffer lives right after the [n_nb][ld] partials
  const int chunks = 256;
  double* tmp = const_cast<double*>(part) + (int64_t)n_nb * ld;
  dim3 g1(grid_for(ld, 64), chunks);
  k_energy_reduce1<<<g1, 64, 0, st>>>(part, n_nb, ld, chunks, tmp);
  k_energy_reduce2<<<grid_for(S, 64), 64, 0, st>>>(tmp, chunks, ld, S, out_row);
  return hipGetLastError();
}

hipError_t launch_starter_f64(int32_t n_nodes, int32_t ld, const double* R, const double* minv,
                              const double* F, const uint8_t* fixed, const double* u0,
                              double* vprev_io, const double* gtab, double dt, double alpha,
                              hipStream_t st) {
  const int64_t n = (int64_t)n_nodes * 3 * ld;
  if (n == 0) return hipSuccess;
  k_starter_f64<<<grid_for(n, 256), 256, 0, st>>>(n_nodes, ld, R, minv, F, fixed, u0, vprev_io,
                                                   gtab, dt, alpha);
  return hipGetLastError();
}

hipError_t launch_starter_f32(int32_t n_nodes, int32_t ld, const float* R, const float* minv,
                              const double* F, const uint8_t* fixed, float* v_io,
                              const double* gtab, double dt, double alpha, hipStream_t st) {
  const int64_t n = (int64_t)n_nodes * 3 * ld;
  if (n == 0) return hipSuccess;
  k_starter_f32<<<grid_for(n, 256), 256, 0, st>>>(n_nodes, ld, R, minv, F, fixed, v_io, gtab, dt,
                                                   alpha);
  return hipGetLastError();
}

hipError_t launch_split_f32(int64_t n, const double* u0, float* uh, float* uc, hipStream_t st) {
  if (n == 0) return hipSuccess;
  k_split_f32<<<grid_for(n, 256), 256, 0, st>>>(n, u0, uh, uc);
  return hipGetLastError();
}

hipError_t launch_qoi_init(int32_t n_nodes, int32_t ld, const double* radial, const double* u_f64,
                           const float* uh, const float* uc, double* q, hipStream_t st) {
  const int64_t n = (int64_t)n_nodes * ld;
  if (n == 0) return hipSuccess;
  k_qoi_init<<<grid_for(n, 256), 256, 0, st>>>(n_nodes, ld, radial, u_f64, uh, uc, q);
  return hipGetLastError();
}

hipError_t launch_combine_f32(int64_t n, const float* uh, const float* uc, double* out,
                              hipStream_t st) {
  if (n == 0) return hipSuccess;
  k_combine_f32<<<grid_for(n, 256), 256, 0, st>>>(n, uh, uc, out);
  return hipGetLastError();
}

hipError_t launch_moments(int32_t n_nodes, int32_t ld, int32_t S, const double* q, double* mean,
                          double* var, hipStream_t st) {
  if (n_nodes == 0) return hipSuccess;
  k_moments<<<n_nodes, 64, 0, st>>>(n_nodes, ld, S, q, mean, var);
  return hipGetLastError();
}

hipError_t launch_check_finite(int64_t n, const void* x, int is_f32, int32_t* flag,
                               hipStream_t st) {
  if (n == 0) return hipSuccess;
  const int64_t blocks = std::min<int64_t>(grid_for(n, 256), 4096);
  k_check_finite<<<(unsigned)blocks, 256, 0, st>>>(n, x, is_f32, flag);
  return hipGetLastError();
}

}  // namespace ensfem
