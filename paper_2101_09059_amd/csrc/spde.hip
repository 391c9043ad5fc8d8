// SPDE / GMRF sampler of Matern fields on the wall mesh (Sec. 2.1):
// x = K^-1 C~^(1/2) z, K = kappa^2 C~ + G, by block conjugate gradients
// over S right-hand sides with a diagonal preconditioner.
//
// Block vectors are [n][ld] with samples fastest (ld = S rounded up to 64).
// A wave owns one matrix row for 64 * SPL samples (SPL consecutive samples
// per lane, SPL = 4, 2 or 1 as ld allows), so the row's column indices and
// values are wave-uniform (scalar loads) and each neighbour load moves
// 512 * SPL contiguous bytes.  The matrix is stored as padded rows (ELL) of
// width W, a multiple of 8: a row's neighbour loads are issued 8 at a time,
// for two rows at once in the product.
//
// Every per-sample scalar of CG (r.z, p.q, r.r) is reduced in a fixed
// order: per-workgroup partials, then one pass over the partials per
// column, so a run is reproducible bit for bit.
#include "ensfem_spde.h"
#include "ensfem.h"

#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <cstring>
#include <new>
#include <string>
#include <vector>

namespace {

constexpr int kRowsWG = 4;      // waves (rows in flight) per workgroup
constexpr int kPartWG = 512;    // most workgroups along the rows (reduction partials)
constexpr int kEllChunk = 8;    // ELL width granularity (loads in flight per row)
constexpr int kRowsWave = 2;    // rows a wave of the product works on at once

// Rows of this wave: r0, r0 + step, ... below n.
struct Rows {
  int64_t r0, step;
};
__device__ __forceinline__ Rows wave_rows() {
  return {(int64_t)blockIdx.x * kRowsWG + threadIdx.x / 64, (int64_t)gridDim.x * kRowsWG};
}

__device__ __forceinline__ int64_t uniform(int64_t row) {
  return (int64_t)__builtin_amdgcn_readfirstlane((int)row);
}

// SPL consecutive doubles of one lane (16-byte aligned for SPL >= 2).
template <int SPL>
struct Lane {
  double v[SPL];
  __device__ __forceinline__ void load(const double* p) {
    if constexpr (SPL == 1) {
      v[0] = *p;
    } else {
#pragma unroll
      for (int k = 0; k < SPL; k += 2) {
        const double2 t = *reinterpret_cast<const double2*>(p + k);
        v[k] = t.x;
        v[k + 1] = t.y;
      }
    }
  }
  __device__ __forceinline__ void store(double* p) const {
    if constexpr (SPL == 1) {
      *p = v[0];
    } else {
#pragma unroll
      for (int k = 0; k < SPL; k += 2) *reinterpret_cast<double2*>(p + k) = make_double2(v[k], v[k + 1]);
    }
  }
};

// Partial sums of up to two per-column quantities over the rows a
// workgroup visits: its 4 waves added in order; one value per column.
template <int SPL>
__device__ __forceinline__ void block_partials(const double (&a)[SPL], const double (&b)[SPL], int lane,
                                               double* __restrict__ part_a, double* __restrict__ part_b,
                                               int64_t col, int32_t ld) {
  __shared__ double ra[256 * SPL], rb[256 * SPL];
#pragma unroll
  for (int k = 0; k < SPL; ++k) {
    ra[threadIdx.x * SPL + k] = a[k];
    rb[threadIdx.x * SPL + k] = b[k];
  }
  __syncthreads();
  if (threadIdx.x < 64) {
#pragma unroll
    for (int k = 0; k < SPL; ++k) {
      double sa = ra[lane * SPL + k], sb = rb[lane * SPL + k];
      for (int w = 1; w < kRowsWG; ++w) {
        sa += ra[(64 * w + lane) * SPL + k];
        sb += rb[(64 * w + lane) * SPL + k];
      }
      part_a[(int64_t)blockIdx.x * ld + col + k] = sa;
      if (part_b) part_b[(int64_t)blockIdx.x * ld + col + k] = sb;
    }
  }
}

template <int SPL>
__device__ __forceinline__ int64_t lane_col(int lane) {
  return ((int64_t)blockIdx.y * 64 + lane) * SPL;
}

// r = sqrt(C~) z, x = 0, p = D^-1 r; partials of r.D^-1.r and r.r.
template <int SPL>
__global__ __launch_bounds__(256) void k_init(int64_t n, int32_t ld, const double* __restrict__ sqrtc,
                                              const double* __restrict__ dinv, const double* __restrict__ z,
                                              double* __restrict__ X, double* __restrict__ R,
                                              double* __restrict__ P, double* __restrict__ part_rz,
                                              double* __restrict__ part_rr) {
  const int lane = threadIdx.x % 64;
  const int64_t col = lane_col<SPL>(lane);
  double rz[SPL] = {}, rr[SPL] = {};
  const Rows w = wave_rows();
  for (int64_t row = w.r0; row < n; row += w.step) {
    const int64_t r = uniform(row);
    const int64_t i = r * ld + col;
    Lane<SPL> zz, x, rv, pv;
    zz.load(z + i);
#pragma unroll
    for (int k = 0; k < SPL; ++k) {
      const double v = sqrtc[r] * zz.v[k];
      x.v[k] = 0.0;
      rv.v[k] = v;
      pv.v[k] = dinv[r] * v;
      rz[k] = fma(v, pv.v[k], rz[k]);
      rr[k] = fma(v, v, rr[k]);
    }
    x.store(X + i);
    rv.store(R + i);
    pv.store(P + i);
  }
  block_partials<SPL>(rz, rr, lane, part_rz, part_rr, col, ld);
}

// Q = K P (ELL rows, kRowsWave rows per wave at once); partials of p.q.
template <int SPL>
__global__ __launch_bounds__(256) void k_spmv(int64_t n, int32_t ld, int32_t W, const int32_t* __restrict__ ecol,
                                              const double* __restrict__ eval, const double* __restrict__ P,
                                              double* __restrict__ Q, double* __restrict__ part_pq) {
  const int lane = threadIdx.x % 64;
  const int64_t col = lane_col<SPL>(lane);
  double pq[SPL] = {}, zero[SPL] = {};
  const Rows w = wave_rows();
  for (int64_t row = w.r0; row < n; row += kRowsWave * w.step) {
    int64_t r[kRowsWave];
#pragma unroll
    for (int m = 0; m < kRowsWave; ++m) {
      const int64_t rm = row + m * w.step;
      r[m] = uniform(rm < n ? rm : row);  // a row past the end repeats the first (not stored)
    }
    double q[kRowsWave][SPL] = {};
    for (int c0 = 0; c0 < W; c0 += kEllChunk) {
      Lane<SPL> pj[kRowsWave][kEllChunk];
#pragma unroll
      for (int m = 0; m < kRowsWave; ++m)
#pragma unroll
        for (int u = 0; u < kEllChunk; ++u) pj[m][u].load(P + (int64_t)ecol[r[m] * W + c0 + u] * ld + col);
#pragma unroll
      for (int m = 0; m < kRowsWave; ++m)
#pragma unroll
        for (int u = 0; u < kEllChunk; ++u) {
          const double a = eval[r[m] * W + c0 + u];
#pragma unroll
          for (int k = 0; k < SPL; ++k) q[m][k] = fma(a, pj[m][u].v[k], q[m][k]);
        }
    }
#pragma unroll
    for (int m = 0; m < kRowsWave; ++m) {
      if (row + m * w.step < n) {
        const int64_t i = r[m] * ld + col;
        Lane<SPL> pv, qv;
        pv.load(P + i);
#pragma unroll
        for (int k = 0; k < SPL; ++k) {
          qv.v[k] = q[m][k];
          pq[k] = fma(pv.v[k], q[m][k], pq[k]);
        }
        qv.store(Q + i);
      }
    }
  }
  block_partials<SPL>(pq, zero, lane, part_pq, nullptr, col, ld);
}

// Column sums of one or two partial arrays [nparts][ld] -> out [ld]: a
// workgroup takes 64 columns, its kColWaves waves sum every kColWaves-th
// partial row (in order) and their results are added in wave order.
constexpr int kColWaves = 16;

__global__ __launch_bounds__(64 * kColWaves) void k_colsum(int32_t ld, int32_t nparts,
                                                           const double* __restrict__ part_a,
                                                           double* __restrict__ out_a,
                                                           const double* __restrict__ part_b,
                                                           double* __restrict__ out_b) {
  __shared__ double ra[64 * kColWaves], rb[64 * kColWaves];
  const int lane = threadIdx.x % 64, g = threadIdx.x / 64;
  const int64_t c = (int64_t)blockIdx.x * 64 + lane;
  double sa = 0.0, sb = 0.0;
#pragma unroll 4
  for (int b = g; b < nparts; b += kColWaves) {
    sa += part_a[(int64_t)b * ld + c];
    if (part_b) sb += part_b[(int64_t)b * ld + c];
  }
  ra[threadIdx.x] = sa;
  rb[threadIdx.x] = sb;
  __syncthreads();
  if (g == 0) {
    for (int w = 1; w < kColWaves; ++w) {
      sa += ra[64 * w + lane];
      sb += rb[64 * w + lane];
    }
    out_a[c] = sa;
    if (part_b) out_b[c] = sb;
  }
}

// alpha = rz / pq; x += alpha p; r -= alpha q; partials of r.D^-1.r, r.r.
template <int SPL>
__global__ __launch_bounds__(256) void k_update_xr(int64_t n, int32_t ld, const double* __restrict__ dinv,
                                                   const double* __restrict__ rz, const double* __restrict__ pq,
                                                   double* __restrict__ X, double* __restrict__ R,
                                                   const double* __restrict__ P, const double* __restrict__ Q,
                                                   double* __restrict__ part_rz, double* __restrict__ part_rr) {
  const int lane = threadIdx.x % 64;
  const int64_t col = lane_col<SPL>(lane);
  double alpha[SPL], srz[SPL] = {}, srr[SPL] = {};
#pragma unroll
  for (int k = 0; k < SPL; ++k) alpha[k] = pq[col + k] > 0.0 ? rz[col + k] / pq[col + k] : 0.0;
  const Rows w = wave_rows();
  for (int64_t row = w.r0; row < n; row += w.step) {
    const int64_t r = uniform(row);
    const int64_t i = r * ld + col;
    Lane<SPL> x, pv, qv, rv;
    x.load(X + i);
    pv.load(P + i);
    qv.load(Q + i);
    rv.load(R + i);
#pragma unroll
    for (int k = 0; k < SPL; ++k) {
      x.v[k] = fma(alpha[k], pv.v[k], x.v[k]);
      const double v = fma(-alpha[k], qv.v[k], rv.v[k]);
      rv.v[k] = v;
      srz[k] = fma(v, dinv[r] * v, srz[k]);
      srr[k] = fma(v, v, srr[k]);
    }
    x.store(X + i);
    rv.store(R + i);
  }
  block_partials<SPL>(srz, srr, lane, part_rz, part_rr, col, ld);
}

// beta = rz_new / rz_old; p = D^-1 r + beta p.
template <int SPL>
__global__ __launch_bounds__(256) void k_update_p(int64_t n, int32_t ld, const double* __restrict__ dinv,
                                                  const double* __restrict__ rz_new,
                                                  const double* __restrict__ rz_old, const double* __restrict__ R,
                                                  double* __restrict__ P) {
  const int lane = threadIdx.x % 64;
  const int64_t col = lane_col<SPL>(lane);
  double beta[SPL];
#pragma unroll
  for (int k = 0; k < SPL; ++k) beta[k] = rz_old[col + k] > 0.0 ? rz_new[col + k] / rz_old[col + k] : 0.0;
  const Rows w = wave_rows();
  for (int64_t row = w.r0; row < n; row += w.step) {
    const int64_t r = uniform(row);
    const int64_t i = r * ld + col;
    Lane<SPL> pv, rv;
    pv.load(P + i);
    rv.load(R + i);
#pragma unroll
    for (int k = 0; k < SPL; ++k) pv.v[k] = fma(beta[k], pv.v[k], dinv[r] * rv.v[k]);
    pv.store(P + i);
  }
}

// One CG solve on the bound workspace with SPL samples per lane.
struct Solve {
  int64_t n;
  int32_t ld, W, S;
  const int32_t* ecol;
  const double *eval, *dinv, *sqrtc, *z;
  double *X, *R, *P, *Q, *pa, *pb, *rz, *rz2, *rr, *pq, *bb;
};

template <int SPL>
hipError_t cg(const Solve& v, double tol, int32_t max_iter, int& it, double& worst) {
  const dim3 grid((unsigned)std::min<int64_t>(kPartWG, (v.n + kRowsWG - 1) / kRowsWG),
                  (unsigned)(v.ld / (64 * SPL)));
  const int nparts = (int)grid.x;
  const unsigned cgrid = (unsigned)(v.ld / 64);
  double *rz = v.rz, *rz2 = v.rz2;
  k_init<SPL><<<grid, 256>>>(v.n, v.ld, v.sqrtc, v.dinv, v.z, v.X, v.R, v.P, v.pa, v.pb);
  k_colsum<<<cgrid, 64 * kColWaves>>>(v.ld, nparts, v.pa, rz, v.pb, v.bb);
  hipError_t e = hipGetLastError();
  if (e != hipSuccess) return e;
  std::vector<double> hbb(v.ld), hrr(v.ld);
  if ((e = hipMemcpy(hbb.data(), v.bb, 8 * (size_t)v.ld, hipMemcpyDeviceToHost)) != hipSuccess) return e;
  it = 0;
  auto converged = [&](const std::vector<double>& r2) {
    worst = 0.0;
    for (int c = 0; c < v.S; ++c) {
      const double rel = hbb[c] > 0.0 ? std::sqrt(r2[c] / hbb[c]) : 0.0;
      worst = std::max(worst, rel);
    }
    return worst <= tol;
  };
  if (converged(hbb)) return hipSuccess;
  while (it < max_iter) {
    k_spmv<SPL><<<grid, 256>>>(v.n, v.ld, v.W, v.ecol, v.eval, v.P, v.Q, v.pa);
    k_colsum<<<cgrid, 64 * kColWaves>>>(v.ld, nparts, v.pa, v.pq, nullptr, nullptr);
    k_update_xr<SPL><<<grid, 256>>>(v.n, v.ld, v.dinv, rz, v.pq, v.X, v.R, v.P, v.Q, v.pa, v.pb);
    k_colsum<<<cgrid, 64 * kColWaves>>>(v.ld, nparts, v.pa, rz2, v.pb, v.rr);
    k_update_p<SPL><<<grid, 256>>>(v.n, v.ld, v.dinv, rz2, rz, v.R, v.P);
    if ((e = hipGetLastError()) != hipSuccess) return e;
    std::swap(rz, rz2);
    ++it;
    if (it % 8 == 0 || it == max_iter) {
      if ((e = hipMemcpy(hrr.data(), v.rr, 8 * (size_t)v.ld, hipMemcpyDeviceToHost)) != hipSuccess) return e;
      if (converged(hrr)) break;
    }
  }
  return hipSuccess;
}

inline size_t align256(size_t x) { return (x + 255) & ~(size_t)255; }

}  // namespace

struct spde_ctx {
  int device = 0;
  std::string err;
  int64_t n = 0;
  std::vector<int32_t> ptr, col;
  std::vector<double> g;  // G values in CSR order
  std::vector<int64_t> diag;  // position of (i, i) in CSR
  std::vector<double> cmass;  // lumped mass
  int32_t W = 0;                // ELL width (multiple of kEllChunk)
  std::vector<int32_t> ecol;    // [n][W] column of each slot (the row itself in padding)
  std::vector<int64_t> epos;    // [n][W] CSR position of each slot, -1 in padding
  bool have_mesh = false;
  // workspace
  char* ws = nullptr;
  int32_t S = 0, ld = 0;
  size_t o_col = 0, o_val = 0, o_dinv = 0, o_sqrtc = 0, o_z = 0, o_x = 0, o_r = 0, o_p = 0, o_q = 0,
         o_pa = 0, o_pb = 0, o_rz = 0, o_rz2 = 0, o_rr = 0, o_pq = 0, o_bb = 0, total = 0;
  bool bound = false;
  template <typename T>
  T* p(size_t off) const { return reinterpret_cast<T*>(ws + off); }
  int32_t fail(int32_t code, const std::string& m) {
    err = m;
    return code;
  }
};

namespace {

void plan(spde_ctx* s, int32_t S) {
  const int32_t ld = ((S + 63) / 64) * 64;
  const size_t n = (size_t)s->n, nnz = n * (size_t)s->W;
  size_t off = 0;
  auto take = [&](size_t b) {
    const size_t o = off;
    off = align256(off + b);
    return o;
  };
  s->o_col = take(4 * nnz);
  s->o_val = take(8 * nnz);
  s->o_dinv = take(8 * n);
  s->o_sqrtc = take(8 * n);
  s->o_z = take(8 * n * ld);
  s->o_x = take(8 * n * ld);
  s->o_r = take(8 * n * ld);
  s->o_p = take(8 * n * ld);
  s->o_q = take(8 * n * ld);
  s->o_pa = take(8 * (size_t)kPartWG * ld);
  s->o_pb = take(8 * (size_t)kPartWG * ld);
  s->o_rz = take(8 * ld);
  s->o_rz2 = take(8 * ld);
  s->o_rr = take(8 * ld);
  s->o_pq = take(8 * ld);
  s->o_bb = take(8 * ld);
  s->total = off;
  s->ld = ld;
}

#define SHIPC(expr)                                                   \
  do {                                                                \
    hipError_t e_ = (expr);                                           \
    if (e_ != hipSuccess) return s->fail(ENS_EDEVICE, hipGetErrorString(e_)); \
  } while (0)

}  // namespace

extern "C" {

int32_t spde_create(int32_t device, spde_ctx** out) {
  if (!out) return ENS_EINVAL;
  *out = nullptr;
  if (hipSetDevice(device) != hipSuccess) return ENS_EDEVICE;
  spde_ctx* s = new (std::nothrow) spde_ctx();
  if (!s) return ENS_EDEVICE;
  s->device = device;
  *out = s;
  return ENS_OK;
}

int32_t spde_destroy(spde_ctx* s) {
  if (!s) return ENS_EINVAL;
  delete s;
  return ENS_OK;
}

const char* spde_last_error(const spde_ctx* s) { return s ? s->err.c_str() : "null context"; }

int32_t spde_set_mesh(spde_ctx* s, int64_t n_nodes, const double* xyz, int64_t n_el, const int32_t* tri) {
  if (!s || !xyz || !tri || n_nodes < 1 || n_el < 1) return ENS_EINVAL;
  if (n_nodes > (int64_t)INT32_MAX) return s->fail(ENS_EINVAL, "spde_set_mesh: too many nodes");
  try {
    struct Trip {
      int32_t i, j;
      double v;
    };
    std::vector<Trip> t;
    t.reserve(9 * (size_t)n_el);
    std::vector<double> cm(n_nodes, 0.0);
    for (int64_t e = 0; e < n_el; ++e) {
      int32_t v[3];
      for (int a = 0; a < 3; ++a) {
        v[a] = tri[3 * e + a];
        if (v[a] < 0 || v[a] >= n_nodes)
          return s->fail(ENS_EINVAL, "spde_set_mesh: node index out of range in element " + std::to_string(e));
      }
      const double* p1 = xyz + 3 * (int64_t)v[0];
      const double* p2 = xyz + 3 * (int64_t)v[1];
      const double* p3 = xyz + 3 * (int64_t)v[2];
      double a[3], b[3];
      for (int c = 0; c < 3; ++c) {
        a[c] = p2[c] - p1[c];
        b[c] = p3[c] - p1[c];
      }
      const double la = std::sqrt(a[0] * a[0] + a[1] * a[1] + a[2] * a[2]);
      const double nz[3] = {a[1] * b[2] - a[2] * b[1], a[2] * b[0] - a[0] * b[2], a[0] * b[1] - a[1] * b[0]};
      const double ln = std::sqrt(nz[0] * nz[0] + nz[1] * nz[1] + nz[2] * nz[2]);
      if (!(la > 0.0) || !(ln > 0.0))
        return s->fail(ENS_EINVAL, "spde_set_mesh: degenerate element " + std::to_string(e));
      double ex[3], ez[3], ey[3];
      for (int c = 0; c < 3; ++c) {
        ex[c] = a[c] / la;
        ez[c] = nz[c] / ln;
      }
      ey[0] = ez[1] * ex[2] - ez[2] * ex[1];
      ey[1] = ez[2] * ex[0] - ez[0] * ex[2];
      ey[2] = ez[0] * ex[1] - ez[1] * ex[0];
      const double x2 = a[0] * ex[0] + a[1] * ex[1] + a[2] * ex[2];
      const double y2 = a[0] * ey[0] + a[1] * ey[1] + a[2] * ey[2];
      const double x3 = b[0] * ex[0] + b[1] * ex[1] + b[2] * ex[2];
      const double y3 = b[0] * ey[0] + b[1] * ey[1] + b[2] * ey[2];
      const double A = 0.5 * (x2 * y3 - x3 * y2);
      if (!(A > 0.0)) return s->fail(ENS_EINVAL, "spde_set_mesh: degenerate element " + std::to_string(e));
      const double inv2A = 1.0 / (2.0 * A);
      const double gx[3] = {(y2 - y3) * inv2A, y3 * inv2A, -y2 * inv2A};
      const double gy[3] = {(x3 - x2) * inv2A, -x3 * inv2A, x2 * inv2A};
      for (int i = 0; i < 3; ++i) {
        cm[v[i]] += A / 3.0;
        for (int j = 0; j < 3; ++j) t.push_back({v[i], v[j], A * (gx[i] * gx[j] + gy[i] * gy[j])});
      }
    }
    // CSR with duplicates summed in element order
    std::stable_sort(t.begin(), t.end(), [](const Trip& x, const Trip& y) {
      return x.i < y.i || (x.i == y.i && x.j < y.j);
    });
    s->ptr.assign(n_nodes + 1, 0);
    s->col.clear();
    s->g.clear();
    for (size_t k = 0; k < t.size();) {
      size_t m = k;
      double v = 0.0;
      while (m < t.size() && t[m].i == t[k].i && t[m].j == t[k].j) v += t[m++].v;
      s->col.push_back(t[k].j);
      s->g.push_back(v);
      s->ptr[t[k].i + 1]++;
      k = m;
    }
    for (int64_t i = 0; i < n_nodes; ++i) s->ptr[i + 1] += s->ptr[i];
    s->diag.assign(n_nodes, -1);
    for (int64_t i = 0; i < n_nodes; ++i)
      for (int32_t k = s->ptr[i]; k < s->ptr[i + 1]; ++k)
        if (s->col[k] == i) s->diag[i] = k;
    for (int64_t i = 0; i < n_nodes; ++i)
      if (s->diag[i] < 0) return s->fail(ENS_EINVAL, "spde_set_mesh: node " + std::to_string(i) + " is in no element");
    int32_t wmax = 0;
    for (int64_t i = 0; i < n_nodes; ++i) wmax = std::max(wmax, s->ptr[i + 1] - s->ptr[i]);
    s->W = (wmax + kEllChunk - 1) / kEllChunk * kEllChunk;
    s->ecol.assign((size_t)n_nodes * s->W, 0);
    s->epos.assign((size_t)n_nodes * s->W, -1);
    for (int64_t i = 0; i < n_nodes; ++i) {
      const int32_t len = s->ptr[i + 1] - s->ptr[i];
      for (int32_t k = 0; k < s->W; ++k) {
        const size_t slot = (size_t)i * s->W + k;
        if (k < len) {
          s->ecol[slot] = s->col[s->ptr[i] + k];
          s->epos[slot] = s->ptr[i] + k;
        } else {
          s->ecol[slot] = (int32_t)i;
        }
      }
    }
    s->cmass = cm;
    s->n = n_nodes;
    s->have_mesh = true;
    s->bound = false;
    return ENS_OK;
  } catch (const std::exception& ex) {
    return s->fail(ENS_EDEVICE, std::string("spde_set_mesh: ") + ex.what());
  }
}

int32_t spde_workspace_size(spde_ctx* s, int32_t S, size_t* bytes) {
  if (!s || !bytes || S < 1) return ENS_EINVAL;
  if (!s->have_mesh) return s->fail(ENS_ESTATE, "spde_workspace_size: set the mesh first");
  plan(s, S);
  *bytes = s->total;
  return ENS_OK;
}

int32_t spde_bind_workspace(spde_ctx* s, int32_t S, void* dptr, size_t bytes) {
  if (!s || !dptr || S < 1) return ENS_EINVAL;
  if (!s->have_mesh) return s->fail(ENS_ESTATE, "spde_bind_workspace: set the mesh first");
  if (reinterpret_cast<uintptr_t>(dptr) % 256 != 0)
    return s->fail(ENS_EWORKSPACE, "spde_bind_workspace: buffer must be 256-byte aligned");
  plan(s, S);
  if (bytes < s->total)
    return s->fail(ENS_EWORKSPACE, "spde_bind_workspace: need " + std::to_string(s->total) + " bytes");
  s->ws = static_cast<char*>(dptr);
  s->S = S;
  SHIPC(hipSetDevice(s->device));
  SHIPC(hipMemcpy(s->p<void>(s->o_col), s->ecol.data(), 4 * s->ecol.size(), hipMemcpyHostToDevice));
  std::vector<double> sq(s->n);
  for (int64_t i = 0; i < s->n; ++i) sq[i] = std::sqrt(s->cmass[i]);
  SHIPC(hipMemcpy(s->p<void>(s->o_sqrtc), sq.data(), 8 * sq.size(), hipMemcpyHostToDevice));
  s->bound = true;
  return ENS_OK;
}

int32_t spde_sample(spde_ctx* s, double kappa, const double* z, double tol, int32_t max_iter, double* x,
                    int32_t* iterations, double* max_relres) {
  if (!s || !z || !x) return ENS_EINVAL;
  if (!s->bound) return s->fail(ENS_EWORKSPACE, "spde_sample: bind a workspace first");
  if (!(kappa > 0.0) || !std::isfinite(kappa)) return s->fail(ENS_EINVAL, "spde_sample: kappa must be positive");
  if (!(tol > 0.0) || max_iter < 1) return s->fail(ENS_EINVAL, "spde_sample: need tol > 0 and max_iter >= 1");
  SHIPC(hipSetDevice(s->device));
  const int64_t n = s->n;
  const int32_t S = s->S, ld = s->ld;
  // K = kappa^2 C~ + G and its diagonal preconditioner
  std::vector<double> val(s->g);
  std::vector<double> dinv(n);
  for (int64_t i = 0; i < n; ++i) {
    val[s->diag[i]] += kappa * kappa * s->cmass[i];
    dinv[i] = 1.0 / val[s->diag[i]];
  }
  {
    std::vector<double> ev(s->epos.size(), 0.0);
    for (size_t k = 0; k < ev.size(); ++k)
      if (s->epos[k] >= 0) ev[k] = val[s->epos[k]];
    SHIPC(hipMemcpy(s->p<void>(s->o_val), ev.data(), 8 * ev.size(), hipMemcpyHostToDevice));
  }
  SHIPC(hipMemcpy(s->p<void>(s->o_dinv), dinv.data(), 8 * n, hipMemcpyHostToDevice));
  {
    std::vector<double> zp((size_t)n * ld, 0.0);
    for (int64_t i = 0; i < n; ++i) std::memcpy(&zp[(size_t)i * ld], z + i * S, 8 * (size_t)S);
    SHIPC(hipMemcpy(s->p<void>(s->o_z), zp.data(), 8 * zp.size(), hipMemcpyHostToDevice));
  }
  Solve v;
  v.n = n;
  v.ld = ld;
  v.W = s->W;
  v.S = S;
  v.ecol = s->p<int32_t>(s->o_col);
  v.eval = s->p<double>(s->o_val);
  v.dinv = s->p<double>(s->o_dinv);
  v.sqrtc = s->p<double>(s->o_sqrtc);
  v.z = s->p<double>(s->o_z);
  v.X = s->p<double>(s->o_x);
  v.R = s->p<double>(s->o_r);
  v.P = s->p<double>(s->o_p);
  v.Q = s->p<double>(s->o_q);
  v.pa = s->p<double>(s->o_pa);
  v.pb = s->p<double>(s->o_pb);
  v.rz = s->p<double>(s->o_rz);
  v.rz2 = s->p<double>(s->o_rz2);
  v.rr = s->p<double>(s->o_rr);
  v.pq = s->p<double>(s->o_pq);
  v.bb = s->p<double>(s->o_bb);
  int it = 0;
  double worst = 0.0;
  if (ld % 256 == 0) SHIPC((cg<4>(v, tol, max_iter, it, worst)));
  else if (ld % 128 == 0) SHIPC((cg<2>(v, tol, max_iter, it, worst)));
  else SHIPC((cg<1>(v, tol, max_iter, it, worst)));
  SHIPC(hipDeviceSynchronize());
  std::vector<double> xp((size_t)n * ld);
  SHIPC(hipMemcpy(xp.data(), v.X, 8 * xp.size(), hipMemcpyDeviceToHost));
  for (int64_t i = 0; i < n; ++i) std::memcpy(x + i * S, &xp[(size_t)i * ld], 8 * (size_t)S);
  if (iterations) *iterations = it;
  if (max_relres) *max_relres = worst;
  return ENS_OK;
}

}  // extern "C"
