// SPDE / GMRF sampler of Matern fields on the wall mesh (Sec. 2.1):
// x = K^-1 C~^(1/2) z, K = kappa^2 C~ + G, by block conjugate gradients
// over S right-hand sides with a diagonal preconditioner.
//
// Block vectors are [n][ld] with samples fastest (ld = S rounded up to 64);
// a wave owns one matrix row for 64 samples, so the row's column indices
// and values are wave-uniform (scalar loads).  Every per-sample scalar of
// CG (r.z, p.q, r.r) is reduced in a fixed order: per-workgroup partials,
// then one pass over the partials per column.
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
constexpr int kPartWG = 512;    // workgroups along the rows (reduction partials)

__device__ __forceinline__ int wave_row(int64_t& r) {
  r = (int64_t)blockIdx.x * kRowsWG + threadIdx.x / 64;
  return threadIdx.x % 64;
}

// Partial sums of up to two per-column quantities over the rows a
// workgroup visits: LDS tree over its 4 waves, one value per column.
__device__ __forceinline__ void block_partials(double a, double b, int lane, double* __restrict__ part_a,
                                               double* __restrict__ part_b, int64_t col, int32_t ld) {
  __shared__ double ra[256], rb[256];
  ra[threadIdx.x] = a;
  rb[threadIdx.x] = b;
  __syncthreads();
  if (threadIdx.x < 64) {
    double sa = ra[lane], sb = rb[lane];
    for (int w = 1; w < kRowsWG; ++w) {
      sa += ra[64 * w + lane];
      sb += rb[64 * w + lane];
    }
    part_a[(int64_t)blockIdx.x * ld + col] = sa;
    if (part_b) part_b[(int64_t)blockIdx.x * ld + col] = sb;
  }
}

// r = sqrt(C~) z, x = 0, p = D^-1 r; partials of r.D^-1.r and r.r.
__global__ __launch_bounds__(256) void k_init(int64_t n, int32_t ld, const double* __restrict__ sqrtc,
                                              const double* __restrict__ dinv, const double* __restrict__ z,
                                              double* __restrict__ X, double* __restrict__ R,
                                              double* __restrict__ P, double* __restrict__ part_rz,
                                              double* __restrict__ part_rr) {
  const int lane = threadIdx.x % 64;
  const int64_t col = (int64_t)blockIdx.y * 64 + lane;
  double rz = 0.0, rr = 0.0;
  for (int64_t row = (int64_t)blockIdx.x * kRowsWG + threadIdx.x / 64; row < n; row += (int64_t)gridDim.x * kRowsWG) {
    const int64_t i = row * ld + col;
    const double r = sqrtc[row] * z[i];
    const double zz = dinv[row] * r;
    X[i] = 0.0;
    R[i] = r;
    P[i] = zz;
    rz += r * zz;
    rr += r * r;
  }
  block_partials(rz, rr, lane, part_rz, part_rr, col, ld);
}

// Q = K P (CSR, wave-uniform rows); partials of p.q.
__global__ __launch_bounds__(256) void k_spmv(int64_t n, int32_t ld, const int32_t* __restrict__ ptr,
                                              const int32_t* __restrict__ colidx, const double* __restrict__ val,
                                              const double* __restrict__ P, double* __restrict__ Q,
                                              double* __restrict__ part_pq) {
  const int lane = threadIdx.x % 64;
  const int64_t col = (int64_t)blockIdx.y * 64 + lane;
  double pq = 0.0;
  for (int64_t row = (int64_t)blockIdx.x * kRowsWG + threadIdx.x / 64; row < n; row += (int64_t)gridDim.x * kRowsWG) {
    const int r = __builtin_amdgcn_readfirstlane((int)row);
    const int kb = ptr[r], ke = ptr[r + 1];
    double q = 0.0;
    for (int k = kb; k < ke; ++k) q = fma(val[k], P[(int64_t)colidx[k] * ld + col], q);
    Q[(int64_t)r * ld + col] = q;
    pq = fma(P[(int64_t)r * ld + col], q, pq);
  }
  block_partials(pq, 0.0, lane, part_pq, nullptr, col, ld);
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
__global__ __launch_bounds__(256) void k_update_xr(int64_t n, int32_t ld, const double* __restrict__ dinv,
                                                   const double* __restrict__ rz, const double* __restrict__ pq,
                                                   double* __restrict__ X, double* __restrict__ R,
                                                   const double* __restrict__ P, const double* __restrict__ Q,
                                                   double* __restrict__ part_rz, double* __restrict__ part_rr) {
  const int lane = threadIdx.x % 64;
  const int64_t col = (int64_t)blockIdx.y * 64 + lane;
  const double alpha = pq[col] > 0.0 ? rz[col] / pq[col] : 0.0;
  double srz = 0.0, srr = 0.0;
  for (int64_t row = (int64_t)blockIdx.x * kRowsWG + threadIdx.x / 64; row < n; row += (int64_t)gridDim.x * kRowsWG) {
    const int64_t i = row * ld + col;
    X[i] = fma(alpha, P[i], X[i]);
    const double r = fma(-alpha, Q[i], R[i]);
    R[i] = r;
    srz = fma(r, dinv[row] * r, srz);
    srr = fma(r, r, srr);
  }
  block_partials(srz, srr, lane, part_rz, part_rr, col, ld);
}

// beta = rz_new / rz_old; p = D^-1 r + beta p.
__global__ __launch_bounds__(256) void k_update_p(int64_t n, int32_t ld, const double* __restrict__ dinv,
                                                  const double* __restrict__ rz_new,
                                                  const double* __restrict__ rz_old, const double* __restrict__ R,
                                                  double* __restrict__ P) {
  const int lane = threadIdx.x % 64;
  const int64_t col = (int64_t)blockIdx.y * 64 + lane;
  const double beta = rz_old[col] > 0.0 ? rz_new[col] / rz_old[col] : 0.0;
  for (int64_t row = (int64_t)blockIdx.x * kRowsWG + threadIdx.x / 64; row < n; row += (int64_t)gridDim.x * kRowsWG) {
    const int64_t i = row * ld + col;
    P[i] = fma(beta, P[i], dinv[row] * R[i]);
  }
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
  bool have_mesh = false;
  // workspace
  char* ws = nullptr;
  int32_t S = 0, ld = 0;
  size_t o_ptr = 0, o_col = 0, o_val = 0, o_dinv = 0, o_sqrtc = 0, o_z = 0, o_x = 0, o_r = 0, o_p = 0, o_q = 0,
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
  const size_t n = (size_t)s->n, nnz = s->col.size();
  size_t off = 0;
  auto take = [&](size_t b) {
    const size_t o = off;
    off = align256(off + b);
    return o;
  };
  s->o_ptr = take(4 * (n + 1));
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
  SHIPC(hipMemcpy(s->p<void>(s->o_ptr), s->ptr.data(), 4 * s->ptr.size(), hipMemcpyHostToDevice));
  SHIPC(hipMemcpy(s->p<void>(s->o_col), s->col.data(), 4 * s->col.size(), hipMemcpyHostToDevice));
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
  SHIPC(hipMemcpy(s->p<void>(s->o_val), val.data(), 8 * val.size(), hipMemcpyHostToDevice));
  SHIPC(hipMemcpy(s->p<void>(s->o_dinv), dinv.data(), 8 * n, hipMemcpyHostToDevice));
  {
    std::vector<double> zp((size_t)n * ld, 0.0);
    for (int64_t i = 0; i < n; ++i) std::memcpy(&zp[(size_t)i * ld], z + i * S, 8 * (size_t)S);
    SHIPC(hipMemcpy(s->p<void>(s->o_z), zp.data(), 8 * zp.size(), hipMemcpyHostToDevice));
  }
  const dim3 grid((unsigned)std::min<int64_t>(kPartWG, (n + kRowsWG - 1) / kRowsWG), (unsigned)(ld / 64));
  const int nparts = (int)grid.x;
  const unsigned cgrid = (unsigned)(ld / 64);
  double *X = s->p<double>(s->o_x), *R = s->p<double>(s->o_r), *P = s->p<double>(s->o_p), *Q = s->p<double>(s->o_q);
  double *pa = s->p<double>(s->o_pa), *pb = s->p<double>(s->o_pb);
  double *rz = s->p<double>(s->o_rz), *rz2 = s->p<double>(s->o_rz2), *rr = s->p<double>(s->o_rr);
  double *pq = s->p<double>(s->o_pq), *bb = s->p<double>(s->o_bb);
  const double* dv = s->p<double>(s->o_dinv);
  k_init<<<grid, 256>>>(n, ld, s->p<double>(s->o_sqrtc), dv, s->p<double>(s->o_z), X, R, P, pa, pb);
  k_colsum<<<cgrid, 64 * kColWaves>>>(ld, nparts, pa, rz, pb, bb);
  SHIPC(hipGetLastError());
  std::vector<double> hbb(ld), hrr(ld);
  SHIPC(hipMemcpy(hbb.data(), bb, 8 * ld, hipMemcpyDeviceToHost));
  int it = 0;
  double worst = 0.0;
  auto converged = [&](const std::vector<double>& r2) {
    worst = 0.0;
    for (int c = 0; c < S; ++c) {
      const double rel = hbb[c] > 0.0 ? std::sqrt(r2[c] / hbb[c]) : 0.0;
      worst = std::max(worst, rel);
    }
    return worst <= tol;
  };
  if (!converged(hbb)) {
    while (it < max_iter) {
      k_spmv<<<grid, 256>>>(n, ld, s->p<int32_t>(s->o_ptr), s->p<int32_t>(s->o_col), s->p<double>(s->o_val), P, Q,
                            pa);
      k_colsum<<<cgrid, 64 * kColWaves>>>(ld, nparts, pa, pq, nullptr, nullptr);
      k_update_xr<<<grid, 256>>>(n, ld, dv, rz, pq, X, R, P, Q, pa, pb);
      k_colsum<<<cgrid, 64 * kColWaves>>>(ld, nparts, pa, rz2, pb, rr);
      k_update_p<<<grid, 256>>>(n, ld, dv, rz2, rz, R, P);
      SHIPC(hipGetLastError());
      std::swap(rz, rz2);
      ++it;
      if (it % 8 == 0 || it == max_iter) {
        SHIPC(hipMemcpy(hrr.data(), rr, 8 * ld, hipMemcpyDeviceToHost));
        if (converged(hrr)) break;
      }
    }
  }
  SHIPC(hipDeviceSynchronize());
  std::vector<double> xp((size_t)n * ld);
  SHIPC(hipMemcpy(xp.data(), X, 8 * xp.size(), hipMemcpyDeviceToHost));
  for (int64_t i = 0; i < n; ++i) std::memcpy(x + i * S, &xp[(size_t)i * ld], 8 * (size_t)S);
  if (iterations) *iterations = it;
  if (max_relres) *max_relres = worst;
  return ENS_OK;
}

}  // extern "C"
