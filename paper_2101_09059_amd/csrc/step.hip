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
//   u_{n+1}   = u_n + dt v_{n+1/2}
// formed in FP64 from the stored FP32 values (F32_KAHAN stores u as a
// compensated pair u_hi - u_lo).
// Clamped dofs are written as zero.  Optional outputs in the same pass:
// running peak radial displacement and the per-sample discrete energy.
#include "internal.h"

#include <cmath>

// Incident elements whose loads a wave keeps in flight together.
#ifndef ENSFEM_GATHER_UNROLL
#define ENSFEM_GATHER_UNROLL 2
#endif
// Issue the node's single-use loads (u_{n-1}, 1/m) before the gather so
// they are in flight during it (FP64 state).
#ifndef ENSFEM_HOIST_STREAMS
#define ENSFEM_HOIST_STREAMS 1
#endif
#define ENSFEM_PRAGMA(x) _Pragma(#x)
#define ENSFEM_UNROLL_GATHER ENSFEM_PRAGMA(unroll ENSFEM_GATHER_UNROLL)

namespace ensfem {
namespace {

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

// Generic view of a global-memory pointer held in an argument struct.
template <typename T>
__device__ __forceinline__ T* gen(ENS_GLOBAL T* ptr) {
  return (T*)ptr;
}

// Read-only view (constant address space) of mesh data that no kernel of
// the step writes: adjacency, stiffness blocks, load, clamp bits, radial
// directions, load factors, and the batch tables.  Uniform loads through it
// go to the scalar unit even where the kernel stores to other arrays in a
// loop (through a global pointer the compiler must assume those stores may
// alias the data and falls back to vector loads).
template <typename T>
using ConstPtr = const T __attribute__((address_space(4)))*;
template <typename T>
__device__ __forceinline__ ConstPtr<T> cst(ENS_GLOBAL T* ptr) {
  return (ConstPtr<T>)ptr;
}
template <typename T>
__device__ __forceinline__ ConstPtr<T> cst(const T* ptr) {
  return (ConstPtr<T>)ptr;
}

// Move a wave-uniform value into a scalar register.  Where the compiler
// already loads it through the scalar unit this folds away; where it had to
// use a vector load (arrays reached through a device table may alias the
// kernel's stores, so the scalar cache cannot be used) it frees the VGPRs.
template <typename T>
__device__ __forceinline__ T uni(T v) {
  if constexpr (sizeof(T) == 4) {
    return __builtin_bit_cast(T, __builtin_amdgcn_readfirstlane(__builtin_bit_cast(int, v)));
  } else if constexpr (sizeof(T) == 8) {
    const unsigned long long u = __builtin_bit_cast(unsigned long long, v);
    const unsigned lo = (unsigned)__builtin_amdgcn_readfirstlane((int)(unsigned)(u & 0xffffffffu));
    const unsigned hi = (unsigned)__builtin_amdgcn_readfirstlane((int)(unsigned)(u >> 32));
    return __builtin_bit_cast(T, ((unsigned long long)hi << 32) | lo);
  } else {
    return v;
  }
}

template <bool U, typename T>
__device__ __forceinline__ T maybe_uni(T v) {
  if constexpr (U) return uni(v);
  else return v;
}

// N consecutive samples per lane: one vector memory access per row.
template <typename T, int N> struct VecOf;
template <typename T> struct VecOf<T, 1> { typedef T type; };
template <> struct VecOf<float, 2> { typedef float type __attribute__((ext_vector_type(2))); };
template <> struct VecOf<float, 4> { typedef float type __attribute__((ext_vector_type(4))); };
template <> struct VecOf<double, 2> { typedef double type __attribute__((ext_vector_type(2))); };
template <> struct VecOf<double, 4> { typedef double type __attribute__((ext_vector_type(4))); };

template <int N, bool NT, typename T>
__device__ __forceinline__ void vload(const T* __restrict__ ptr, T (&out)[N]) {
  typedef typename VecOf<T, N>::type V;
  V v;
  if constexpr (NT) v = __builtin_nontemporal_load(reinterpret_cast<const V*>(ptr));
  else v = *reinterpret_cast<const V*>(ptr);
  if constexpr (N == 1) {
    out[0] = v;
  } else {
#pragma unroll
    for (int i = 0; i < N; ++i) out[i] = v[i];
  }
}

template <int N, bool NT, typename T>
__device__ __forceinline__ void vstore(T* __restrict__ ptr, const T (&in)[N]) {
  typedef typename VecOf<T, N>::type V;
  V v;
  if constexpr (N == 1) {
    v = in[0];
  } else {
#pragma unroll
    for (int i = 0; i < N; ++i) v[i] = in[i];
  }
  if constexpr (NT) __builtin_nontemporal_store(v, reinterpret_cast<V*>(ptr));
  else *reinterpret_cast<V*>(ptr) = v;
}

// One row of the 3x6 block times the six differences, as a fixed chain of
// fused multiply-adds (the library is built without implicit contraction so
// every lane mapping performs exactly these operations).
template <typename AT>
__device__ __forceinline__ AT row6(const AT* __restrict__ k, AT d0, AT d1, AT d2, AT d3, AT d4, AT d5) {
  AT f = k[0] * d0;
  f = fma(k[1], d1, f);
  f = fma(k[2], d2, f);
  f = fma(k[3], d3, f);
  f = fma(k[4], d4, f);
  return fma(k[5], d5, f);
}

// Row of node n in a caller buffer: map[n] (caller numbering) or n itself.
template <bool MAP>
__device__ __forceinline__ int64_t node_row(const int32_t* __restrict__ map, int n) {
  if constexpr (MAP) return (int64_t)map[n] * 3;
  else return (int64_t)n * 3;
}

// R for one node and SPL consecutive samples starting at s0, in two forms.
// Rows form (the FP64 apply): the walk's shared neighbour is carried as its
// loaded row; an entry that closes the fan is loaded again.
template <typename AT, typename ST, int SPL, bool UNI, bool MAP = false>
__device__ __forceinline__ void gather_apply_rows(const StepArgs& p, int node, int64_t ld, int s0,
                                                  const ST* __restrict__ U, const ST (&ua)[3][SPL],
                                                  AT (&r)[3][SPL], const int32_t* __restrict__ map = nullptr) {
  const int kb = maybe_uni<UNI>(cst(p.adj.ptr)[node]);
  const int ke = maybe_uni<UNI>(cst(p.adj.ptr)[node + 1]);
  const ConstPtr<AT> KB = (ConstPtr<AT>)cst(p.adj.k);
  const AT* __restrict__ EH = static_cast<const AT*>(gen(p.eh));
#pragma unroll
  for (int c = 0; c < 3; ++c)
#pragma unroll
    for (int i = 0; i < SPL; ++i) r[c][i] = AT(0);
  ST ub[3][SPL], uc[3][SPL];
  ENSFEM_UNROLL_GATHER
  for (int k = kb; k < ke; ++k) {
    const int64_t e = maybe_uni<UNI>(cst(p.adj.el)[k]);
    const ConstPtr<int> nb = (ConstPtr<int>)cst(p.adj.nb);
    const int2 bc0 = make_int2(nb[2 * k], nb[2 * k + 1]);
    const int2 bc = make_int2(maybe_uni<UNI>(bc0.x), maybe_uni<UNI>(bc0.y));
    AT kk[18];
#pragma unroll
    for (int i = 0; i < 18; ++i) kk[i] = maybe_uni<UNI>(KB[(int64_t)k * 18 + i]);
    AT eh[SPL];
    vload<SPL, false>(EH + e * ld + s0, eh);
    // bc.x < 0: this element's first neighbour is the previous one's second
    if (bc.x >= 0) {
      const int64_t rb = node_row<MAP>(map, bc.x);
#pragma unroll
      for (int c = 0; c < 3; ++c) vload<SPL, false>(U + (rb + c) * ld + s0, ub[c]);
    } else {
#pragma unroll
      for (int c = 0; c < 3; ++c)
#pragma unroll
        for (int i = 0; i < SPL; ++i) ub[c][i] = uc[c][i];
    }
    const int64_t rc = node_row<MAP>(map, bc.y < 0 ? ~bc.y : bc.y);
#pragma unroll
    for (int c = 0; c < 3; ++c) vload<SPL, false>(U + (rc + c) * ld + s0, uc[c]);
#pragma unroll
    for (int i = 0; i < SPL; ++i) {
      const AT d0 = (AT)(ub[0][i] - ua[0][i]);
      const AT d1 = (AT)(ub[1][i] - ua[1][i]);
      const AT d2 = (AT)(ub[2][i] - ua[2][i]);
      const AT d3 = (AT)(uc[0][i] - ua[0][i]);
      const AT d4 = (AT)(uc[1][i] - ua[1][i]);
      const AT d5 = (AT)(uc[2][i] - ua[2][i]);
      const AT f0 = row6(kk + 0, d0, d1, d2, d3, d4, d5);
      const AT f1 = row6(kk + 6, d0, d1, d2, d3, d4, d5);
      const AT f2 = row6(kk + 12, d0, d1, d2, d3, d4, d5);
      r[0][i] = fma(eh[i], f0, r[0][i]);
      r[1][i] = fma(eh[i], f1, r[1][i]);
      r[2][i] = fma(eh[i], f2, r[2][i]);
    }
  }
}

// Differences form (the FP32 apply): the walk's shared neighbour (and, with
// CLOSE, the fan's first one for the element that closes the fan) is
// carried as its converted differences u_b - u_a rather than its rows: the
// same operations in the same order as the rows form, fewer registers.
template <typename AT, typename ST, int SPL, bool UNI, bool MAP = false, bool CLOSE = true>
__device__ __forceinline__ void gather_apply_diff(const StepArgs& p, int node, int64_t ld, int s0,
                                                  const ST* __restrict__ U, const ST (&ua)[3][SPL],
                                                  AT (&r)[3][SPL], const int32_t* __restrict__ map = nullptr) {
  constexpr bool kClose = CLOSE && ENSFEM_CLOSE_REUSE;
  const int kb = maybe_uni<UNI>(cst(p.adj.ptr)[node]);
  const int ke = maybe_uni<UNI>(cst(p.adj.ptr)[node + 1]);
  const ConstPtr<AT> KB = (ConstPtr<AT>)cst(p.adj.k);
  const AT* __restrict__ EH = static_cast<const AT*>(gen(p.eh));
#pragma unroll
  for (int c = 0; c < 3; ++c)
#pragma unroll
    for (int i = 0; i < SPL; ++i) r[c][i] = AT(0);
  AT db[3][SPL], dc[3][SPL];
  AT d0s[kClose ? 3 : 1][kClose ? SPL : 1];  // the walk's first neighbour's differences
  ENSFEM_UNROLL_GATHER
  for (int k = kb; k < ke; ++k) {
    const int64_t e = maybe_uni<UNI>(cst(p.adj.el)[k]);
    const ConstPtr<int> nb = (ConstPtr<int>)cst(p.adj.nb);
    const int2 bc0 = make_int2(nb[2 * k], nb[2 * k + 1]);
    const int2 bc = make_int2(maybe_uni<UNI>(bc0.x), maybe_uni<UNI>(bc0.y));
    AT kk[18];
#pragma unroll
    for (int i = 0; i < 18; ++i) kk[i] = maybe_uni<UNI>(KB[(int64_t)k * 18 + i]);
    AT eh[SPL];
    vload<SPL, false>(EH + e * ld + s0, eh);
    // bc.x < 0: this element's first neighbour is the previous one's second
    if (bc.x >= 0) {
      const int64_t rb = node_row<MAP>(map, bc.x);
      ST ub[3][SPL];
#pragma unroll
      for (int c = 0; c < 3; ++c) vload<SPL, false>(U + (rb + c) * ld + s0, ub[c]);
#pragma unroll
      for (int c = 0; c < 3; ++c)
#pragma unroll
        for (int i = 0; i < SPL; ++i) db[c][i] = (AT)(ub[c][i] - ua[c][i]);
      if constexpr (kClose)
        if (k == kb)
#pragma unroll
          for (int c = 0; c < 3; ++c)
#pragma unroll
            for (int i = 0; i < SPL; ++i) d0s[c][i] = db[c][i];
    } else {
#pragma unroll
      for (int c = 0; c < 3; ++c)
#pragma unroll
        for (int i = 0; i < SPL; ++i) db[c][i] = dc[c][i];
    }
    // bc.y < 0: this element's second neighbour is the walk's first one
    if (kClose && bc.y < 0) {
#pragma unroll
      for (int c = 0; c < 3; ++c)
#pragma unroll
        for (int i = 0; i < SPL; ++i) dc[c][i] = d0s[kClose ? c : 0][kClose ? i : 0];
    } else {
      const int64_t rc = node_row<MAP>(map, bc.y < 0 ? ~bc.y : bc.y);
      ST uc[3][SPL];
#pragma unroll
      for (int c = 0; c < 3; ++c) vload<SPL, false>(U + (rc + c) * ld + s0, uc[c]);
#pragma unroll
      for (int c = 0; c < 3; ++c)
#pragma unroll
        for (int i = 0; i < SPL; ++i) dc[c][i] = (AT)(uc[c][i] - ua[c][i]);
    }
#pragma unroll
    for (int i = 0; i < SPL; ++i) {
      const AT f0 = row6(kk + 0, db[0][i], db[1][i], db[2][i], dc[0][i], dc[1][i], dc[2][i]);
      const AT f1 = row6(kk + 6, db[0][i], db[1][i], db[2][i], dc[0][i], dc[1][i], dc[2][i]);
      const AT f2 = row6(kk + 12, db[0][i], db[1][i], db[2][i], dc[0][i], dc[1][i], dc[2][i]);
      r[0][i] = fma(eh[i], f0, r[0][i]);
      r[1][i] = fma(eh[i], f1, r[1][i]);
      r[2][i] = fma(eh[i], f2, r[2][i]);
    }
  }
}

// CLOSE: the element that closes a node's fan takes the walk's first
// neighbour from registers (the FP32 single-mesh step kernels).
template <typename AT, typename ST, int SPL, bool UNI, bool MAP = false, bool CLOSE = true>
__device__ __forceinline__ void gather_apply(const StepArgs& p, int node, int64_t ld, int s0,
                                             const ST* __restrict__ U, const ST (&ua)[3][SPL],
                                             AT (&r)[3][SPL], const int32_t* __restrict__ map = nullptr) {
  // the FP32 apply carries differences (fewer registers: 70 against 82 for
  // the headline step, 7 waves per SIMD against 5); the FP64 apply keeps rows
  if constexpr (std::is_same<AT, float>::value)
    gather_apply_diff<AT, ST, SPL, UNI, MAP, CLOSE>(p, node, ld, s0, U, ua, r, map);
  else
    gather_apply_rows<AT, ST, SPL, UNI, MAP>(p, node, ld, s0, U, ua, r, map);
}

// Shared stiffness: R_i = sum_j K_ij (u_j - u_i) over the assembled
// off-diagonal 3x3 blocks of row i.
template <typename AT, typename ST, int SPL, bool UNI, bool MAP = false>
__device__ __forceinline__ void gather_blocks(const StepArgs& p, int node, int64_t ld, int s0,
                                              const ST* __restrict__ U, const ST (&ua)[3][SPL],
                                              AT (&r)[3][SPL], const int32_t* __restrict__ map = nullptr) {
  const int kb = maybe_uni<UNI>(cst(p.bsr.ptr)[node]);
  const int ke = maybe_uni<UNI>(cst(p.bsr.ptr)[node + 1]);
  const ConstPtr<AT> V = (ConstPtr<AT>)cst(p.bsr.val);
#pragma unroll
  for (int c = 0; c < 3; ++c)
#pragma unroll
    for (int i = 0; i < SPL; ++i) r[c][i] = AT(0);
#pragma unroll 2
  for (int k = kb; k < ke; ++k) {
    const int64_t rj = node_row<MAP>(map, maybe_uni<UNI>(cst(p.bsr.col)[k]));
    AT B[9];
#pragma unroll
    for (int i = 0; i < 9; ++i) B[i] = maybe_uni<UNI>(V[(int64_t)k * 9 + i]);
    ST uj[3][SPL];
#pragma unroll
    for (int c = 0; c < 3; ++c) vload<SPL, false>(U + (rj + c) * ld + s0, uj[c]);
#pragma unroll
    for (int i = 0; i < SPL; ++i) {
      const AT d0 = (AT)(uj[0][i] - ua[0][i]);
      const AT d1 = (AT)(uj[1][i] - ua[1][i]);
      const AT d2 = (AT)(uj[2][i] - ua[2][i]);
#pragma unroll
      for (int c = 0; c < 3; ++c) r[c][i] = fma(B[3 * c + 2], d2, fma(B[3 * c + 1], d1, fma(B[3 * c], d0, r[c][i])));
    }
  }
}

// Geometry form: K(x + u_m) (u_n - u_m) for one node, with element matrices
// evaluated on each sample's geometry of the last refresh x + u_m (matrix-
// free, no stored K^e); the caller adds the force base R_m.  For the
// element (i, b, c) of the walk, with a = P_b - P_i and w = P_c - P_i:
// e_x = a/|a|, e_z = a x w/|a x w|, e_y = e_z x e_x; node i sits at the
// local origin, b at (x2, 0), c at (x3, y3).  With the increments
// du = u_n - u_m, the local differences d_b = R (du_b - du_i),
// d_c = R (du_c - du_i) give the strains
// (the rows of the strain-displacement matrix: du_x/dx, du_y/dy, gamma_xy,
// du_z/dx, du_z/dy, Sec. 2.2.1), the constitutive matrix per unit (E h)
// the stresses, and node i's force A B_i^T sigma is rotated back to global
// axes.  The element matrix is invariant under a proper rotation of its
// local frame (isotropic material), so the walk's vertex order serves as
// well as the connectivity's.  Edge vectors are formed in FP64 before the
// conversion to AT.
__device__ __forceinline__ float rsq(float x) { return rsqrtf(x); }
__device__ __forceinline__ double rsq(double x) { return rsqrt(x); }

template <typename AT, int SPL, bool UNI>
__device__ __forceinline__ void gather_geom(const StepArgs& p, int node, int64_t ld, int s0,
                                            const double* __restrict__ U, const double (&ua)[3][SPL],
                                            AT (&r)[3][SPL]) {
  const int kb = maybe_uni<UNI>(cst(p.adj.ptr)[node]);
  const int ke = maybe_uni<UNI>(cst(p.adj.ptr)[node + 1]);
  const AT* __restrict__ EH = static_cast<const AT*>(gen(p.eh));
  const double* __restrict__ US = gen(p.usnap);
  const ConstPtr<double> X = cst(p.xyz);
  const int64_t row = (int64_t)node * 3;
  const AT nu = (AT)p.nu;
  const AT c0 = (AT)(1.0 / (1.0 - p.nu * p.nu));
  const AT cg = (AT)(0.5 * (1.0 - p.nu) / (1.0 - p.nu * p.nu));
  const AT cs = (AT)(0.5 * p.shear_k * (1.0 - p.nu) / (1.0 - p.nu * p.nu));
  double xi[3], si[3][SPL];
#pragma unroll
  for (int c = 0; c < 3; ++c) {
    xi[c] = maybe_uni<UNI>(X[row + c]);
    vload<SPL, false>(US + (row + c) * ld + s0, si[c]);
  }
#pragma unroll
  for (int c = 0; c < 3; ++c)
#pragma unroll
    for (int i = 0; i < SPL; ++i) r[c][i] = AT(0);
  double dui[3][SPL];  // u_n - u_m at node i
#pragma unroll
  for (int c = 0; c < 3; ++c)
#pragma unroll
    for (int i = 0; i < SPL; ++i) dui[c][i] = ua[c][i] - si[c][i];
  // edge vector and increment difference to the element's second neighbour,
  // in the apply precision; a reused first neighbour takes them over
  AT wc[3][SPL], dcc[3][SPL];
#pragma unroll 2
  for (int k = kb; k < ke; ++k) {
    const int64_t e = maybe_uni<UNI>(cst(p.adj.el)[k]);
    const ConstPtr<int> nb = (ConstPtr<int>)cst(p.adj.nb);
    const int bx = maybe_uni<UNI>(nb[2 * k]);
    const int cx0 = maybe_uni<UNI>(nb[2 * k + 1]);
    const int cx = cx0 < 0 ? ~cx0 : cx0;  // a closing entry names the walk's first neighbour
    AT eh[SPL];
    vload<SPL, false>(EH + e * ld + s0, eh);
    AT ab[3][SPL], dbb[3][SPL];
    // bx < 0: this element's first neighbour is the previous one's second
    if (bx >= 0) {
      const int64_t rb = (int64_t)bx * 3;
#pragma unroll
      for (int c = 0; c < 3; ++c) {
        const double xb = maybe_uni<UNI>(X[rb + c]);
        double ub[SPL], sb[SPL];
        vload<SPL, false>(U + (rb + c) * ld + s0, ub);
        vload<SPL, false>(US + (rb + c) * ld + s0, sb);
#pragma unroll
        for (int i = 0; i < SPL; ++i) {
          ab[c][i] = (AT)((xb - xi[c]) + (sb[i] - si[c][i]));
          dbb[c][i] = (AT)((ub[i] - sb[i]) - dui[c][i]);
        }
      }
    } else {
#pragma unroll
      for (int c = 0; c < 3; ++c)
#pragma unroll
        for (int i = 0; i < SPL; ++i) {
          ab[c][i] = wc[c][i];
          dbb[c][i] = dcc[c][i];
        }
    }
    const int64_t rc = (int64_t)cx * 3;
#pragma unroll
    for (int c = 0; c < 3; ++c) {
      const double xc = maybe_uni<UNI>(X[rc + c]);
      double uc[SPL], sc[SPL];
      vload<SPL, false>(U + (rc + c) * ld + s0, uc);
      vload<SPL, false>(US + (rc + c) * ld + s0, sc);
#pragma unroll
      for (int i = 0; i < SPL; ++i) {
        wc[c][i] = (AT)((xc - xi[c]) + (sc[i] - si[c][i]));
        dcc[c][i] = (AT)((uc[i] - sc[i]) - dui[c][i]);
      }
    }
#pragma unroll
    for (int i = 0; i < SPL; ++i) {
      AT a[3], w[3], db[3], dc[3];
#pragma unroll
      for (int c = 0; c < 3; ++c) {
        a[c] = ab[c][i];
        w[c] = wc[c][i];
        db[c] = dbb[c][i];
        dc[c] = dcc[c][i];
      }
      // frame
      const AT aa = fma(a[2], a[2], fma(a[1], a[1], a[0] * a[0]));
      const AT ia = rsq(aa);  // 1 / x2
      const AT ex[3] = {a[0] * ia, a[1] * ia, a[2] * ia};
      const AT n[3] = {fma(a[1], w[2], -(a[2] * w[1])), fma(a[2], w[0], -(a[0] * w[2])),
                       fma(a[0], w[1], -(a[1] * w[0]))};
      const AT nn = fma(n[2], n[2], fma(n[1], n[1], n[0] * n[0]));
      const AT in = rsq(nn);
      const AT ez[3] = {n[0] * in, n[1] * in, n[2] * in};
      const AT ey[3] = {fma(ez[1], ex[2], -(ez[2] * ex[1])), fma(ez[2], ex[0], -(ez[0] * ex[2])),
                        fma(ez[0], ex[1], -(ez[1] * ex[0]))};
      const AT area = (AT)0.5 * (nn * in);                   // x2 y3 / 2
      const AT x3 = fma(w[2], ex[2], fma(w[1], ex[1], w[0] * ex[0]));
      const AT iy = (aa * ia) * in;                          // 1 / y3 = x2 / |n|
      const AT q = x3 * ia * iy;                             // x3 / (x2 y3)
      // local differences
      const AT b0 = fma(ex[2], db[2], fma(ex[1], db[1], ex[0] * db[0]));
      const AT b1 = fma(ey[2], db[2], fma(ey[1], db[1], ey[0] * db[0]));
      const AT b2 = fma(ez[2], db[2], fma(ez[1], db[1], ez[0] * db[0]));
      const AT d0 = fma(ex[2], dc[2], fma(ex[1], dc[1], ex[0] * dc[0]));
      const AT d1 = fma(ey[2], dc[2], fma(ey[1], dc[1], ey[0] * dc[0]));
      const AT d2 = fma(ez[2], dc[2], fma(ez[1], dc[1], ez[0] * dc[0]));
      // strains
      const AT exx = b0 * ia;
      const AT eyy = fma(d1, iy, -(q * b1));
      const AT gxy = fma(b1, ia, fma(d0, iy, -(q * b0)));
      const AT gxz = b2 * ia;
      const AT gyz = fma(d2, iy, -(q * b2));
      // stresses per unit (E h)
      const AT sxx = c0 * fma(nu, eyy, exx);
      const AT syy = c0 * fma(nu, exx, eyy);
      const AT txy = cg * gxy;
      const AT txz = cs * gxz;
      const AT tyz = cs * gyz;
      // node i: dN/dx = -1/x2, dN/dy = x3/(x2 y3) - 1/y3
      const AT gx = -ia, gy = q - iy;
      const AT fx = area * fma(gy, txy, gx * sxx);
      const AT fy = area * fma(gx, txy, gy * syy);
      const AT fz = area * fma(gy, tyz, gx * txz);
#pragma unroll
      for (int c = 0; c < 3; ++c) {
        const AT fg = fma(ez[c], fz, fma(ey[c], fy, ex[c] * fx));
        r[c][i] = fma(eh[i], fg, r[c][i]);
      }
    }
  }
}

// Rising bits use a sample-indexed layout, independent of the lane mapping:
// per node ld/64 words, sample s in word s/64, bit s%64.  With SPL samples
// per lane, lane l holds samples SPL*l + i of its block: word
// (SPL*l + i)/64, bit SPL*(l % (64/SPL)) + i.
template <int SPL>
__device__ __forceinline__ uint64_t spread_bits(uint64_t x) {
  if constexpr (SPL == 1) {
    return x;
  } else if constexpr (SPL == 2) {  // bit k of a 32-bit value -> bit 2k
    x &= 0xffffffffull;
    x = (x | (x << 16)) & 0x0000ffff0000ffffull;
    x = (x | (x << 8)) & 0x00ff00ff00ff00ffull;
    x = (x | (x << 4)) & 0x0f0f0f0f0f0f0f0full;
    x = (x | (x << 2)) & 0x3333333333333333ull;
    x = (x | (x << 1)) & 0x5555555555555555ull;
    return x;
  } else {  // SPL == 4: bit k of a 16-bit value -> bit 4k
    x &= 0xffffull;
    x = (x | (x << 24)) & 0x000000ff000000ffull;
    x = (x | (x << 12)) & 0x000f000f000f000full;
    x = (x | (x << 6)) & 0x0303030303030303ull;
    x = (x | (x << 3)) & 0x1111111111111111ull;
    return x;
  }
}

// Work of one wave-or-lane-group on one node and SPL samples per lane:
// stiffness apply, central-difference update, QoI and energy terms.
// `lane` in [0, LPN); samples base + lane*SPL + i (base a multiple of
// LPN*SPL, and of 64 when LPN = 64).
// nwords < SPL (batched step only): the wave's upper lanes are idle and only
// the first nwords rising-bit words belong to this block of samples.
template <typename AT, int MODE, int LPN, int SPL, bool QOI, bool ENERGY, bool SHARED, bool GEOM = false,
          bool CLOSE = true>
__device__ __forceinline__ void step_node(const StepArgs& p, int j, int node, int base, int lane,
                                          double (&e_loc)[SPL], int nwords = SPL) {
  static_assert(!GEOM || (MODE == kStateF64 && !SHARED && !ENERGY), "geometry form: FP64 state only");
  const int s0 = base + lane * SPL;
  const int64_t ld = p.ld;
  using ST = typename std::conditional<MODE == kStateF64, double, float>::type;
  const ST* __restrict__ U = nullptr;
  if constexpr (MODE == kStateF64) U = gen(p.u_cur); else U = gen(p.uh_cur);
  const int64_t row = (int64_t)node * 3;
  ST ua[3][SPL];
#pragma unroll
  for (int c = 0; c < 3; ++c) vload<SPL, false>(U + (row + c) * ld + s0, ua[c]);
  constexpr bool HOIST = ENSFEM_HOIST_STREAMS && MODE == kStateF64;
  const int64_t ms = (int64_t)node * ld + s0;
  double up_h[3][SPL];
  double minv_h[SPL];
  if constexpr (HOIST) {
#pragma unroll
    for (int c = 0; c < 3; ++c) vload<SPL, true>(gen(p.u_prev) + (row + c) * ld + s0, up_h[c]);
    if constexpr (std::is_same<AT, double>::value) {
      vload<SPL, true>(static_cast<const double*>(gen(p.minv)) + ms, minv_h);
    } else {
      float mf[SPL];
      vload<SPL, true>(static_cast<const float*>(gen(p.minv)) + ms, mf);
#pragma unroll
      for (int i = 0; i < SPL; ++i) minv_h[i] = (double)mf[i];
    }
  }
  AT r[3][SPL];
  constexpr bool UNI = LPN == 64;
  // geometry form: force R_m + K_m (u_n - u_m); a refresh step moves the
  // base to the force at u_n (own rows only: no other wave reads them)
  double rf[3][SPL];
  if constexpr (GEOM) {
    gather_geom<AT, SPL, UNI>(p, node, ld, s0, U, ua, r);
#pragma unroll
    for (int c = 0; c < 3; ++c) {
      double rb[SPL];
      vload<SPL, true>(gen(p.rbase) + (row + c) * ld + s0, rb);
#pragma unroll
      for (int i = 0; i < SPL; ++i) rf[c][i] = rb[i] + (double)r[c][i];
      if (p.refresh) vstore<SPL, true>(gen(p.rbase) + (row + c) * ld + s0, rf[c]);
    }
  } else {
    if constexpr (SHARED) gather_blocks<AT, ST, SPL, UNI>(p, node, ld, s0, U, ua, r);
    else gather_apply<AT, ST, SPL, UNI, false, CLOSE>(p, node, ld, s0, U, ua, r);
#pragma unroll
    for (int c = 0; c < 3; ++c)
#pragma unroll
      for (int i = 0; i < SPL; ++i) rf[c][i] = (double)r[c][i];
  }

  const double g = maybe_uni<UNI>(cst(p.gtab)[j]);
  const unsigned fx = maybe_uni<UNI>((unsigned)cst(p.fixed)[node]);
  double un[3][SPL];
  double uo[3][SPL];  // u_n as the QoI sees it
  if constexpr (MODE == kStateF64) {
#pragma unroll
    for (int c = 0; c < 3; ++c)
#pragma unroll
      for (int i = 0; i < SPL; ++i) uo[c][i] = ua[c][i];
    double minv[SPL];
    if constexpr (HOIST) {
#pragma unroll
      for (int i = 0; i < SPL; ++i) minv[i] = minv_h[i];
    } else if constexpr (std::is_same<AT, double>::value) {
      vload<SPL, true>(static_cast<const double*>(gen(p.minv)) + ms, minv);
    } else {
      float mf[SPL];
      vload<SPL, true>(static_cast<const float*>(gen(p.minv)) + ms, mf);
#pragma unroll
      for (int i = 0; i < SPL; ++i) minv[i] = (double)mf[i];
    }
    const double dt2 = p.dt * p.dt;
    const double inv1pa = 1.0 / (1.0 + p.a);
    const double oma = 1.0 - p.a;
#pragma unroll
    for (int c = 0; c < 3; ++c) {
      const int64_t idx = (row + c) * ld + s0;
      double up[SPL];
      if constexpr (HOIST) {
#pragma unroll
        for (int i = 0; i < SPL; ++i) up[i] = up_h[c][i];
      } else {
        vload<SPL, true>(gen(p.u_prev) + idx, up);
      }
      const double fc = g * maybe_uni<UNI>(cst(p.F)[row + c]);
#pragma unroll
      for (int i = 0; i < SPL; ++i) {
        double acc = (dt2 * minv[i]) * (fc - rf[c][i]);
        // explicit viscous force -c_d (u_n - u_{n-1}) / dt
        if (p.cd != 0.0) acc = fma(-(p.dt * minv[i] * p.cd), ua[c][i] - up[i], acc);
        double v = fma(-oma, up[i], fma(2.0, ua[c][i], acc)) * inv1pa;
        if (fx & (1u << c)) v = 0.0;
        un[c][i] = v;
      }
      vstore<SPL, true>(gen(p.u_next) + idx, un[c]);
    }
    if constexpr (ENERGY) {
#pragma unroll
      for (int i = 0; i < SPL; ++i) {
        const double m = 1.0 / minv[i];
#pragma unroll
        for (int c = 0; c < 3; ++c) {
          const double vel = (un[c][i] - ua[c][i]) / p.dt;
          e_loc[i] += 0.5 * m * vel * vel + 0.5 * un[c][i] * (double)r[c][i];
        }
      }
    }
  } else {
    // FP32 storage, FP64 arithmetic: the stored pair (or single value) and
    // velocity are widened, the velocity-form update is formed in FP64
    // with the exact coefficients, and the results are rounded once on the
    // way out.  F32_KAHAN keeps the rounding of u in the low part:
    // u_hi = fl32(u), u_lo = fl32(u_hi - u), so u = u_hi - u_lo carries
    // every increment's rounding (compensated summation, the increment
    // itself held exactly).
    float minv[SPL];
    vload<SPL, true>(static_cast<const float*>(gen(p.minv)) + ms, minv);
    const double inv1pa = 1.0 / (1.0 + p.a);
    const double oma = 1.0 - p.a;
#pragma unroll
    for (int c = 0; c < 3; ++c) {
      const int64_t idx = (row + c) * ld + s0;
      const double fc = g * maybe_uni<UNI>(cst(p.F)[row + c]);
      float vel[SPL], cc[SPL], uh[SPL];
      vload<SPL, true>(gen(p.v) + idx, vel);
      if constexpr (MODE == kStateF32Kahan) vload<SPL, true>(gen(p.uc) + idx, cc);
#pragma unroll
      for (int i = 0; i < SPL; ++i) {
        double u0 = (double)ua[c][i];
        if constexpr (MODE == kStateF32Kahan) u0 -= (double)cc[i];
        uo[c][i] = u0;
        const double m = (double)minv[i];
        const double v0 = (double)vel[i];
        double acc = m * (fc - (double)r[c][i]);
        // explicit viscous force -c_d v_{n-1/2}
        if (p.cd != 0.0) acc = fma(-(m * p.cd), v0, acc);
        const double vn = fma(p.dt, acc, oma * v0) * inv1pa;
        const double un_ = fma(p.dt, vn, u0);
        float hi = (float)un_;
        float lo = 0.0f;
        if constexpr (MODE == kStateF32Kahan) lo = (float)((double)hi - un_);
        float vf = (float)vn;
        if (fx & (1u << c)) {
          hi = 0.0f;
          lo = 0.0f;
          vf = 0.0f;
        }
        uh[i] = hi;
        cc[i] = lo;
        vel[i] = vf;
        un[c][i] = (double)hi - (double)lo;
        if constexpr (ENERGY) {
          e_loc[i] += 0.5 / m * (double)vf * (double)vf + 0.5 * un[c][i] * (double)r[c][i];
        }
      }
      vstore<SPL, true>(gen(p.uh_next) + idx, uh);
      if constexpr (MODE == kStateF32Kahan) vstore<SPL, true>(gen(p.uc) + idx, cc);
      vstore<SPL, true>(gen(p.v) + idx, vel);
    }
  }
  if constexpr (QOI) {
    const double e0 = maybe_uni<UNI>(cst(p.radial)[row + 0]);
    const double e1 = maybe_uni<UNI>(cst(p.radial)[row + 1]);
    const double e2 = maybe_uni<UNI>(cst(p.radial)[row + 2]);
    if constexpr (LPN == 64) {
      // q is only touched at local maxima: the bit records that the last
      // step raised the radial displacement; when a rise ends, its top
      // (the current value) is compared with q and kept if larger.  A rise
      // still open is folded in at read-back.
      constexpr int LPW = 64 / SPL;  // lanes per mask word
      uint64_t* __restrict__ mw = gen(p.qmask) + (int64_t)node * p.qwords + base / 64;
      uint64_t words[SPL];
#pragma unroll
      for (int w = 0; w < SPL; ++w) words[w] = w < nwords ? uni(mw[w]) : 0ull;
      uint64_t mine = words[0];
#pragma unroll
      for (int w = 1; w < SPL; ++w)
        if (lane / LPW == w) mine = words[w];
      uint64_t ballots[SPL];
#pragma unroll
      for (int i = 0; i < SPL; ++i) {
        const bool rose = (mine >> (SPL * (lane % LPW) + i)) & 1ull;
        const double rc = fma(e2, uo[2][i], fma(e1, uo[1][i], e0 * uo[0][i]));
        const double rn = fma(e2, un[2][i], fma(e1, un[1][i], e0 * un[0][i]));
        const bool rises = rn > rc;
        if (rose && !rises && rc > __builtin_nontemporal_load(gen(p.q) + ms + i))
          __builtin_nontemporal_store(rc, gen(p.q) + ms + i);
        ballots[i] = __ballot(rises);
      }
#pragma unroll
      for (int w = 0; w < SPL; ++w) {
        uint64_t nw = 0;
#pragma unroll
        for (int i = 0; i < SPL; ++i) nw |= spread_bits<SPL>(ballots[i] >> (w * LPW)) << i;
        if (w < nwords && nw != words[w] && lane == 0) mw[w] = nw;
      }
    } else {
      double qo[SPL];
      vload<SPL, true>(gen(p.q) + ms, qo);
      bool upd = false;
#pragma unroll
      for (int i = 0; i < SPL; ++i) {
        const double qv = fma(e2, un[2][i], fma(e1, un[1][i], e0 * un[0][i]));
        if (qv > qo[i]) {
          qo[i] = qv;
          upd = true;
        }
      }
      if (upd) vstore<SPL, true>(gen(p.q) + ms, qo);
    }
  }
}

// LPN lanes per node, SPL consecutive samples per lane: a workgroup covers
// StepBlock/LPN nodes times LPN*SPL samples.  With LPN = 64 a wave owns one
// node, so adjacency and stiffness blocks are wave-uniform (scalar loads).
template <typename AT, int MODE, int LPN, int SPL, bool QOI, bool ENERGY, bool SHARED, bool GEOM = false>
__global__ __launch_bounds__((StepBlock<AT, LPN, SPL, ENERGY, MODE == kStateF64>::value)) void k_step(StepArgs p) {
  constexpr int NPB = StepBlock<AT, LPN, SPL, ENERGY, MODE == kStateF64>::value / LPN;
  int nb, sbk;
  if (!wg_coords(p, nb, sbk)) return;  // uniform over the workgroup
  const int ln = threadIdx.x / LPN;
  const int lane = threadIdx.x % LPN;
  int node = nb * NPB + ln;
  if (LPN >= 64) node = __builtin_amdgcn_readfirstlane(node);
  double e_loc[SPL];
#pragma unroll
  for (int i = 0; i < SPL; ++i) e_loc[i] = 0.0;
  if (node < p.n_nodes)
    step_node<AT, MODE, LPN, SPL, QOI, ENERGY, SHARED, GEOM>(p, p.j, node, sbk * LPN * SPL, lane, e_loc);
  if constexpr (ENERGY) {
    __shared__ double red[kBlock * SPL];
#pragma unroll
    for (int i = 0; i < SPL; ++i) red[threadIdx.x * SPL + i] = e_loc[i];
    __syncthreads();
    if (ln == 0) {
      const int s0 = sbk * LPN * SPL + lane * SPL;
#pragma unroll
      for (int i = 0; i < SPL; ++i) {
        double sum = 0.0;
        for (int n = 0; n < NPB; ++n) sum += red[(n * LPN + lane) * SPL + i];
        gen(p.energy_part)[(int64_t)nb * p.ld + s0 + i] = sum;
      }
    }
  }
}

// Batched step: one launch per step for every mesh of a batch, one
// workgroup per tile (mesh, first node, node count <= 4, tail flag, first
// sample) of a list ordered mesh by mesh; workgroups are dealt to the 8
// XCDs so that each XCD takes a contiguous eighth of the list (tiles that
// share neighbours run close in time on one L2).  Each wave takes one node
// of its tile (no loop: a node loop keeps hoisted addresses live and costs
// a wave per SIMD) with 64 lanes x SPL samples.  A tail tile holds the
// last samples of a mesh when no full block remains (64 or 32 at SPL = 2,
// where a remainder of 96 runs as one block on 48 lanes instead; 32 at
// SPL = 1 for a padded width that is an odd multiple of 32) and runs one
// sample per lane on as many lanes (one kernel, one register budget).
// Per-mesh arguments come from a device table indexed by mesh and by the
// parity of the step (which state buffer is current).
template <typename AT, int MODE, int SPL, bool QOI>
__global__ __launch_bounds__(kBlock) void k_batch_step(const BatchTile* __restrict__ tiles, int32_t n_tiles,
                                                       const StepArgs* __restrict__ desc, int32_t j) {
  const int wave = threadIdx.x / 64;
  const int lane = threadIdx.x % 64;
  const int x = blockIdx.x & 7, rank = blockIdx.x >> 3;
  const int t = (int)(((int64_t)n_tiles * x) >> 3) + rank;
  if (t >= (int)(((int64_t)n_tiles * (x + 1)) >> 3)) return;  // uniform over the workgroup
  // tile and mesh arguments are uniform: keep them in scalar registers
  const ConstPtr<BatchTile> tile = cst(tiles) + t;
  const int mesh = __builtin_amdgcn_readfirstlane(tile->mesh);
  const int cw = __builtin_amdgcn_readfirstlane(tile->count);
  if (wave >= (cw & kTileCount)) return;
  const int node = __builtin_amdgcn_readfirstlane(tile->node0 + wave);
  const int sample0 = __builtin_amdgcn_readfirstlane(tile->sample0);
  // the mesh's arguments are read in place (scalar loads where they are
  // used) rather than copied: a copy holds them all in registers
  const StepArgs& p = *(const StepArgs*)(cst(desc) + 2 * mesh + (j & 1));
  // a tail tile covers min(64, ld - sample0) samples, one per lane, within
  // the block's first rising-bit word (in a launch with 2 samples per lane
  // the tails take the one-sample code path, so they interleave with the
  // full blocks in one launch)
  if (cw & kTileTail) {
    double e1[1];
    if (lane < min(64, p.ld - sample0))
      step_node<AT, MODE, 64, 1, QOI, false, false, false, true>(p, j, node, sample0, lane, e1, 1);
    return;
  }
  // a block of 64 < n < 128 samples (a padded width of 96 more than a
  // multiple of 128) runs at two samples per lane on n / 2 lanes
  const int rem = p.ld - sample0;
  double e_loc[SPL];
  if (SPL == 1 || rem >= 64 * SPL)
    step_node<AT, MODE, 64, SPL, QOI, false, false, false, true>(p, j, node, sample0, lane, e_loc, SPL);
  else if (lane < rem / SPL)
    step_node<AT, MODE, 64, SPL, QOI, false, false, false, true>(p, j, node, sample0, lane, e_loc, (rem + 63) / 64);
}

// Stand-alone apply; with MAP the rows of U and R are in the numbering
// given by map (internal node -> buffer node).
template <typename AT, int LPN, int SPL, bool SHARED, bool MAP>
__global__ __launch_bounds__((StepBlock<AT, LPN, SPL>::value)) void k_apply(StepArgs p, const AT* __restrict__ U,
                                                  AT* __restrict__ R, const int32_t* __restrict__ map) {
  constexpr int SB = LPN * SPL;
  constexpr int NPB = StepBlock<AT, LPN, SPL>::value / LPN;
  int nb, sbk;
  if (!wg_coords(p, nb, sbk)) return;
  int node = nb * NPB + (int)(threadIdx.x / LPN);
  if (LPN >= 64) node = __builtin_amdgcn_readfirstlane(node);
  if (node >= p.n_nodes) return;
  const int s0 = sbk * SB + (int)(threadIdx.x % LPN) * SPL;
  const int64_t ld = p.ld;
  const int64_t row = node_row<MAP>(map, node);
  AT ua[3][SPL];
#pragma unroll
  for (int c = 0; c < 3; ++c) vload<SPL, false>(U + (row + c) * ld + s0, ua[c]);
  AT r[3][SPL];
  if constexpr (SHARED) gather_blocks<AT, AT, SPL, (LPN == 64), MAP>(p, node, ld, s0, U, ua, r, map);
  // the apply's 4 samples per lane already hold many registers: no fan-closing reuse
  else gather_apply<AT, AT, SPL, (LPN == 64), MAP, false>(p, node, ld, s0, U, ua, r, map);
#pragma unroll
  for (int c = 0; c < 3; ++c) vstore<SPL, true>(R + (row + c) * ld + s0, r[c]);
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

__global__ __launch_bounds__(256) void k_copy_f64(int64_t n, const double* __restrict__ src,
                                                  double* __restrict__ dst) {
  for (int64_t i = (int64_t)blockIdx.x * 256 + threadIdx.x; i < n; i += (int64_t)gridDim.x * 256) dst[i] = src[i];
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

// Kinetic energy per sample in node chunks (fixed order), for the watchdog.
__global__ __launch_bounds__(64) void k_kinetic_part(int32_t n_nodes, int32_t ld, int32_t chunks,
                                                     const double* __restrict__ un1, const double* __restrict__ un,
                                                     const float* __restrict__ vel, const double* __restrict__ minv,
                                                     double inv_dt, double* __restrict__ tmp) {
  const int s = blockIdx.x * 64 + threadIdx.x;
  const int ch = blockIdx.y;
  if (s >= ld) return;
  const int per = (n_nodes + chunks - 1) / chunks;
  const int i0 = ch * per, i1 = min(n_nodes, i0 + per);
  double sum = 0.0;
  for (int i = i0; i < i1; ++i) {
    const double m = 1.0 / minv[(int64_t)i * ld + s];
    double v2 = 0.0;
    for (int c = 0; c < 3; ++c) {
      const int64_t idx = ((int64_t)i * 3 + c) * ld + s;
      const double v = vel ? (double)vel[idx] : (un1[idx] - un[idx]) * inv_dt;
      v2 = fma(v, v, v2);
    }
    sum = fma(0.5 * m, v2, sum);
  }
  tmp[(int64_t)ch * ld + s] = sum;
}

__global__ __launch_bounds__(64) void k_watch(int32_t S, const double* __restrict__ krow,
                                              const double* __restrict__ erow, double coef,
                                              int32_t* __restrict__ flag) {
  const int s = blockIdx.x * 64 + threadIdx.x;
  if (s >= S) return;
  const double T = krow[s], E = erow[s];
  if (!(coef * T <= E + 1e-12 * T)) *flag = 1;  // also trips on NaN
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
                                                     double alpha, double cd) {
  const int64_t t = (int64_t)blockIdx.x * 256 + threadIdx.x;
  if (t >= (int64_t)n_nodes * 3 * ld) return;
  const int64_t row = t / ld;
  const int s = (int)(t % ld);
  const int64_t node = row / 3;
  const int c = (int)(row % 3);
  const double v0 = vprev[t];
  const double acc = minv[node * ld + s] * (gtab[0] * F[row] - R[t] - cd * v0) - alpha * v0;
  double um = u0[t] - dt * v0 + 0.5 * dt * dt * acc;
  if (fixed[node] & (1u << c)) um = 0.0;
  vprev[t] = um;
}

// Starter in velocity form: v_{-1/2} = v_0 - dt/2 (m^-1 (g_0 F - K u_0 - c_d v_0) - alpha v_0).
__global__ __launch_bounds__(256) void k_starter_f32(int32_t n_nodes, int32_t ld,
                                                     const float* __restrict__ R,
                                                     const float* __restrict__ minv,
                                                     const double* __restrict__ F,
                                                     const uint8_t* __restrict__ fixed,
                                                     float* __restrict__ v,
                                                     const double* __restrict__ gtab, double dt,
                                                     double alpha, double cd) {
  const int64_t t = (int64_t)blockIdx.x * 256 + threadIdx.x;
  if (t >= (int64_t)n_nodes * 3 * ld) return;
  const int64_t row = t / ld;
  const int s = (int)(t % ld);
  const int64_t node = row / 3;
  const int c = (int)(row % 3);
  const double v0 = (double)v[t];
  const double acc = (double)minv[node * ld + s] * (gtab[0] * F[row] - (double)R[t] - cd * v0) - alpha * v0;
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

// Fold the open rises into q: where a bit is set, q = max(q, the current
// radial displacement) (same operation order as the step kernel).
// Idempotent.
__global__ __launch_bounds__(256) void k_qoi_resolve(int32_t n_nodes, int32_t ld,
                                                     const double* __restrict__ radial,
                                                     const double* __restrict__ u,
                                                     const float* __restrict__ uh,
                                                     const float* __restrict__ uc,
                                                     double* __restrict__ q,
                                                     const uint64_t* __restrict__ qmask) {
  const int64_t t = (int64_t)blockIdx.x * 256 + threadIdx.x;
  if (t >= (int64_t)n_nodes * ld) return;
  const int64_t node = t / ld;
  const int s = (int)(t % ld);
  const int qwords = (ld + 63) / 64;
  const uint64_t word = qmask[node * qwords + s / 64];
  if (!((word >> (s % 64)) & 1ull)) return;
  double x[3];
  for (int c = 0; c < 3; ++c) {
    const int64_t idx = (node * 3 + c) * ld + s;
    if (u) x[c] = u[idx];
    else x[c] = (double)uh[idx] - (uc ? (double)uc[idx] : 0.0);
  }
  const double* e = radial + node * 3;
  const double r = fma(e[2], x[2], fma(e[1], x[1], e[0] * x[0]));
  if (r > q[t]) q[t] = r;
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
// With out_row the results of node i go to row out_row[i] (the caller's
// numbering), else to row i.
__global__ __launch_bounds__(64) void k_moments(int32_t n_nodes, int32_t ld, int32_t S,
                                                const double* __restrict__ q,
                                                double* __restrict__ mean,
                                                double* __restrict__ var,
                                                const int32_t* __restrict__ out_row) {
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
    const int64_t o = out_row ? (int64_t)out_row[node] : (int64_t)node;
    mean[o] = mu;
    var[o] = S > 1 ? ss / (S - 1) : 0.0;
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

// The arguments with the node-block count of a workgroup of blk threads
// at lpn lanes per node.
inline StepArgs with_blocks(const StepArgs& a, int blk, int lpn) {
  StepArgs b = a;
  const int npb = blk / lpn;
  b.n_nb = (int32_t)((a.n_nodes + npb - 1) / npb);
  return b;
}

template <typename AT, int MODE, int LPN, int SPL, bool QOI, bool ENERGY, bool SH, bool GEOM = false>
void launch_k_step(const StepArgs& a, hipStream_t st) {
  constexpr int BLK = StepBlock<AT, LPN, SPL, ENERGY, MODE == kStateF64>::value;
  const StepArgs b = with_blocks(a, BLK, LPN);
  k_step<AT, MODE, LPN, SPL, QOI, ENERGY, SH, GEOM><<<step_grid(b), BLK, 0, st>>>(b);
}

template <typename AT, int MODE, int LPN, int SPL, bool SH>
hipError_t dispatch_flags(const StepArgs& a, bool qoi, bool energy, hipStream_t st) {
  if (qoi && energy) launch_k_step<AT, MODE, LPN, SPL, true, true, SH>(a, st);
  else if (qoi) launch_k_step<AT, MODE, LPN, SPL, true, false, SH>(a, st);
  else if (energy) launch_k_step<AT, MODE, LPN, SPL, false, true, SH>(a, st);
  else launch_k_step<AT, MODE, LPN, SPL, false, false, SH>(a, st);
  return hipGetLastError();
}

template <typename AT, int MODE, bool SH>
hipError_t dispatch_sb(const StepArgs& a, int sb, bool qoi, bool energy, hipStream_t st) {
  switch (sb) {
    case 8: return dispatch_flags<AT, MODE, 8, 1, SH>(a, qoi, energy, st);
    case 16: return dispatch_flags<AT, MODE, 16, 1, SH>(a, qoi, energy, st);
    case 32: return dispatch_flags<AT, MODE, 32, 1, SH>(a, qoi, energy, st);
    case 64: return dispatch_flags<AT, MODE, 64, 1, SH>(a, qoi, energy, st);
    case 128: return dispatch_flags<AT, MODE, 64, 2, SH>(a, qoi, energy, st);
    case 256: return dispatch_flags<AT, MODE, 64, 4, SH>(a, qoi, energy, st);
    default: return hipErrorInvalidValue;
  }
}

template <typename AT, int LPN, int SPL>
hipError_t dispatch_geom_flags(const StepArgs& a, bool qoi, hipStream_t st) {
  if (qoi) launch_k_step<AT, kStateF64, LPN, SPL, true, false, false, true>(a, st);
  else launch_k_step<AT, kStateF64, LPN, SPL, false, false, false, true>(a, st);
  return hipGetLastError();
}

template <typename AT>
hipError_t dispatch_geom(const StepArgs& a, int sb, bool qoi, hipStream_t st) {
  switch (sb) {
    case 8: return dispatch_geom_flags<AT, 8, 1>(a, qoi, st);
    case 16: return dispatch_geom_flags<AT, 16, 1>(a, qoi, st);
    case 32: return dispatch_geom_flags<AT, 32, 1>(a, qoi, st);
    case 64: return dispatch_geom_flags<AT, 64, 1>(a, qoi, st);
    case 128: return dispatch_geom_flags<AT, 64, 2>(a, qoi, st);
    case 256: return dispatch_geom_flags<AT, 64, 4>(a, qoi, st);
    default: return hipErrorInvalidValue;
  }
}

template <typename AT, int MODE>
hipError_t dispatch_shared(const StepArgs& a, int sb, bool qoi, bool energy, bool shared, hipStream_t st) {
  return shared ? dispatch_sb<AT, MODE, true>(a, sb, qoi, energy, st)
                : dispatch_sb<AT, MODE, false>(a, sb, qoi, energy, st);
}

template <typename AT, bool SH, bool MAP>
hipError_t dispatch_apply(const StepArgs& a, int sb, const void* U, void* R, const int32_t* map,
                          hipStream_t st) {
  const AT* u = static_cast<const AT*>(U);
  AT* r = static_cast<AT*>(R);
#define ENSFEM_APPLY(LPN, SPL)                                                           \
  do {                                                                                   \
    constexpr int blk = StepBlock<AT, LPN, SPL>::value;                                  \
    const StepArgs b = with_blocks(a, blk, LPN);                                         \
    k_apply<AT, LPN, SPL, SH, MAP><<<step_grid(b), blk, 0, st>>>(b, u, r, map);          \
  } while (0)
  switch (sb) {
    case 8: ENSFEM_APPLY(8, 1); break;
    case 16: ENSFEM_APPLY(16, 1); break;
    case 32: ENSFEM_APPLY(32, 1); break;
    case 64: ENSFEM_APPLY(64, 1); break;
    case 128: ENSFEM_APPLY(64, 2); break;
    case 256: ENSFEM_APPLY(64, 4); break;
    default: return hipErrorInvalidValue;
  }
#undef ENSFEM_APPLY
  return hipGetLastError();
}

template <typename AT, bool SH>
hipError_t dispatch_apply_map(const StepArgs& a, int sb, const void* U, void* R, const int32_t* map,
                              hipStream_t st) {
  return map ? dispatch_apply<AT, SH, true>(a, sb, U, R, map, st)
             : dispatch_apply<AT, SH, false>(a, sb, U, R, nullptr, st);
}

}  // namespace

hipError_t launch_step(const StepArgs& a, bool apply_f32, int mode, int sample_block, bool qoi,
                       bool energy, bool shared, hipStream_t st) {
  if (a.n_nb == 0 || a.n_sb == 0) return hipSuccess;
  if (a.usnap) {  // geometry form
    if (mode != kStateF64 || energy || shared) return hipErrorInvalidValue;
    return apply_f32 ? dispatch_geom<float>(a, sample_block, qoi, st) : dispatch_geom<double>(a, sample_block, qoi, st);
  }
  if (!apply_f32) {
    if (mode != kStateF64) return hipErrorInvalidValue;
    return dispatch_shared<double, kStateF64>(a, sample_block, qoi, energy, shared, st);
  }
  switch (mode) {
    case kStateF64: return dispatch_shared<float, kStateF64>(a, sample_block, qoi, energy, shared, st);
    case kStateF32Kahan:
      return dispatch_shared<float, kStateF32Kahan>(a, sample_block, qoi, energy, shared, st);
    case kStateF32: return dispatch_shared<float, kStateF32>(a, sample_block, qoi, energy, shared, st);
    default: return hipErrorInvalidValue;
  }
}

hipError_t launch_apply(const StepArgs& a, bool f32, int sample_block, bool shared, const void* U,
                        void* R, const int32_t* map, hipStream_t st) {
  if (a.n_nb == 0 || a.n_sb == 0) return hipSuccess;
  if (shared)
    return f32 ? dispatch_apply_map<float, true>(a, sample_block, U, R, map, st)
               : dispatch_apply_map<double, true>(a, sample_block, U, R, map, st);
  return f32 ? dispatch_apply_map<float, false>(a, sample_block, U, R, map, st)
             : dispatch_apply_map<double, false>(a, sample_block, U, R, map, st);
}

hipError_t launch_batch_step(const BatchTile* tiles, int32_t n_tiles, int spl, const StepArgs* desc, int32_t j,
                             bool apply_f32, int mode, bool qoi, hipStream_t st) {
  if (n_tiles == 0) return hipSuccess;
  if (n_tiles < 0 || (spl != 1 && spl != 2)) return hipErrorInvalidValue;
  // One workgroup per tile: eight equal slices of workgroups (one per XCD
  // under round-robin dispatch), each covering a contiguous eighth of the
  // tile list.
  const int grid = (int)(((int64_t)n_tiles + 7) / 8 * 8);
#define ENSFEM_BATCH_Q(AT, MODE, SPL)                                                                     \
  do {                                                                                                    \
    if (qoi) k_batch_step<AT, MODE, SPL, true><<<grid, kBlock, 0, st>>>(tiles, n_tiles, desc, j); \
    else k_batch_step<AT, MODE, SPL, false><<<grid, kBlock, 0, st>>>(tiles, n_tiles, desc, j);   \
  } while (0)
#define ENSFEM_BATCH(AT, MODE)                  \
  do {                                          \
    if (spl == 2) ENSFEM_BATCH_Q(AT, MODE, 2);  \
    else ENSFEM_BATCH_Q(AT, MODE, 1);           \
    return hipGetLastError();                   \
  } while (0)
  if (!apply_f32) {
    if (mode != kStateF64) return hipErrorInvalidValue;
    ENSFEM_BATCH(double, kStateF64);
  }
  if (mode == kStateF64) ENSFEM_BATCH(float, kStateF64);
  if (mode == kStateF32Kahan) ENSFEM_BATCH(float, kStateF32Kahan);
  if (mode == kStateF32) ENSFEM_BATCH(float, kStateF32);
#undef ENSFEM_BATCH
#undef ENSFEM_BATCH_Q
  return hipErrorInvalidValue;
}

hipError_t launch_schedule(double* gtab, int64_t* base, int32_t k, double dt, Schedule s,
                           hipStream_t st) {
  k_schedule<<<1, 256, 0, st>>>(gtab, base, k, dt, s);
  return hipGetLastError();
}

hipError_t launch_copy_f64(int64_t n, const double* src, double* dst, hipStream_t st) {
  if (n == 0) return hipSuccess;
  const unsigned g = (unsigned)std::min<int64_t>(grid_for(n, 256), 65536);
  k_copy_f64<<<g, 256, 0, st>>>(n, src, dst);
  return hipGetLastError();
}

hipError_t launch_advance(int64_t* base, int32_t k, hipStream_t st) {
  k_advance<<<1, 64, 0, st>>>(base, k);
  return hipGetLastError();
}

hipError_t launch_kinetic(int32_t n_nodes, int32_t ld, int32_t S, const double* u_next, const double* u_cur,
                          const float* vel, const double* minv, double dt, double* tmp, double* krow,
                          const double* erow, double coef, int32_t* flag, hipStream_t st) {
  const int chunks = 256;
  dim3 g1(grid_for(ld, 64), chunks);
  k_kinetic_part<<<g1, 64, 0, st>>>(n_nodes, ld, chunks, u_next, u_cur, vel, minv, 1.0 / dt, tmp);
  k_energy_reduce2<<<grid_for(S, 64), 64, 0, st>>>(tmp, chunks, ld, S, krow);
  k_watch<<<grid_for(S, 64), 64, 0, st>>>(S, krow, erow, coef, flag);
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
                              double cd, hipStream_t st) {
  const int64_t n = (int64_t)n_nodes * 3 * ld;
  if (n == 0) return hipSuccess;
  k_starter_f64<<<grid_for(n, 256), 256, 0, st>>>(n_nodes, ld, R, minv, F, fixed, u0, vprev_io,
                                                   gtab, dt, alpha, cd);
  return hipGetLastError();
}

hipError_t launch_starter_f32(int32_t n_nodes, int32_t ld, const float* R, const float* minv,
                              const double* F, const uint8_t* fixed, float* v_io,
                              const double* gtab, double dt, double alpha, double cd, hipStream_t st) {
  const int64_t n = (int64_t)n_nodes * 3 * ld;
  if (n == 0) return hipSuccess;
  k_starter_f32<<<grid_for(n, 256), 256, 0, st>>>(n_nodes, ld, R, minv, F, fixed, v_io, gtab, dt,
                                                   alpha, cd);
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

hipError_t launch_qoi_resolve(int32_t n_nodes, int32_t ld, const double* radial, const double* u_f64,
                              const float* uh, const float* uc, double* q, const uint64_t* qmask,
                              hipStream_t st) {
  const int64_t n = (int64_t)n_nodes * ld;
  if (n == 0) return hipSuccess;
  k_qoi_resolve<<<grid_for(n, 256), 256, 0, st>>>(n_nodes, ld, radial, u_f64, uh, uc, q, qmask);
  return hipGetLastError();
}

hipError_t launch_combine_f32(int64_t n, const float* uh, const float* uc, double* out,
                              hipStream_t st) {
  if (n == 0) return hipSuccess;
  k_combine_f32<<<grid_for(n, 256), 256, 0, st>>>(n, uh, uc, out);
  return hipGetLastError();
}

hipError_t launch_moments(int32_t n_nodes, int32_t ld, int32_t S, const double* q, double* mean,
                          double* var, const int32_t* out_row, hipStream_t st) {
  if (n_nodes == 0) return hipSuccess;
  k_moments<<<n_nodes, 64, 0, st>>>(n_nodes, ld, S, q, mean, var, out_row);
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
