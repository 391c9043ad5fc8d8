// Internal declarations shared by the host API and the kernel translation
// units of libensfem.  Each .hip file launches only its own kernels through
// the launch_* wrappers declared here, so no relocatable device code is
// needed.
#pragma once

#include <hip/hip_runtime.h>

#include <cstddef>
#include <cstdint>

namespace ensfem {

constexpr int kBlock = 256;       // threads per workgroup for the ensemble kernels
// Workgroup of the single-mesh step and apply kernels: 512 threads (8
// nodes of 64 lanes) for the FP32 apply with 2 or 4 samples per lane and
// the FP64 state (and the stand-alone apply), whose eight neighbouring
// nodes per workgroup share neighbour rows in L1 (2 % faster on the
// headline step); kBlock otherwise (the FP64 apply's 5 waves per SIMD
// would leave a CU 16 waves instead of 20 at 512; smaller sample blocks
// and the FP32 states measured slower), and always for the steps that
// record energy, whose per-workgroup partial sums then group the same
// nodes whatever the sample block.  The host's node-block count (energy
// partials) is the kBlock one; each launch derives its own grid.
template <typename AT, int LPN, int SPL, bool ENERGY = false, bool F64_STATE = true>
struct StepBlock {
  static constexpr int value = (sizeof(AT) == 4 && LPN == 64 && SPL >= 2 && !ENERGY && F64_STATE) ? 512 : kBlock;
};
// Batch tile order within a mesh: 1 node tile by node tile with its sample
// blocks together (a node's stiffness blocks are reused from L2 by its
// other sample blocks), 0 sample block by sample block.
#ifndef ENSFEM_BATCH_NODE_MAJOR
#define ENSFEM_BATCH_NODE_MAJOR 1
#endif
// The element that closes a node's fan takes the walk's first neighbour
// from registers instead of loading it again (host marking and kernels).
#ifndef ENSFEM_CLOSE_REUSE
#define ENSFEM_CLOSE_REUSE 1
#endif
constexpr int kEnergyCap = 4096;  // energy records kept (ring)

// Device arrays referenced from argument structs are global memory; the
// qualifier keeps that knowledge when a struct is read from a device table
// (plain pointers loaded from memory are generic to the compiler).
#define ENS_GLOBAL __attribute__((address_space(1)))

template <class T>
__host__ __device__ inline ENS_GLOBAL T* gptr(T* p) {
  return (ENS_GLOBAL T*)p;
}

// Load-schedule kinds (mirror the public enum).
struct Schedule {
  int kind;
  double t_ramp, amp, period;
};

// Node-gather adjacency: for node i, entries adj_ptr[i] .. adj_ptr[i+1]-1,
// one per incident element e, with the element's other two nodes (b, c) in
// cyclic order after i and the 3x6 block [Khat_ib | Khat_ic] (global frame).
// Entries walk around the node; nb.x < 0 (stored as ~b) marks an entry whose
// b is the previous entry's c, nb.y < 0 (stored as ~c) the last entry of a
// closed fan, whose c is the first entry's b.
struct Adjacency {
  ENS_GLOBAL const int32_t* ptr;
  ENS_GLOBAL const int32_t* el;
  ENS_GLOBAL const int2* nb;
  ENS_GLOBAL const void* k;  // double[18] or float[18] per entry
};

// Shared-stiffness block rows (used when (E h)_{e,s} does not depend on s):
// for node i, blocks ptr[i] .. ptr[i+1]-1 hold K_ij (3x3, row-major) for
// every neighbour j != i, with the diagonal block implied by the rows'
// translation null space: (K u)_i = sum_j K_ij (u_j - u_i).
struct BlockRows {
  ENS_GLOBAL const int32_t* ptr;
  ENS_GLOBAL const int32_t* col;
  ENS_GLOBAL const void* val;  // double[9] or float[9] per block
};

// State storage modes.
enum StateMode { kStateF64 = 0, kStateF32Kahan = 1, kStateF32 = 2 };

struct StepArgs {
  int32_t n_nodes;
  int32_t ld;          // padded sample count (row stride of every ensemble array)
  int32_t n_nb;        // node blocks
  int32_t n_sb;        // sample blocks
  int32_t sb_inner;    // workgroup order: sample block fastest (1) or node block fastest (0)
  Adjacency adj;
  BlockRows bsr;
  ENS_GLOBAL const void* eh;      // (E h)_{e,s} in the apply precision, [n_el][ld]
  ENS_GLOBAL const void* minv;    // 1/m per node and sample, double (F64 apply) or float, [n_nodes][ld]
  ENS_GLOBAL const double* F;     // nodal load [n_nodes][3]
  ENS_GLOBAL const uint8_t* fixed;   // clamped-dof bits per node
  ENS_GLOBAL const double* radial;   // [n_nodes][3]
  // FP64 two-level state
  ENS_GLOBAL const double* u_cur;
  ENS_GLOBAL const double* u_prev;
  ENS_GLOBAL double* u_next;
  // FP32 velocity-form state
  ENS_GLOBAL const float* uh_cur;
  ENS_GLOBAL float* uh_next;
  ENS_GLOBAL float* uc;           // Kahan compensation (in place)
  ENS_GLOBAL float* v;            // velocity v_{n-1/2} -> v_{n+1/2} (in place)
  ENS_GLOBAL double* q;           // running peak radial displacement [n_nodes][ld]
  // Rising bits (wave-per-node kernels): bit set <=> the last step raised
  // the sample's radial displacement; q holds the maximum of the initial
  // value and every completed rise's top, an open rise is folded in at
  // read-back.  Per node ceil(ld/64) words; sample s in word s/64, bit s%64.
  ENS_GLOBAL uint64_t* qmask;
  int32_t qwords;
  ENS_GLOBAL const double* gtab;  // load factors of the current chunk
  int32_t j;           // index into gtab
  double dt, a;        // step, alpha dt / 2
  double cd;           // explicit viscous force coefficient (0: none)
  ENS_GLOBAL double* energy_part; // [n_nb][ld] per node-block energy partial sums
  // Geometry form (usnap non-null): force R_m + K(x + u_m) (u_n - u_m)
  // with u_m the displacement of the last refresh.
  ENS_GLOBAL const double* usnap; // u_m [n_nodes*3][ld]
  ENS_GLOBAL double* rbase;       // R_m [n_nodes*3][ld]
  ENS_GLOBAL const double* xyz;   // reference coordinates [n_nodes][3]
  double nu, shear_k;
  int32_t refresh;                // 1: this step moves the base (R_m <- the force at u_n)
  int32_t pad_;
};

// One work item of the batched step: nodes node0 .. node0 + (count &
// kTileCount) - 1 of mesh `mesh` (at most 4, one per wave), samples from
// sample0: a full block of 64 * spl (spl fixed per launch; at spl = 2 a
// mesh's last 96 samples also form one block, on 48 lanes) or, with
// kTileTail set in count, a mesh's last min(64, ld - sample0).
struct BatchTile {
  int32_t mesh;
  int32_t node0;
  int32_t count;
  int32_t sample0;
};
constexpr int32_t kTileCount = 0xff;
constexpr int32_t kTileTail = 0x100;

// ---- set-up kernels (setup.hip) -------------------------------------------
// Doubles per element in the frame table written by the element set-up:
// rows e_x, e_y, e_z of the local frame (9), dN_j/dx (3), dN_j/dy (3), pad.
constexpr int kFrameWords = 16;

hipError_t launch_element_setup(int64_t n_el, const double* xyz, const int32_t* tri, double nu,
                                double shear_k, double* khat, double* area, double* lam,
                                double* frame, int32_t* bad, hipStream_t st);
hipError_t launch_adjacency_blocks(int64_t n_adj, const int32_t* adj_el, const uint8_t* adj_loc,
                                   const double* khat, double* k64, float* k32, hipStream_t st);
// Nodal 1/m per sample; dt_t > 0 scales each element's density by
// max(1, omega^2 dt_t^2 / 4) (mass scaling), 0 leaves it.
hipError_t launch_lumped_mass(int32_t n_nodes, int32_t ld, const int32_t* adj_ptr,
                              const int32_t* adj_el, const double* area, const double* h, double rho,
                              const double* eh, const double* lam, double dt_t, double* minv64, float* minv32,
                              hipStream_t st);
hipError_t launch_cfl_max(int64_t n_el, int32_t ld, int32_t S, const double* eh, const double* h,
                          const double* lam, const double* area, double rho, double dt_t,
                          unsigned long long* out_bits, hipStream_t st);
hipError_t launch_cast_f32(int64_t n, const double* src, float* dst, hipStream_t st);
hipError_t launch_bsr_assemble(int32_t n_nodes, int32_t ld, const int32_t* adj_ptr,
                               const int32_t* adj_el, const uint8_t* adj_loc, const int2* adj_slot,
                               const int32_t* bsr_ptr, const double* khat, const double* eh,
                               double* bsr64, hipStream_t st);

// ---- time-stepping kernels (step.hip) -------------------------------------
// One explicit step of the node-gather fused kernel.  apply_f32 selects
// the apply precision; mode the state storage; qoi / energy the outputs.
hipError_t launch_step(const StepArgs& a, bool apply_f32, int mode, int sample_block, bool qoi,
                       bool energy, bool shared, hipStream_t st);
// Stand-alone R = K U; map (internal node -> buffer node) or null when U and
// R are in the internal numbering.
hipError_t launch_apply(const StepArgs& a, bool f32, int sample_block, bool shared, const void* U,
                        void* R, const int32_t* map, hipStream_t st);
hipError_t launch_schedule(double* gtab, int64_t* base, int32_t k, double dt, Schedule s,
                           hipStream_t st);
hipError_t launch_copy_f64(int64_t n, const double* src, double* dst, hipStream_t st);
hipError_t launch_advance(int64_t* base, int32_t k, hipStream_t st);
// Energy watchdog of one record: T_s = sum over nodes of 1/2 m |v|^2 per
// sample (v = (u_next - u_cur) / dt for the FP64 state, the stored velocity
// otherwise), through chunk partials in tmp [256][ld] into krow [S]; then
// *flag = 1 if coef T_s > E_s + 1e-12 T_s for some sample (E_s = erow[s]).
hipError_t launch_kinetic(int32_t n_nodes, int32_t ld, int32_t S, const double* u_next, const double* u_cur,
                          const float* vel, const double* minv, double dt, double* tmp, double* krow,
                          const double* erow, double coef, int32_t* flag, hipStream_t st);
hipError_t launch_energy_reduce(const double* part, int32_t n_nb, int32_t ld, int32_t S,
                                double* out_row, hipStream_t st);
hipError_t launch_starter_f64(int32_t n_nodes, int32_t ld, const double* R, const double* minv,
                              const double* F, const uint8_t* fixed, const double* u0,
                              double* vprev_io, const double* gtab, double dt, double alpha,
                              double cd, hipStream_t st);
hipError_t launch_starter_f32(int32_t n_nodes, int32_t ld, const float* R, const float* minv,
                              const double* F, const uint8_t* fixed, float* v_io,
                              const double* gtab, double dt, double alpha, double cd, hipStream_t st);
hipError_t launch_split_f32(int64_t n, const double* u0, float* uh, float* uc, hipStream_t st);
hipError_t launch_qoi_init(int32_t n_nodes, int32_t ld, const double* radial, const double* u_f64,
                           const float* uh, const float* uc, double* q, hipStream_t st);
// spl samples per lane; tail tiles (kTileTail) hold min(64, ld - sample0)
// samples run on the lower lanes of a wave
hipError_t launch_batch_step(const BatchTile* tiles, int32_t n_tiles, int spl, const StepArgs* desc, int32_t j,
                             bool apply_f32, int mode, bool qoi, hipStream_t st);
// Folds each sample's open rise (its rising bit) into q.
hipError_t launch_qoi_resolve(int32_t n_nodes, int32_t ld, const double* radial, const double* u_f64,
                              const float* uh, const float* uc, double* q, const uint64_t* qmask,
                              hipStream_t st);
hipError_t launch_combine_f32(int64_t n, const float* uh, const float* uc, double* out,
                              hipStream_t st);
// out_row: optional row of each node in the outputs (nullptr: node i -> row i)
hipError_t launch_moments(int32_t n_nodes, int32_t ld, int32_t S, const double* q, double* mean,
                          double* var, const int32_t* out_row, hipStream_t st);
hipError_t launch_check_finite(int64_t n, const void* x, int is_f32, int32_t* flag,
                               hipStream_t st);

// ---- stress post-processing (stress.hip) ------------------------------------
// Component comp (0 theta-theta, 1 z-z, 2 theta-z, 3 r-z) of the wall stress
// in the cylindrical frame per element and sample, from the current state
// (u: FP64 state, or uh - uc for the FP32 states); axial [n_el][3] centreline
// tangents (internal element order); out [n_el][ld].  bad is set if a
// tangent is (numerically) parallel to its element's normal.
hipError_t launch_stress(int64_t n_el, int32_t ld, const int32_t* tri, const double* frame,
                         const double* u, const float* uh, const float* uc, const double* eh,
                         const double* h, const double* axial, double nu, double shear_k, int comp,
                         double* out, int32_t* bad, hipStream_t st);
// Per row of vals [n_rows][ld] (first S columns): mean and the p_lo / p_hi
// quantiles (linear interpolation between order statistics at p (S - 1)).
// S <= kBandsMax.
constexpr int kBandsMax = 4096;
hipError_t launch_bands(int64_t n_rows, int32_t ld, int32_t S, const double* vals, double p_lo, double p_hi,
                        double* mean, double* lo, double* hi, hipStream_t st);

}  // namespace ensfem
