// Host side of libensfem: the C ABI declared in include/ensfem.h, argument
// checking, the mesh adjacency and workspace planners, uploads, the step
// driver and read-backs.  All arithmetic of the method runs in the kernels
// of setup.hip and step.hip.
#include "ensfem.h"
#include "internal.h"

#include <algorithm>
#include <cmath>
#include <cstdio>
#include <cstring>
#include <exception>
#include <mutex>
#include <new>
#include <string>
#include <vector>

using namespace ensfem;

namespace {

// Scratch of the allocation-free entry point (ens_moments_noalloc): a
// file-scope device array, one copy per GPU, held until the process ends.
// Host code never passes the array's name to a kernel or a copy (on the
// host it only names the symbol); it uses the device address looked up once
// per device with hipGetSymbolAddress.
constexpr size_t kScratchBytes = size_t(16) << 20;
constexpr int kMaxDevices = 64;
static __device__ __align__(256) unsigned char scratch[kScratchBytes];
std::mutex g_scratch_mu;
void* g_scratch_ptr[kMaxDevices] = {};

// Device address of `scratch` on `device`, which must be current.
hipError_t scratch_setup(int device) {
  if (device < 0 || device >= kMaxDevices) return hipErrorInvalidDevice;
  std::lock_guard<std::mutex> lk(g_scratch_mu);
  if (g_scratch_ptr[device]) return hipSuccess;
  void* ptr = nullptr;
  const hipError_t e = hipGetSymbolAddress(&ptr, HIP_SYMBOL(scratch));
  if (e != hipSuccess) return e;
  if (!ptr) return hipErrorInvalidSymbol;
  g_scratch_ptr[device] = ptr;
  return hipSuccess;
}

void* scratch_ptr(int device) {
  if (device < 0 || device >= kMaxDevices) return nullptr;
  std::lock_guard<std::mutex> lk(g_scratch_mu);
  return g_scratch_ptr[device];
}

constexpr size_t kAlign = 256;
constexpr int kChunk = 1024;  // steps per load-factor table
constexpr int kGraphSteps = 64;  // steps per captured graph (even: keeps the state parity)
static_assert(kGraphSteps % 2 == 0 && kGraphSteps <= kChunk, "graph chunk");

size_t align_up(size_t x) { return (x + kAlign - 1) & ~(kAlign - 1); }

struct Layout {
  size_t xyz, tri, khat, area, lam, flags, adj_ptr, adj_el, adj_nb, adj_loc, k64, k32, fixed,
      radial, perm, F, eh64, eh32, h, minv64, minv32, u[2], uh[2], uc, v, usnap, rbase, q, qmask, bsr_ptr, bsr_col,
      adj_slot, bsr64, bsr32, epart, erec, gtab, base, frame, stress,
      mean, var, aux, total;
};

struct Flags {  // small device scalars
  int32_t bad;
  int32_t nonfinite;
  int32_t unstable;  // energy watchdog fired since the state was set
  int32_t pad_;
  unsigned long long omega2_bits;
};

}  // namespace

struct ens_ctx {
  int device = 0;
  std::string err;
  // mesh
  int64_t n_nodes = 0, n_el = 0;
  std::vector<double> xyz, radial;
  std::vector<int32_t> tri;
  std::vector<uint8_t> fixed;  // bits per node
  // internal numbering: node i is the caller's node perm[i], element e the
  // caller's element eperm[e]
  std::vector<int32_t> perm, eperm;
  bool have_mesh = false;
  // adjacency
  std::vector<int32_t> adj_ptr, adj_el;
  std::vector<int2> adj_nb;
  std::vector<uint8_t> adj_loc;
  // shared-stiffness block rows (off-diagonal neighbours per node)
  std::vector<int32_t> bsr_ptr, bsr_col;
  std::vector<int2> adj_slot;
  // material
  double nu = 0.49, shear_k = 5.0 / 6.0, rho = 1.0, alpha = 0.0;
  double cd = 0.0;       // explicit viscous force coefficient
  double mass_dt = 0.0;  // mass-scaling target step (0: none)
  int32_t geom_every = 0;  // geometry refresh interval in steps (0: reference geometry)
  bool have_material = false;
  // ensemble (padded [n_el][ld])
  int32_t S = 0, ld = 0, SB = 0;
  std::vector<double> eh, h;
  bool have_ens = false, shared = false;
  // load
  std::vector<double> F;
  Schedule sched{0, 0.0, 0.0, 1.0};
  bool have_load = false;
  // configuration
  int32_t apply_prec = ENS_F64, state_prec = ENS_STATE_F64, variant = ENS_VARIANT_AUTO;
  int32_t qoi_mask = ENS_QOI_PEAK_RADIAL, energy_every = 0;
  int32_t tune_sb = 0, sb_inner = 0;
  // device
  char* ws = nullptr;
  size_t ws_bytes = 0;
  Layout L{};
  bool bound = false;
  double omega2 = 0.0;
  // state
  bool state_init = false, started = false, u0_zero = true;
  // rising bits may be set: wave-per-node steps (padded width >= 64) and
  // batched steps track the peak through them, lane-group steps do not
  bool mask_live = false;
  int cur = 0;
  double dt = 0.0;
  int64_t steps = 0;
  int64_t energy_records = 0;
  std::vector<int64_t> energy_steps;
  hipStream_t last_stream = nullptr;
  uint64_t gen = 0;  // bumped by every change a captured step graph depends on
  // captured chunk of kGraphSteps plain steps (no energy records, reference
  // geometry), valid for the generation and state parity it was taken at
  hipStream_t cap_st = nullptr;
  hipGraph_t graph = nullptr;
  hipGraphExec_t exec = nullptr;
  uint64_t graph_gen = 0;
  int graph_cur = -1;

  void drop_graph() {
    if (exec) (void)hipGraphExecDestroy(exec);
    if (graph) (void)hipGraphDestroy(graph);
    exec = nullptr;
    graph = nullptr;
  }
  ~ens_ctx() {
    drop_graph();
    if (cap_st) (void)hipStreamDestroy(cap_st);
  }

  template <class T>
  T* p(size_t off) const { return reinterpret_cast<T*>(ws + off); }
  int32_t fail(int32_t code, const std::string& msg) {
    err = msg;
    return code;
  }
};

#define HIPC(expr)                                                                          \
  do {                                                                                      \
    hipError_t e_ = (expr);                                                                 \
    if (e_ != hipSuccess)                                                                   \
      return ctx->fail(ENS_EDEVICE, std::string("HIP error: ") + hipGetErrorString(e_) +    \
                                        " at " #expr);                                      \
  } while (0)

#define GUARD_BEGIN try {
#define GUARD_END                                                   \
  }                                                                 \
  catch (const std::bad_alloc&) {                                   \
    return ctx->fail(ENS_EINVAL, "host allocation failed");         \
  }                                                                 \
  catch (const std::exception& ex) {                                \
    return ctx->fail(ENS_EINVAL, ex.what());                        \
  }                                                                 \
  catch (...) {                                                     \
    return ctx->fail(ENS_EINVAL, "unknown error");                  \
  }

namespace {

// Samples per node handled by one workgroup pass: 8..64 lanes with one
// sample each, or 64 lanes with 2 or 4 consecutive samples each (128, 256).
// Auto: the widest block up to 128 that adds no padding beyond 64-sample
// granularity (128 measured fastest on MI355X for the 200k-node cylinder).
int pick_sample_block(int S, int requested) {
  if (requested == 8 || requested == 16 || requested == 32 || requested == 64 || requested == 128 ||
      requested == 256)
    return requested;
  if (S <= 64) {
    int sb = 8;
    while (sb < S) sb <<= 1;
    return sb;
  }
  const int64_t pad64 = ((S + 63) / 64) * 64;
  for (int sb = 128; sb > 64; sb >>= 1)
    if (((S + sb - 1) / sb) * (int64_t)sb <= pad64) return sb;
  return 64;
}

// nodes per workgroup for a sample block
// node blocks of a kBlock workgroup (the energy partials; each launch
// derives the grid of its own workgroup size)
int nodes_per_block(int SB) { return kBlock / (SB >= 64 ? 64 : SB); }

bool use_shared(const ens_ctx* c);

Layout plan(const ens_ctx* c) {
  Layout L{};
  size_t off = 0;
  auto take = [&](size_t bytes) {
    const size_t o = off;
    off = align_up(off + bytes);
    return o;
  };
  const int64_t nn = c->n_nodes, ne = c->n_el, nadj = 3 * ne, ld = c->ld;
  const int64_t ndof = 3 * nn;
  L.xyz = take(sizeof(double) * 3 * nn);
  L.tri = take(sizeof(int32_t) * 3 * ne);
  L.khat = take(sizeof(double) * 81 * ne);
  L.area = take(sizeof(double) * ne);
  L.lam = take(sizeof(double) * ne);
  L.frame = take(sizeof(double) * kFrameWords * ne);
  L.flags = take(sizeof(Flags));
  L.adj_ptr = take(sizeof(int32_t) * (nn + 1));
  L.adj_el = take(sizeof(int32_t) * nadj);
  L.adj_nb = take(sizeof(int2) * nadj);
  L.adj_loc = take(nadj);
  L.k64 = take(sizeof(double) * 18 * nadj);
  L.k32 = take(sizeof(float) * 18 * nadj);
  L.fixed = take(nn);
  L.radial = take(sizeof(double) * 3 * nn);
  L.perm = take(sizeof(int32_t) * nn);

  L.F = take(sizeof(double) * 3 * nn);
  L.eh64 = take(sizeof(double) * ne * ld);
  L.eh32 = take(sizeof(float) * ne * ld);
  L.h = take(sizeof(double) * ne * ld);
  L.minv64 = take(sizeof(double) * nn * ld);
  L.minv32 = take(sizeof(float) * nn * ld);
  if (c->state_prec == ENS_STATE_F64) {
    L.u[0] = take(sizeof(double) * ndof * ld);
    L.u[1] = take(sizeof(double) * ndof * ld);
  } else {
    L.uh[0] = take(sizeof(float) * ndof * ld);
    L.uh[1] = take(sizeof(float) * ndof * ld);
    if (c->state_prec == ENS_STATE_F32_KAHAN) L.uc = take(sizeof(float) * ndof * ld);
    L.v = take(sizeof(float) * ndof * ld);
  }
  // displacement and internal force at the last geometry refresh
  if (c->geom_every > 0) {
    L.usnap = take(sizeof(double) * ndof * ld);
    L.rbase = take(sizeof(double) * ndof * ld);
  }
  if (use_shared(c)) {
    const int64_t nb = (int64_t)c->bsr_col.size();
    L.bsr_ptr = take(sizeof(int32_t) * (nn + 1));
    L.bsr_col = take(sizeof(int32_t) * nb);
    L.adj_slot = take(sizeof(int2) * nadj);
    L.bsr64 = take(sizeof(double) * 9 * nb);
    L.bsr32 = take(sizeof(float) * 9 * nb);
  }
  L.q = take(sizeof(double) * nn * ld);
  L.qmask = take(sizeof(uint64_t) * nn * ((ld + 63) / 64));
  const int64_t n_nb = (nn + nodes_per_block(c->SB) - 1) / nodes_per_block(c->SB);
  // energy partials, then the second-level rows of the energy and of the
  // kinetic energy (256 each) and the kinetic energy row of the watchdog
  L.epart = take(sizeof(double) * (n_nb + 2 * 256 + 1) * ld);
  L.erec = take(sizeof(double) * kEnergyCap * ld);
  L.gtab = take(sizeof(double) * kChunk);
  L.base = take(sizeof(int64_t));
  L.mean = take(sizeof(double) * nn);
  L.var = take(sizeof(double) * nn);
  L.aux = take(sizeof(double) * ndof * ld);
  // stress values of one component [n_el][ld], the tangents [n_el][3] and
  // the bands (mean, lo, hi) [3][n_el]
  if (c->qoi_mask & ENS_QOI_STRESS) L.stress = take(sizeof(double) * (ne * ld + 6 * ne));
  L.total = off;
  return L;
}

// Block rows for the shared-stiffness variant: per node the sorted distinct
// neighbours, and per adjacency entry the block slots of its b and c.
void build_block_rows(ens_ctx* c) {
  const int64_t nn = c->n_nodes, ne = c->n_el;
  c->bsr_ptr.assign(nn + 1, 0);
  c->bsr_col.clear();
  c->adj_slot.resize(3 * ne);
  std::vector<int32_t> cols;
  for (int64_t i = 0; i < nn; ++i) {
    cols.clear();
    for (int32_t k = c->adj_ptr[i]; k < c->adj_ptr[i + 1]; ++k) {
      const int2 v = c->adj_nb[k];
      cols.push_back(v.x < 0 ? ~v.x : v.x);
      cols.push_back(v.y);
    }
    std::sort(cols.begin(), cols.end());
    cols.erase(std::unique(cols.begin(), cols.end()), cols.end());
    const int32_t base = (int32_t)c->bsr_col.size();
    c->bsr_col.insert(c->bsr_col.end(), cols.begin(), cols.end());
    c->bsr_ptr[i + 1] = (int32_t)c->bsr_col.size();
    for (int32_t k = c->adj_ptr[i]; k < c->adj_ptr[i + 1]; ++k) {
      const int2 v = c->adj_nb[k];
      const int32_t b = v.x < 0 ? ~v.x : v.x;
      const int32_t sb = base + (int32_t)(std::lower_bound(cols.begin(), cols.end(), b) - cols.begin());
      const int32_t sc = base + (int32_t)(std::lower_bound(cols.begin(), cols.end(), v.y) - cols.begin());
      c->adj_slot[k] = make_int2(sb, sc);
    }
  }
}

// Node-gather adjacency.  Each node's incident elements are ordered as a
// walk around the node (element j+1 shares the edge (node, c_j) with
// element j) so that consecutive entries share a neighbour: an entry whose
// first neighbour equals the previous entry's second one is flagged (its b
// index stored as ~b) and the kernel reuses the values already loaded.
void build_adjacency(ens_ctx* c) {
  const int64_t nn = c->n_nodes, ne = c->n_el;
  c->adj_ptr.assign(nn + 1, 0);
  for (int64_t i = 0; i < 3 * ne; ++i) c->adj_ptr[c->tri[i] + 1]++;
  for (int64_t i = 0; i < nn; ++i) c->adj_ptr[i + 1] += c->adj_ptr[i];
  std::vector<int32_t> next(c->adj_ptr.begin(), c->adj_ptr.end() - 1);
  std::vector<int32_t> el(3 * ne);
  std::vector<int2> nb(3 * ne);
  std::vector<uint8_t> loc(3 * ne);
  for (int64_t e = 0; e < ne; ++e) {
    for (int a = 0; a < 3; ++a) {
      const int32_t node = c->tri[3 * e + a];
      const int32_t pos = next[node]++;
      el[pos] = (int32_t)e;
      nb[pos] = make_int2(c->tri[3 * e + (a + 1) % 3], c->tri[3 * e + (a + 2) % 3]);
      loc[pos] = (uint8_t)a;
    }
  }
  c->adj_el.resize(3 * ne);
  c->adj_nb.resize(3 * ne);
  c->adj_loc.resize(3 * ne);
  std::vector<int32_t> order;
  std::vector<char> used;
  for (int64_t i = 0; i < nn; ++i) {
    const int32_t b0 = c->adj_ptr[i], b1 = c->adj_ptr[i + 1], k = b1 - b0;
    order.clear();
    used.assign(k, 0);
    int32_t prev_c = -1;
    while ((int32_t)order.size() < k) {
      int32_t pick = -1;
      if (prev_c >= 0)  // continue the walk across the shared edge
        for (int32_t j = 0; j < k; ++j)
          if (!used[j] && nb[b0 + j].x == prev_c) { pick = j; break; }
      if (pick < 0) {  // start a walk: prefer an entry no other unused entry leads into
        for (int32_t j = 0; j < k && pick < 0; ++j) {
          if (used[j]) continue;
          bool has_pred = false;
          for (int32_t t = 0; t < k; ++t)
            if (!used[t] && t != j && nb[b0 + t].y == nb[b0 + j].x) { has_pred = true; break; }
          if (!has_pred) pick = j;
        }
        if (pick < 0)
          for (int32_t j = 0; j < k; ++j)
            if (!used[j]) { pick = j; break; }
      }
      used[pick] = 1;
      order.push_back(pick);
      prev_c = nb[b0 + pick].y;
    }
    int32_t last_c = -1;
    for (int32_t t = 0; t < k; ++t) {
      const int32_t src = b0 + order[t], dst = b0 + t;
      c->adj_el[dst] = el[src];
      c->adj_loc[dst] = loc[src];
      int2 v = nb[src];
      const bool reuse = (t > 0 && v.x == last_c);
      last_c = v.y;
      if (reuse) v.x = ~v.x;
      c->adj_nb[dst] = v;
    }
  }
  // block rows for the shared-stiffness variant: sorted distinct neighbours
  build_block_rows(c);
  // an entry that closes a node's fan (its second neighbour is the first
  // entry's first one, the walk having reused every neighbour in between)
  // names it as ~c: the kernel takes it from registers
  for (int64_t i = 0; i < nn && ENSFEM_CLOSE_REUSE; ++i) {
    const int32_t b0 = c->adj_ptr[i], b1 = c->adj_ptr[i + 1];
    if (b1 - b0 < 3) continue;
    bool chain = true;
    for (int32_t t = b0 + 1; t < b1; ++t) chain = chain && c->adj_nb[t].x < 0;
    if (chain && c->adj_nb[b1 - 1].y == c->adj_nb[b0].x) c->adj_nb[b1 - 1].y = ~c->adj_nb[b1 - 1].y;
  }
}

bool use_shared(const ens_ctx* c) {
  return c->variant == ENS_VARIANT_CSR_SHARED || (c->variant == ENS_VARIANT_AUTO && c->shared);
}

bool ready_for_workspace(const ens_ctx* c, std::string* why) {
  if (!c->have_mesh) { *why = "mesh not set"; return false; }
  if (!c->have_ens) { *why = "ensemble not set"; return false; }
  return true;
}

StepArgs base_args(const ens_ctx* c, bool f32) {
  StepArgs a{};
  a.n_nodes = (int32_t)c->n_nodes;
  a.ld = c->ld;
  const int npb = nodes_per_block(c->SB);
  a.n_nb = (int32_t)((c->n_nodes + npb - 1) / npb);
  a.n_sb = c->ld / c->SB;
  a.sb_inner = c->sb_inner;
  a.adj.ptr = gptr(c->p<int32_t>(c->L.adj_ptr));
  a.adj.el = gptr(c->p<int32_t>(c->L.adj_el));
  a.adj.nb = gptr(c->p<int2>(c->L.adj_nb));
  a.adj.k = gptr(f32 ? (const void*)c->p<float>(c->L.k32) : (const void*)c->p<double>(c->L.k64));
  a.eh = gptr(f32 ? (const void*)c->p<float>(c->L.eh32) : (const void*)c->p<double>(c->L.eh64));
  if (use_shared(c)) {
    a.bsr.ptr = gptr(c->p<int32_t>(c->L.bsr_ptr));
    a.bsr.col = gptr(c->p<int32_t>(c->L.bsr_col));
    a.bsr.val = gptr(f32 ? (const void*)c->p<float>(c->L.bsr32) : (const void*)c->p<double>(c->L.bsr64));
  }
  a.minv = gptr(f32 ? (const void*)c->p<float>(c->L.minv32) : (const void*)c->p<double>(c->L.minv64));
  a.F = gptr(c->p<double>(c->L.F));
  a.fixed = gptr(c->p<uint8_t>(c->L.fixed));
  a.radial = gptr(c->p<double>(c->L.radial));
  a.q = gptr(c->p<double>(c->L.q));
  a.qmask = gptr(c->p<uint64_t>(c->L.qmask));
  a.qwords = (c->ld + 63) / 64;
  a.gtab = gptr(c->p<double>(c->L.gtab));
  a.energy_part = gptr(c->p<double>(c->L.epart));
  a.cd = c->cd;
  return a;
}

// State buffers of the step whose current displacement is buffer
// cur ^ flip.
void set_state_ptrs(const ens_ctx* c, StepArgs& a, int flip) {
  const int cur = c->cur ^ flip;
  if (c->state_prec == ENS_STATE_F64) {
    a.u_cur = gptr(c->p<double>(c->L.u[cur]));
    a.u_prev = gptr(c->p<double>(c->L.u[1 - cur]));
    a.u_next = gptr(c->p<double>(c->L.u[1 - cur]));
  } else {
    a.uh_cur = gptr(c->p<float>(c->L.uh[cur]));
    a.uh_next = gptr(c->p<float>(c->L.uh[1 - cur]));
    a.uc = gptr(c->state_prec == ENS_STATE_F32_KAHAN ? c->p<float>(c->L.uc) : nullptr);
    a.v = gptr(c->p<float>(c->L.v));
  }
}

// Caller rows <-> internal rows.  Internal row r holds caller row
// map[r / rep] * rep + r % rep (rep = 3 for dof rows of the node map,
// 1 for node or element rows); map == null: identity.
inline int64_t caller_row(const std::vector<int32_t>* map, int rep, int64_t r) {
  return map ? (int64_t)(*map)[r / rep] * rep + r % rep : r;
}

// pad [rows][S] caller data to internal [rows][ld]; pads copy column 0
void pad_rows(const double* src, int64_t rows, int S, int ld, std::vector<double>& dst,
              const std::vector<int32_t>* map = nullptr, int rep = 1) {
  dst.resize((size_t)rows * ld);
  for (int64_t r = 0; r < rows; ++r) {
    const double* s = src + caller_row(map, rep, r) * S;
    double* d = dst.data() + r * ld;
    std::memcpy(d, s, sizeof(double) * S);
    for (int k = S; k < ld; ++k) d[k] = s[0];
  }
}

void unpad_rows(const double* src, int64_t rows, int S, int ld, double* dst,
                const std::vector<int32_t>* map = nullptr, int rep = 1) {
  for (int64_t r = 0; r < rows; ++r)
    std::memcpy(dst + caller_row(map, rep, r) * S, src + r * ld, sizeof(double) * S);
}

// Locality order of the nodes: recursive coordinate bisection (split at the
// median of the longest bounding-box axis) down to patches of <= 64 nodes,
// patches in recursion order, nodes in a patch along its longest axis.  A
// workgroup's nodes and their neighbours then lie in one compact surface
// patch, and consecutive node blocks stay close on the surface.
void rcb_order(const std::vector<double>& xyz, std::vector<int32_t>& idx, size_t lo, size_t hi) {
  double mn[3] = {1e300, 1e300, 1e300}, mx[3] = {-1e300, -1e300, -1e300};
  for (size_t i = lo; i < hi; ++i)
    for (int k = 0; k < 3; ++k) {
      mn[k] = std::min(mn[k], xyz[3 * (size_t)idx[i] + k]);
      mx[k] = std::max(mx[k], xyz[3 * (size_t)idx[i] + k]);
    }
  int ax = 0;
  for (int k = 1; k < 3; ++k)
    if (mx[k] - mn[k] > mx[ax] - mn[ax]) ax = k;
  auto less = [&](int32_t a, int32_t b) {
    const double xa = xyz[3 * (size_t)a + ax], xb = xyz[3 * (size_t)b + ax];
    return xa < xb || (xa == xb && a < b);
  };
  if (hi - lo <= 64) {
    std::sort(idx.begin() + lo, idx.begin() + hi, less);
    return;
  }
  const size_t mid = lo + (hi - lo) / 2;
  std::nth_element(idx.begin() + lo, idx.begin() + mid, idx.begin() + hi, less);
  rcb_order(xyz, idx, lo, mid);
  rcb_order(xyz, idx, mid, hi);
}

int32_t upload_all(ens_ctx* ctx) {
  const Layout& L = ctx->L;
  hipStream_t st = nullptr;
  const int64_t nn = ctx->n_nodes, ne = ctx->n_el, ld = ctx->ld;
  HIPC(hipMemcpy(ctx->p<void>(L.xyz), ctx->xyz.data(), sizeof(double) * 3 * nn, hipMemcpyHostToDevice));
  HIPC(hipMemcpy(ctx->p<void>(L.tri), ctx->tri.data(), sizeof(int32_t) * 3 * ne, hipMemcpyHostToDevice));
  HIPC(hipMemcpy(ctx->p<void>(L.adj_ptr), ctx->adj_ptr.data(), sizeof(int32_t) * (nn + 1), hipMemcpyHostToDevice));
  HIPC(hipMemcpy(ctx->p<void>(L.adj_el), ctx->adj_el.data(), sizeof(int32_t) * 3 * ne, hipMemcpyHostToDevice));
  HIPC(hipMemcpy(ctx->p<void>(L.adj_nb), ctx->adj_nb.data(), sizeof(int2) * 3 * ne, hipMemcpyHostToDevice));
  HIPC(hipMemcpy(ctx->p<void>(L.adj_loc), ctx->adj_loc.data(), 3 * ne, hipMemcpyHostToDevice));
  HIPC(hipMemcpy(ctx->p<void>(L.fixed), ctx->fixed.data(), nn, hipMemcpyHostToDevice));
  HIPC(hipMemcpy(ctx->p<void>(L.radial), ctx->radial.data(), sizeof(double) * 3 * nn, hipMemcpyHostToDevice));
  HIPC(hipMemcpy(ctx->p<void>(L.perm), ctx->perm.data(), sizeof(int32_t) * nn, hipMemcpyHostToDevice));

  if (ctx->have_load)
    HIPC(hipMemcpy(ctx->p<void>(L.F), ctx->F.data(), sizeof(double) * 3 * nn, hipMemcpyHostToDevice));
  else
    HIPC(hipMemset(ctx->p<void>(L.F), 0, sizeof(double) * 3 * nn));
  HIPC(hipMemcpy(ctx->p<void>(L.eh64), ctx->eh.data(), sizeof(double) * ne * ld, hipMemcpyHostToDevice));
  HIPC(hipMemcpy(ctx->p<void>(L.h), ctx->h.data(), sizeof(double) * ne * ld, hipMemcpyHostToDevice));
  HIPC(hipMemset(ctx->p<void>(L.flags), 0, sizeof(Flags)));
  Flags* fl = ctx->p<Flags>(L.flags);
  HIPC(launch_element_setup(ne, ctx->p<double>(L.xyz), ctx->p<int32_t>(L.tri), ctx->nu, ctx->shear_k,
                            ctx->p<double>(L.khat), ctx->p<double>(L.area), ctx->p<double>(L.lam),
                            ctx->p<double>(L.frame), &fl->bad, st));
  HIPC(launch_adjacency_blocks(3 * ne, ctx->p<int32_t>(L.adj_el), ctx->p<uint8_t>(L.adj_loc),
                               ctx->p<double>(L.khat), ctx->p<double>(L.k64), ctx->p<float>(L.k32), st));
  HIPC(launch_cast_f32(ne * ld, ctx->p<double>(L.eh64), ctx->p<float>(L.eh32), st));
  if (use_shared(ctx)) {
    const int64_t nb = (int64_t)ctx->bsr_col.size();
    HIPC(hipMemcpy(ctx->p<void>(L.bsr_ptr), ctx->bsr_ptr.data(), sizeof(int32_t) * (nn + 1), hipMemcpyHostToDevice));
    HIPC(hipMemcpy(ctx->p<void>(L.bsr_col), ctx->bsr_col.data(), sizeof(int32_t) * nb, hipMemcpyHostToDevice));
    HIPC(hipMemcpy(ctx->p<void>(L.adj_slot), ctx->adj_slot.data(), sizeof(int2) * 3 * ne, hipMemcpyHostToDevice));
    HIPC(launch_bsr_assemble((int32_t)nn, (int32_t)ld, ctx->p<int32_t>(L.adj_ptr), ctx->p<int32_t>(L.adj_el),
                             ctx->p<uint8_t>(L.adj_loc), ctx->p<int2>(L.adj_slot), ctx->p<int32_t>(L.bsr_ptr),
                             ctx->p<double>(L.khat), ctx->p<double>(L.eh64), ctx->p<double>(L.bsr64), st));
    HIPC(launch_cast_f32(9 * nb, ctx->p<double>(L.bsr64), ctx->p<float>(L.bsr32), st));
  }
  HIPC(launch_lumped_mass((int32_t)nn, (int32_t)ld, ctx->p<int32_t>(L.adj_ptr), ctx->p<int32_t>(L.adj_el),
                          ctx->p<double>(L.area), ctx->p<double>(L.h), ctx->rho, ctx->p<double>(L.eh64),
                          ctx->p<double>(L.lam), ctx->mass_dt, ctx->p<double>(L.minv64), ctx->p<float>(L.minv32),
                          st));
  HIPC(launch_cfl_max(ne, (int32_t)ld, ctx->S, ctx->p<double>(L.eh64), ctx->p<double>(L.h),
                      ctx->p<double>(L.lam), ctx->p<double>(L.area), ctx->rho, ctx->mass_dt, &fl->omega2_bits,
                      st));
  HIPC(hipDeviceSynchronize());
  Flags hf{};
  HIPC(hipMemcpy(&hf, fl, sizeof(Flags), hipMemcpyDeviceToHost));
  if (hf.bad) return ctx->fail(ENS_EINVAL, "degenerate triangle found by the element set-up");
  double w2;
  std::memcpy(&w2, &hf.omega2_bits, sizeof(double));
  if (!(w2 > 0.0) || !std::isfinite(w2)) return ctx->fail(ENS_EINVAL, "stability bound is not finite");
  ctx->omega2 = w2;
  return ENS_OK;
}

}  // namespace

extern "C" {

int32_t ens_create(int32_t device, ens_ctx** out) {
  if (!out) return ENS_EINVAL;
  *out = nullptr;
  int n = 0;
  if (hipGetDeviceCount(&n) != hipSuccess || device < 0 || device >= n) return ENS_EDEVICE;
  if (hipSetDevice(device) != hipSuccess) return ENS_EDEVICE;
  // once per device, with it current: the allocation-free scratch's address
  if (scratch_setup(device) != hipSuccess) return ENS_EDEVICE;
  ens_ctx* c = new (std::nothrow) ens_ctx();
  if (!c) return ENS_EINVAL;
  c->device = device;
  *out = c;
  return ENS_OK;
}

int32_t ens_destroy(ens_ctx* ctx) {
  if (!ctx) return ENS_EINVAL;
  if (ctx->bound) (void)hipDeviceSynchronize();  // teardown: nothing to report
  delete ctx;
  return ENS_OK;
}

const char* ens_last_error(const ens_ctx* ctx) { return ctx ? ctx->err.c_str() : "null context"; }

int32_t ens_info(ens_ctx* ctx, ens_info_t* out) {
  if (!ctx || !out) return ENS_EINVAL;
  out->n_nodes = ctx->n_nodes;
  out->n_el = ctx->n_el;
  out->n_dof = 3 * ctx->n_nodes;
  out->S = ctx->S;
  out->S_pad = ctx->ld;
  out->sample_block = ctx->SB;
  out->apply_prec = ctx->apply_prec;
  out->state_prec = ctx->state_prec;
  out->variant = use_shared(ctx) ? ENS_VARIANT_CSR_SHARED : ENS_VARIANT_NODE_GATHER;
  out->shared_stiffness = ctx->shared ? 1 : 0;
  out->steps_done = ctx->steps;
  out->dt = ctx->dt;
  out->workspace_bytes = ctx->have_mesh && ctx->have_ens ? plan(ctx).total : 0;
  return ENS_OK;
}

int32_t ens_set_mesh(ens_ctx* ctx, int64_t n_nodes, const double* xyz, int64_t n_el,
                     const int32_t* tri, const uint8_t* fixed_dof, const double* radial) {
  if (!ctx) return ENS_EINVAL;
  ctx->gen++;
  GUARD_BEGIN
  if (n_nodes < 3 || n_el < 1 || !xyz || !tri || !fixed_dof || !radial)
    return ctx->fail(ENS_EINVAL, "ens_set_mesh: need n_nodes >= 3, n_el >= 1 and non-null arrays");
  if (n_nodes > INT32_MAX / 3 || n_el > INT32_MAX / 3)
    return ctx->fail(ENS_EINVAL, "ens_set_mesh: mesh too large for 32-bit indices");
  for (int64_t i = 0; i < 3 * n_el; ++i)
    if (tri[i] < 0 || tri[i] >= n_nodes)
      return ctx->fail(ENS_EINVAL, "ens_set_mesh: element index out of range at entry " + std::to_string(i));
  for (int64_t i = 0; i < 3 * n_nodes; ++i)
    if (!std::isfinite(xyz[i])) return ctx->fail(ENS_EINVAL, "ens_set_mesh: non-finite coordinate");
  for (int64_t e = 0; e < n_el; ++e) {  // reject degenerate triangles up front
    const int32_t* t = tri + 3 * e;
    if (t[0] == t[1] || t[1] == t[2] || t[0] == t[2])
      return ctx->fail(ENS_EINVAL, "ens_set_mesh: repeated node in element " + std::to_string(e));
    double a[3], b[3];
    for (int k = 0; k < 3; ++k) {
      a[k] = xyz[3 * t[1] + k] - xyz[3 * t[0] + k];
      b[k] = xyz[3 * t[2] + k] - xyz[3 * t[0] + k];
    }
    const double cx = a[1] * b[2] - a[2] * b[1], cy = a[2] * b[0] - a[0] * b[2], cz = a[0] * b[1] - a[1] * b[0];
    if (!(cx * cx + cy * cy + cz * cz > 0.0))
      return ctx->fail(ENS_EINVAL, "ens_set_mesh: degenerate triangle " + std::to_string(e));
  }
  for (int64_t i = 0; i < n_nodes; ++i) {
    const double* r = radial + 3 * i;
    const double nrm = std::sqrt(r[0] * r[0] + r[1] * r[1] + r[2] * r[2]);
    if (!(std::fabs(nrm - 1.0) <= 1e-6))
      return ctx->fail(ENS_EINVAL, "ens_set_mesh: radial vector of node " + std::to_string(i) + " is not unit length");
  }
  ctx->n_nodes = n_nodes;
  ctx->n_el = n_el;
  {
    std::vector<double> cxyz(xyz, xyz + 3 * n_nodes);
    std::vector<int32_t>& perm = ctx->perm;
    perm.resize(n_nodes);
    for (int64_t i = 0; i < n_nodes; ++i) perm[i] = (int32_t)i;
    rcb_order(cxyz, perm, 0, (size_t)n_nodes);
    std::vector<int32_t> inv(n_nodes);
    for (int64_t i = 0; i < n_nodes; ++i) inv[perm[i]] = (int32_t)i;
    // elements in order of their first (internal) node, ties by caller index
    std::vector<int32_t> key(n_el);
    for (int64_t e = 0; e < n_el; ++e)
      key[e] = std::min(inv[tri[3 * e]], std::min(inv[tri[3 * e + 1]], inv[tri[3 * e + 2]]));
    ctx->eperm.resize(n_el);
    for (int64_t e = 0; e < n_el; ++e) ctx->eperm[e] = (int32_t)e;
    std::stable_sort(ctx->eperm.begin(), ctx->eperm.end(), [&](int32_t a, int32_t b) { return key[a] < key[b]; });
    ctx->xyz.resize(3 * n_nodes);
    ctx->radial.resize(3 * n_nodes);
    ctx->fixed.assign(n_nodes, 0);
    for (int64_t i = 0; i < n_nodes; ++i) {
      const int64_t o = perm[i];
      for (int k = 0; k < 3; ++k) {
        ctx->xyz[3 * i + k] = xyz[3 * o + k];
        ctx->radial[3 * i + k] = radial[3 * o + k];
        if (fixed_dof[3 * o + k]) ctx->fixed[i] |= (uint8_t)(1u << k);
      }
    }
    ctx->tri.resize(3 * n_el);
    for (int64_t e = 0; e < n_el; ++e)
      for (int k = 0; k < 3; ++k) ctx->tri[3 * e + k] = inv[tri[3 * (int64_t)ctx->eperm[e] + k]];
  }
  build_adjacency(ctx);
  ctx->have_mesh = true;
  ctx->have_ens = false;  // fields are per element: re-set them for a new mesh
  ctx->have_load = false;
  ctx->bound = false;
  ctx->state_init = false;
  return ENS_OK;
  GUARD_END
}

int32_t ens_set_material(ens_ctx* ctx, double nu, double shear_k, double rho, double alpha) {
  if (!ctx) return ENS_EINVAL;
  ctx->gen++;
  if (!(nu >= 0.0 && nu < 0.5) || !(shear_k >= 0.0) || !(rho > 0.0) || !(alpha >= 0.0) ||
      !std::isfinite(shear_k) || !std::isfinite(rho) || !std::isfinite(alpha))
    return ctx->fail(ENS_EINVAL, "ens_set_material: need 0 <= nu < 0.5, k >= 0, rho > 0, alpha >= 0");
  ctx->nu = nu;
  ctx->shear_k = shear_k;
  ctx->rho = rho;
  ctx->alpha = alpha;
  ctx->have_material = true;
  ctx->bound = false;
  ctx->state_init = false;
  return ENS_OK;
}

int32_t ens_set_mass_scaling(ens_ctx* ctx, double dt_target) {
  if (!ctx) return ENS_EINVAL;
  if (!(dt_target >= 0.0) || !std::isfinite(dt_target))
    return ctx->fail(ENS_EINVAL, "ens_set_mass_scaling: need a finite dt_target >= 0");
  ctx->gen++;
  ctx->mass_dt = dt_target;
  ctx->bound = false;
  ctx->state_init = false;
  return ENS_OK;
}

int32_t ens_set_geometry_refresh(ens_ctx* ctx, int32_t every) {
  if (!ctx) return ENS_EINVAL;
  if (every < 0) return ctx->fail(ENS_EINVAL, "ens_set_geometry_refresh: need every >= 0");
  if (every == ctx->geom_every) return ENS_OK;  // unchanged: the state stays
  ctx->gen++;
  if ((every > 0) != (ctx->geom_every > 0)) ctx->bound = false;  // the snapshot buffer comes or goes
  ctx->geom_every = every;
  ctx->state_init = false;
  return ENS_OK;
}

int32_t ens_set_viscous(ens_ctx* ctx, double c_d) {
  if (!ctx) return ENS_EINVAL;
  if (!(c_d >= 0.0) || !std::isfinite(c_d)) return ctx->fail(ENS_EINVAL, "ens_set_viscous: need a finite c_d >= 0");
  ctx->gen++;
  ctx->cd = c_d;
  ctx->state_init = false;
  return ENS_OK;
}

int32_t ens_set_ensemble(ens_ctx* ctx, int32_t S, const double* eh, const double* h) {
  if (!ctx) return ENS_EINVAL;
  ctx->gen++;
  GUARD_BEGIN
  if (!ctx->have_mesh) return ctx->fail(ENS_ESTATE, "ens_set_ensemble: set the mesh first");
  if (S < 1 || !eh || !h) return ctx->fail(ENS_EINVAL, "ens_set_ensemble: need S >= 1 and non-null arrays");
  const int64_t n = ctx->n_el * (int64_t)S;
  for (int64_t i = 0; i < n; ++i)
    if (!(eh[i] > 0.0) || !(h[i] > 0.0) || !std::isfinite(eh[i]) || !std::isfinite(h[i]))
      return ctx->fail(ENS_EINVAL, "ens_set_ensemble: (E h) and h must be finite and positive (entry " +
                                       std::to_string(i) + ")");
  ctx->S = S;
  ctx->SB = pick_sample_block(S, ctx->tune_sb);
  ctx->ld = ((S + ctx->SB - 1) / ctx->SB) * ctx->SB;
  pad_rows(eh, ctx->n_el, S, ctx->ld, ctx->eh, &ctx->eperm);
  pad_rows(h, ctx->n_el, S, ctx->ld, ctx->h, &ctx->eperm);
  bool shared = true;
  for (int64_t e = 0; e < ctx->n_el && shared; ++e)
    for (int s = 1; s < S; ++s)
      if (eh[e * S + s] != eh[e * S]) { shared = false; break; }
  ctx->shared = shared;
  ctx->have_ens = true;
  ctx->bound = false;
  ctx->state_init = false;
  return ENS_OK;
  GUARD_END
}

int32_t ens_set_load(ens_ctx* ctx, const double* F, ens_schedule sched) {
  if (!ctx) return ENS_EINVAL;
  ctx->gen++;
  GUARD_BEGIN
  if (!ctx->have_mesh) return ctx->fail(ENS_ESTATE, "ens_set_load: set the mesh first");
  if (!F) return ctx->fail(ENS_EINVAL, "ens_set_load: null load");
  if (sched.kind < ENS_LOAD_STEP || sched.kind > ENS_LOAD_PULSATILE)
    return ctx->fail(ENS_EINVAL, "ens_set_load: unknown schedule kind");
  if (sched.kind != ENS_LOAD_STEP && !(sched.t_ramp > 0.0))
    return ctx->fail(ENS_EINVAL, "ens_set_load: ramp time must be positive");
  if (sched.kind == ENS_LOAD_PULSATILE && !(sched.period > 0.0))
    return ctx->fail(ENS_EINVAL, "ens_set_load: period must be positive");
  for (int64_t i = 0; i < 3 * ctx->n_nodes; ++i)
    if (!std::isfinite(F[i])) return ctx->fail(ENS_EINVAL, "ens_set_load: non-finite load");
  ctx->F.resize(3 * ctx->n_nodes);
  for (int64_t i = 0; i < ctx->n_nodes; ++i)
    for (int k = 0; k < 3; ++k) ctx->F[3 * i + k] = F[3 * (int64_t)ctx->perm[i] + k];
  ctx->sched = Schedule{sched.kind, sched.t_ramp, sched.amp, sched.period};
  ctx->have_load = true;
  if (ctx->bound) {
    hipError_t e = hipMemcpy(ctx->p<void>(ctx->L.F), ctx->F.data(), sizeof(double) * 3 * ctx->n_nodes,
                             hipMemcpyHostToDevice);
    if (e != hipSuccess) return ctx->fail(ENS_EDEVICE, hipGetErrorString(e));
  }
  return ENS_OK;
  GUARD_END
}

int32_t ens_configure(ens_ctx* ctx, int32_t apply_prec, int32_t state_prec, int32_t variant,
                      int32_t qoi_mask, int32_t energy_every) {
  if (!ctx) return ENS_EINVAL;
  ctx->gen++;
  if (apply_prec != ENS_F64 && apply_prec != ENS_F32)
    return ctx->fail(ENS_EINVAL, "ens_configure: apply_prec must be ENS_F64 or ENS_F32");
  if (state_prec < ENS_STATE_F64 || state_prec > ENS_STATE_F32)
    return ctx->fail(ENS_EINVAL, "ens_configure: unknown state precision");
  if (state_prec != ENS_STATE_F64 && apply_prec != ENS_F32)
    return ctx->fail(ENS_EUNSUPPORTED, "ens_configure: FP32 states need the FP32 apply");
  if (variant != ENS_VARIANT_AUTO && variant != ENS_VARIANT_NODE_GATHER && variant != ENS_VARIANT_CSR_SHARED)
    return ctx->fail(ENS_EINVAL, "ens_configure: unknown variant");
  if (qoi_mask & ~(ENS_QOI_PEAK_RADIAL | ENS_QOI_STRESS)) return ctx->fail(ENS_EINVAL, "ens_configure: unknown QoI bit");
  if (energy_every < 0) return ctx->fail(ENS_EINVAL, "ens_configure: energy_every must be >= 0");
  const bool relayout = state_prec != ctx->state_prec || variant != ctx->variant;
  ctx->apply_prec = apply_prec;
  ctx->state_prec = state_prec;
  ctx->variant = variant;
  ctx->qoi_mask = qoi_mask;
  ctx->energy_every = energy_every;
  if (relayout) {
    ctx->bound = false;
    ctx->state_init = false;
  }
  return ENS_OK;
}

int32_t ens_set_tuning(ens_ctx* ctx, int32_t sample_block, int32_t sb_inner);

int32_t ens_workspace_size(ens_ctx* ctx, size_t* bytes) {
  if (!ctx || !bytes) return ENS_EINVAL;
  std::string why;
  if (!ready_for_workspace(ctx, &why)) return ctx->fail(ENS_ESTATE, "ens_workspace_size: " + why);
  *bytes = plan(ctx).total;
  return ENS_OK;
}

int32_t ens_bind_workspace(ens_ctx* ctx, void* dptr, size_t bytes) {
  if (!ctx) return ENS_EINVAL;
  ctx->gen++;
  GUARD_BEGIN
  std::string why;
  if (!ready_for_workspace(ctx, &why)) return ctx->fail(ENS_ESTATE, "ens_bind_workspace: " + why);
  if (ctx->variant == ENS_VARIANT_CSR_SHARED && !ctx->shared)
    return ctx->fail(ENS_EUNSUPPORTED, "ens_bind_workspace: the shared-stiffness variant needs (E h) constant over samples");
  const Layout L = plan(ctx);
  if (!dptr || (reinterpret_cast<uintptr_t>(dptr) % kAlign) != 0)
    return ctx->fail(ENS_EWORKSPACE, "ens_bind_workspace: null or unaligned (256 B) buffer");
  if (bytes < L.total)
    return ctx->fail(ENS_EWORKSPACE, "ens_bind_workspace: need " + std::to_string(L.total) + " bytes, got " +
                                         std::to_string(bytes));
  HIPC(hipSetDevice(ctx->device));
  ctx->ws = static_cast<char*>(dptr);
  ctx->ws_bytes = bytes;
  ctx->L = L;
  ctx->bound = false;
  ctx->state_init = false;
  const int32_t rc = upload_all(ctx);
  if (rc != ENS_OK) return rc;
  ctx->bound = true;
  return ENS_OK;
  GUARD_END
}

int32_t ens_cfl_dt(ens_ctx* ctx, double safety, double* dt_out) {
  if (!ctx || !dt_out) return ENS_EINVAL;
  if (!ctx->bound) return ctx->fail(ENS_EWORKSPACE, "ens_cfl_dt: bind a workspace first");
  if (!(safety > 0.0)) return ctx->fail(ENS_EINVAL, "ens_cfl_dt: safety must be positive");
  *dt_out = safety * 2.0 / std::sqrt(ctx->omega2);
  return ENS_OK;
}

int32_t ens_init_state(ens_ctx* ctx, const double* u0, const double* v0) {
  if (!ctx) return ENS_EINVAL;
  ctx->gen++;
  GUARD_BEGIN
  if (!ctx->bound) return ctx->fail(ENS_EWORKSPACE, "ens_init_state: bind a workspace first");
  const Layout& L = ctx->L;
  HIPC(hipMemset(&ctx->p<Flags>(L.flags)->unstable, 0, sizeof(int32_t)));
  const int64_t ndof = 3 * ctx->n_nodes, ld = ctx->ld, n = ndof * ld;
  std::vector<double> buf;
  hipStream_t st = nullptr;
  ctx->u0_zero = (u0 == nullptr);
  if (u0)
    for (int64_t i = 0; i < ndof * ctx->S; ++i)
      if (!std::isfinite(u0[i]) || (v0 && !std::isfinite(v0[i])))
        return ctx->fail(ENS_EINVAL, "ens_init_state: non-finite initial state");
  if (ctx->state_prec == ENS_STATE_F64) {
    if (u0) {
      pad_rows(u0, ndof, ctx->S, (int)ld, buf, &ctx->perm, 3);
      HIPC(hipMemcpy(ctx->p<void>(L.u[0]), buf.data(), sizeof(double) * n, hipMemcpyHostToDevice));
    } else {
      HIPC(hipMemset(ctx->p<void>(L.u[0]), 0, sizeof(double) * n));
    }
    if (v0) {
      pad_rows(v0, ndof, ctx->S, (int)ld, buf, &ctx->perm, 3);
      HIPC(hipMemcpy(ctx->p<void>(L.u[1]), buf.data(), sizeof(double) * n, hipMemcpyHostToDevice));
    } else {
      HIPC(hipMemset(ctx->p<void>(L.u[1]), 0, sizeof(double) * n));
    }
    HIPC(launch_qoi_init((int32_t)ctx->n_nodes, (int32_t)ld, ctx->p<double>(L.radial),
                         ctx->p<double>(L.u[0]), nullptr, nullptr, ctx->p<double>(L.q), st));
    // the first refresh interval is the linear model (u_m = 0, R_m = 0)
    if (ctx->geom_every > 0) {
      HIPC(hipMemset(ctx->p<void>(L.usnap), 0, sizeof(double) * n));
      HIPC(hipMemset(ctx->p<void>(L.rbase), 0, sizeof(double) * n));
    }
  } else {
    float* uc = ctx->state_prec == ENS_STATE_F32_KAHAN ? ctx->p<float>(L.uc) : nullptr;
    if (u0) {
      pad_rows(u0, ndof, ctx->S, (int)ld, buf, &ctx->perm, 3);
      HIPC(hipMemcpy(ctx->p<void>(L.aux), buf.data(), sizeof(double) * n, hipMemcpyHostToDevice));
      HIPC(launch_split_f32(n, ctx->p<double>(L.aux), ctx->p<float>(L.uh[0]), uc, st));
    } else {
      HIPC(hipMemset(ctx->p<void>(L.uh[0]), 0, sizeof(float) * n));
      if (uc) HIPC(hipMemset(uc, 0, sizeof(float) * n));
    }
    if (v0) {
      pad_rows(v0, ndof, ctx->S, (int)ld, buf, &ctx->perm, 3);
      HIPC(hipMemcpy(ctx->p<void>(L.aux), buf.data(), sizeof(double) * n, hipMemcpyHostToDevice));
      HIPC(launch_cast_f32(n, ctx->p<double>(L.aux), ctx->p<float>(L.v), st));
    } else {
      HIPC(hipMemset(ctx->p<void>(L.v), 0, sizeof(float) * n));
    }
    HIPC(launch_qoi_init((int32_t)ctx->n_nodes, (int32_t)ld, ctx->p<double>(L.radial), nullptr,
                         ctx->p<float>(L.uh[0]), uc, ctx->p<double>(L.q), st));
  }
  HIPC(hipMemset(ctx->p<void>(L.qmask), 0, sizeof(uint64_t) * ctx->n_nodes * ((ld + 63) / 64)));
  ctx->mask_live = false;
  HIPC(hipMemset(ctx->p<void>(L.base), 0, sizeof(int64_t)));
  HIPC(hipDeviceSynchronize());
  ctx->cur = 0;
  ctx->steps = 0;
  ctx->dt = 0.0;
  ctx->started = false;
  ctx->energy_records = 0;
  ctx->energy_steps.assign(kEnergyCap, -1);
  ctx->state_init = true;
  return ENS_OK;
  GUARD_END
}

namespace {

int32_t run_starter(ens_ctx* ctx, double dt, hipStream_t st) {
  const Layout& L = ctx->L;
  const int64_t n = 3 * ctx->n_nodes * (int64_t)ctx->ld;
  if (ctx->state_prec == ENS_STATE_F64) {
    double* R = ctx->p<double>(L.aux);
    if (ctx->u0_zero) {
      HIPC(hipMemsetAsync(R, 0, sizeof(double) * n, st));
    } else {
      StepArgs a = base_args(ctx, false);
      HIPC(launch_apply(a, false, ctx->SB, use_shared(ctx), ctx->p<double>(L.u[ctx->cur]), R, nullptr, st));
    }
    HIPC(launch_starter_f64((int32_t)ctx->n_nodes, ctx->ld, R, ctx->p<double>(L.minv64), ctx->p<double>(L.F),
                            ctx->p<uint8_t>(L.fixed), ctx->p<double>(L.u[ctx->cur]),
                            ctx->p<double>(L.u[1 - ctx->cur]), ctx->p<double>(L.gtab), dt, ctx->alpha, ctx->cd,
                            st));
  } else {
    float* R = ctx->p<float>(L.aux);
    if (ctx->u0_zero) {
      HIPC(hipMemsetAsync(R, 0, sizeof(float) * n, st));
    } else {
      StepArgs a = base_args(ctx, true);
      HIPC(launch_apply(a, true, ctx->SB, use_shared(ctx), ctx->p<float>(L.uh[ctx->cur]), R, nullptr, st));
    }
    HIPC(launch_starter_f32((int32_t)ctx->n_nodes, ctx->ld, R, ctx->p<float>(L.minv32), ctx->p<double>(L.F),
                            ctx->p<uint8_t>(L.fixed), ctx->p<float>(L.v), ctx->p<double>(L.gtab), dt,
                            ctx->alpha, ctx->cd, st));
  }
  return ENS_OK;
}

// Fold the open rises into q so q holds every sample's running peak.
int32_t resolve_qoi(ens_ctx* ctx) {
  const Layout& L = ctx->L;
  if (ctx->SB < 64 && !ctx->mask_live) return ENS_OK;  // q is already up to date
  if (ctx->state_prec == ENS_STATE_F64)
    HIPC(launch_qoi_resolve((int32_t)ctx->n_nodes, ctx->ld, ctx->p<double>(L.radial),
                            ctx->p<double>(L.u[ctx->cur]), nullptr, nullptr, ctx->p<double>(L.q),
                            ctx->p<uint64_t>(L.qmask), nullptr));
  else
    HIPC(launch_qoi_resolve((int32_t)ctx->n_nodes, ctx->ld, ctx->p<double>(L.radial), nullptr,
                            ctx->p<float>(L.uh[ctx->cur]),
                            ctx->state_prec == ENS_STATE_F32_KAHAN ? ctx->p<float>(L.uc) : nullptr,
                            ctx->p<double>(L.q), ctx->p<uint64_t>(L.qmask), nullptr));
  HIPC(hipDeviceSynchronize());
  return ENS_OK;
}

}  // namespace

int32_t ens_step(ens_ctx* ctx, int64_t n_steps, double dt, int32_t force, void* stream) {
  if (!ctx) return ENS_EINVAL;
  GUARD_BEGIN
  if (!ctx->bound) return ctx->fail(ENS_EWORKSPACE, "ens_step: bind a workspace first");
  if (!ctx->have_load) return ctx->fail(ENS_ESTATE, "ens_step: load not set");
  if (!ctx->have_material) return ctx->fail(ENS_ESTATE, "ens_step: material not set");
  if (!ctx->state_init) return ctx->fail(ENS_ESTATE, "ens_step: call ens_init_state first");
  if (n_steps < 0) return ctx->fail(ENS_EINVAL, "ens_step: n_steps must be >= 0");
  if (!(dt > 0.0) || !std::isfinite(dt)) return ctx->fail(ENS_EINVAL, "ens_step: dt must be positive");
  if (ctx->started && dt != ctx->dt)
    return ctx->fail(ENS_EINVAL, "ens_step: dt is fixed once stepping has started (re-init the state to change it)");
  const bool geom = ctx->geom_every > 0;
  if (geom && (ctx->state_prec != ENS_STATE_F64 || ctx->energy_every > 0))
    return ctx->fail(ENS_EUNSUPPORTED, "ens_step: the geometry refresh needs the FP64 state and no energy records");
  const double dt_max = 2.0 / std::sqrt(ctx->omega2);
  if (dt > dt_max && !force)
    return ctx->fail(ENS_EUNSTABLE, "ens_step: dt " + std::to_string(dt) + " exceeds the stability bound " +
                                        std::to_string(dt_max));
  HIPC(hipSetDevice(ctx->device));
  hipStream_t st = static_cast<hipStream_t>(stream);
  ctx->last_stream = st;
  const Layout& L = ctx->L;
  const bool f32 = ctx->apply_prec == ENS_F32;
  const bool qoi = (ctx->qoi_mask & ENS_QOI_PEAK_RADIAL) != 0;
  StepArgs a = base_args(ctx, f32);
  a.dt = dt;
  a.a = 0.5 * ctx->alpha * dt;
  if (geom) {
    a.usnap = gptr(ctx->p<double>(L.usnap));
    a.rbase = gptr(ctx->p<double>(L.rbase));
    a.xyz = gptr(ctx->p<double>(L.xyz));
    a.nu = ctx->nu;
    a.shear_k = ctx->shear_k;
  }
  if (!ctx->started) {  // Taylor starter at t = 0, fixes dt
    HIPC(launch_schedule(ctx->p<double>(L.gtab), ctx->p<int64_t>(L.base), 1, dt, ctx->sched, st));
    const int32_t rc = run_starter(ctx, dt, st);
    if (rc != ENS_OK) return rc;
    ctx->started = true;
    ctx->dt = dt;
    ctx->gen++;
  }
  if (qoi && ctx->mask_live && ctx->SB < 64) {
    // lane-group steps keep q up to date and leave the rising bits alone:
    // fold in the rises that batched steps left open, then clear the bits
    HIPC(hipDeviceSynchronize());
    const int32_t rc = resolve_qoi(ctx);
    if (rc != ENS_OK) return rc;
    HIPC(hipMemset(ctx->p<void>(L.qmask), 0, sizeof(uint64_t) * ctx->n_nodes * ((ctx->ld + 63) / 64)));
    // the clear runs on the null stream: finish it before steps on `st`
    // (possibly a non-blocking stream) or a later batch step reads the bits
    HIPC(hipDeviceSynchronize());
    ctx->mask_live = false;
  }
  int64_t left = n_steps;
  // plain steps go in replays of a captured graph of kGraphSteps steps
  // (load-factor table, the steps, the step counter): the same kernels with
  // the same arguments as the direct launches below
  if (!geom && ctx->energy_every == 0 && left >= kGraphSteps) {
    if (ctx->exec && (ctx->graph_gen != ctx->gen || ctx->graph_cur != ctx->cur)) ctx->drop_graph();
    if (!ctx->exec) {
      if (!ctx->cap_st) HIPC(hipStreamCreateWithFlags(&ctx->cap_st, hipStreamNonBlocking));
      HIPC(hipStreamBeginCapture(ctx->cap_st, hipStreamCaptureModeThreadLocal));
      hipError_t e = launch_schedule(ctx->p<double>(L.gtab), ctx->p<int64_t>(L.base), kGraphSteps, dt,
                                     ctx->sched, ctx->cap_st);
      for (int j = 0; j < kGraphSteps && e == hipSuccess; ++j) {
        a.j = j;
        a.refresh = 0;
        set_state_ptrs(ctx, a, j & 1);
        e = launch_step(a, f32, ctx->state_prec, ctx->SB, qoi, false, use_shared(ctx), ctx->cap_st);
      }
      if (e == hipSuccess) e = launch_advance(ctx->p<int64_t>(L.base), kGraphSteps, ctx->cap_st);
      hipGraph_t g = nullptr;
      const hipError_t e2 = hipStreamEndCapture(ctx->cap_st, &g);
      if (e != hipSuccess || e2 != hipSuccess) {
        if (g) (void)hipGraphDestroy(g);
        return ctx->fail(ENS_EDEVICE, std::string("ens_step: graph capture: ") +
                                          hipGetErrorString(e != hipSuccess ? e : e2));
      }
      ctx->graph = g;
      HIPC(hipGraphInstantiate(&ctx->exec, ctx->graph, nullptr, nullptr, 0));
      ctx->graph_gen = ctx->gen;
      ctx->graph_cur = ctx->cur;
    }
    while (left >= kGraphSteps) {
      HIPC(hipGraphLaunch(ctx->exec, st));
      ctx->steps += kGraphSteps;
      left -= kGraphSteps;
    }
  }
  while (left > 0) {
    const int k = (int)std::min<int64_t>(left, kChunk);
    HIPC(launch_schedule(ctx->p<double>(L.gtab), ctx->p<int64_t>(L.base), k, dt, ctx->sched, st));
    for (int j = 0; j < k; ++j) {
      const int64_t n = ctx->steps + j;
      const bool energy = ctx->energy_every > 0 && (n % ctx->energy_every) == 0;
      a.j = j;
      // geometry refresh at step n: the kernel moves the force base to the
      // force at u_n, then u_n becomes the snapshot for steps n .. n+every-1
      const bool refresh = geom && n > 0 && n % ctx->geom_every == 0;
      a.refresh = refresh ? 1 : 0;
      set_state_ptrs(ctx, a, 0);
      HIPC(launch_step(a, f32, ctx->state_prec, ctx->SB, qoi, energy, use_shared(ctx) && !geom, st));
      if (refresh)
        HIPC(launch_copy_f64(3 * ctx->n_nodes * (int64_t)ctx->ld, ctx->p<double>(L.u[ctx->cur]),
                             ctx->p<double>(L.usnap), st));
      if (energy) {
        const int64_t rec = ctx->energy_records % kEnergyCap;
        HIPC(launch_energy_reduce(ctx->p<double>(L.epart), a.n_nb, ctx->ld, ctx->ld,
                                  ctx->p<double>(L.erec) + rec * ctx->ld, st));
        // watchdog: with omega_hat the stability bound's frequency and
        // s = omega_hat dt / 2 < 1, the discrete energy E_{n+1/2} is at least
        // (1 - s^2) times its kinetic part in any state (per mode
        // E = m/(2 dt^2) [(1 - W^2/4)(u_{n+1} - u_n)^2 + (W^2/4)(u_{n+1} + u_n)^2],
        // W = omega dt <= 2 s); a step that is not stable lets the kinetic
        // part grow while E stays bounded
        const double s_bound = std::min(0.5 * dt * std::sqrt(ctx->omega2), 0.999);
        const double coef = (1.0 - s_bound * s_bound) / 1.01;
        double* epart = ctx->p<double>(L.epart);
        double* ktmp = epart + (int64_t)(a.n_nb + 256) * ctx->ld;
        double* krow = epart + (int64_t)(a.n_nb + 512) * ctx->ld;
        Flags* fl = ctx->p<Flags>(L.flags);
        if (ctx->state_prec == ENS_STATE_F64)
          HIPC(launch_kinetic((int32_t)ctx->n_nodes, ctx->ld, ctx->S, ctx->p<double>(L.u[1 - ctx->cur]),
                              ctx->p<double>(L.u[ctx->cur]), nullptr, ctx->p<double>(L.minv64), dt, ktmp, krow,
                              ctx->p<double>(L.erec) + rec * ctx->ld, coef, &fl->unstable, st));
        else
          HIPC(launch_kinetic((int32_t)ctx->n_nodes, ctx->ld, ctx->S, nullptr, nullptr, ctx->p<float>(L.v),
                              ctx->p<double>(L.minv64), dt, ktmp, krow, ctx->p<double>(L.erec) + rec * ctx->ld,
                              coef, &fl->unstable, st));
        ctx->energy_steps[rec] = n;
        ctx->energy_records++;
      }
      ctx->cur = 1 - ctx->cur;
    }
    HIPC(launch_advance(ctx->p<int64_t>(L.base), k, st));
    ctx->steps += k;
    left -= k;
  }
  return ENS_OK;
  GUARD_END
}

int32_t ens_sync(ens_ctx* ctx) {
  if (!ctx) return ENS_EINVAL;
  if (!ctx->bound || !ctx->state_init) return ctx->fail(ENS_ESTATE, "ens_sync: nothing to wait for");
  HIPC(hipSetDevice(ctx->device));
  HIPC(hipDeviceSynchronize());
  const Layout& L = ctx->L;
  Flags* fl = ctx->p<Flags>(L.flags);
  HIPC(hipMemset(&fl->nonfinite, 0, sizeof(int32_t)));
  const int64_t n = 3 * ctx->n_nodes * (int64_t)ctx->ld;
  if (ctx->state_prec == ENS_STATE_F64)
    HIPC(launch_check_finite(n, ctx->p<double>(L.u[ctx->cur]), 0, &fl->nonfinite, nullptr));
  else
    HIPC(launch_check_finite(n, ctx->p<float>(L.uh[ctx->cur]), 1, &fl->nonfinite, nullptr));
  int32_t flags[2] = {0, 0};  // nonfinite, unstable
  HIPC(hipMemcpy(flags, &fl->nonfinite, sizeof flags, hipMemcpyDeviceToHost));
  if (flags[1])
    return ctx->fail(ENS_EUNSTABLE, "ens_sync: energy watchdog: the kinetic energy of a sample exceeded what a "
                                    "stable step allows for its discrete energy (the step is unstable)");
  if (flags[0]) return ctx->fail(ENS_ENONFINITE, "ens_sync: non-finite values in the displacement state");
  return ENS_OK;
}

int32_t ens_read_state(ens_ctx* ctx, double* u) {
  if (!ctx || !u) return ENS_EINVAL;
  GUARD_BEGIN
  if (!ctx->bound || !ctx->state_init) return ctx->fail(ENS_ESTATE, "ens_read_state: no state");
  HIPC(hipSetDevice(ctx->device));
  HIPC(hipDeviceSynchronize());
  const Layout& L = ctx->L;
  const int64_t ndof = 3 * ctx->n_nodes, n = ndof * ctx->ld;
  std::vector<double> buf(n);
  if (ctx->state_prec == ENS_STATE_F64) {
    HIPC(hipMemcpy(buf.data(), ctx->p<void>(L.u[ctx->cur]), sizeof(double) * n, hipMemcpyDeviceToHost));
  } else {
    const float* uc = ctx->state_prec == ENS_STATE_F32_KAHAN ? ctx->p<float>(L.uc) : nullptr;
    HIPC(launch_combine_f32(n, ctx->p<float>(L.uh[ctx->cur]), uc, ctx->p<double>(L.aux), nullptr));
    HIPC(hipMemcpy(buf.data(), ctx->p<void>(L.aux), sizeof(double) * n, hipMemcpyDeviceToHost));
  }
  unpad_rows(buf.data(), ndof, ctx->S, ctx->ld, u, &ctx->perm, 3);
  return ENS_OK;
  GUARD_END
}

int32_t ens_read_qoi(ens_ctx* ctx, int32_t kind, double* out) {
  if (!ctx || !out) return ENS_EINVAL;
  GUARD_BEGIN
  if (kind != ENS_QOI_PEAK_RADIAL) return ctx->fail(ENS_EINVAL, "ens_read_qoi: unknown kind");
  if (!(ctx->qoi_mask & ENS_QOI_PEAK_RADIAL)) return ctx->fail(ENS_ESTATE, "ens_read_qoi: QoI not enabled");
  if (!ctx->bound || !ctx->state_init) return ctx->fail(ENS_ESTATE, "ens_read_qoi: no state");
  HIPC(hipSetDevice(ctx->device));
  HIPC(hipDeviceSynchronize());
  {
    const int32_t rc = resolve_qoi(ctx);
    if (rc != ENS_OK) return rc;
  }
  const int64_t n = ctx->n_nodes * ctx->ld;
  std::vector<double> buf(n);
  HIPC(hipMemcpy(buf.data(), ctx->p<void>(ctx->L.q), sizeof(double) * n, hipMemcpyDeviceToHost));
  unpad_rows(buf.data(), ctx->n_nodes, ctx->S, ctx->ld, out, &ctx->perm, 1);
  return ENS_OK;
  GUARD_END
}

int32_t ens_read_energy(ens_ctx* ctx, int64_t max_records, int64_t* steps_out, double* e_out,
                        int64_t* n_out) {
  if (!ctx || !n_out || max_records < 0) return ENS_EINVAL;
  GUARD_BEGIN
  if (!ctx->bound || !ctx->state_init) return ctx->fail(ENS_ESTATE, "ens_read_energy: no state");
  HIPC(hipSetDevice(ctx->device));
  HIPC(hipDeviceSynchronize());
  const int64_t have = std::min<int64_t>(ctx->energy_records, kEnergyCap);
  const int64_t take = std::min<int64_t>(have, max_records);
  *n_out = take;
  if (take == 0) return ENS_OK;
  if (!steps_out || !e_out) return ctx->fail(ENS_EINVAL, "ens_read_energy: null output");
  std::vector<double> row(ctx->ld);
  for (int64_t k = 0; k < take; ++k) {
    const int64_t r = ctx->energy_records - take + k;
    const int64_t slot = r % kEnergyCap;
    HIPC(hipMemcpy(row.data(), ctx->p<double>(ctx->L.erec) + slot * ctx->ld, sizeof(double) * ctx->ld,
                   hipMemcpyDeviceToHost));
    std::memcpy(e_out + k * ctx->S, row.data(), sizeof(double) * ctx->S);
    steps_out[k] = ctx->energy_steps[slot];
  }
  return ENS_OK;
  GUARD_END
}

namespace {
// One stress component of the current state into the stress scratch
// ([n_el][ld], internal element order); axial in the caller's order.
int32_t stress_values(ens_ctx* ctx, const char* who, const double* axial, int32_t comp) {
  if (!(ctx->qoi_mask & ENS_QOI_STRESS))
    return ctx->fail(ENS_ESTATE, std::string(who) + ": enable ENS_QOI_STRESS in ens_configure first");
  if (!ctx->bound || !ctx->state_init) return ctx->fail(ENS_ESTATE, std::string(who) + ": no state");
  if (!axial) return ctx->fail(ENS_EINVAL, std::string(who) + ": null tangents");
  if (comp < ENS_STRESS_THETA_THETA || comp > ENS_STRESS_R_Z)
    return ctx->fail(ENS_EINVAL, std::string(who) + ": unknown stress component");
  const int64_t ne = ctx->n_el;
  std::vector<double> ax(3 * ne);
  for (int64_t e = 0; e < ne; ++e) {
    const double* a = axial + 3 * (int64_t)ctx->eperm[e];
    if (!std::isfinite(a[0]) || !std::isfinite(a[1]) || !std::isfinite(a[2]) ||
        !(a[0] * a[0] + a[1] * a[1] + a[2] * a[2] > 0.0))
      return ctx->fail(ENS_EINVAL, std::string(who) + ": tangent of element " + std::to_string(ctx->eperm[e]) +
                                       " is zero or not finite");
    for (int k = 0; k < 3; ++k) ax[3 * e + k] = a[k];
  }
  const Layout& L = ctx->L;
  HIPC(hipSetDevice(ctx->device));
  HIPC(hipDeviceSynchronize());
  double* vals = ctx->p<double>(L.stress);
  double* dax = vals + ne * ctx->ld;
  HIPC(hipMemcpy(dax, ax.data(), sizeof(double) * 3 * ne, hipMemcpyHostToDevice));
  Flags* fl = ctx->p<Flags>(L.flags);
  HIPC(hipMemset(&fl->bad, 0, sizeof(int32_t)));
  const bool f64 = ctx->state_prec == ENS_STATE_F64;
  const float* uc = ctx->state_prec == ENS_STATE_F32_KAHAN ? ctx->p<float>(L.uc) : nullptr;
  HIPC(launch_stress(ne, ctx->ld, ctx->p<int32_t>(L.tri), ctx->p<double>(L.frame),
                     f64 ? ctx->p<double>(L.u[ctx->cur]) : nullptr, f64 ? nullptr : ctx->p<float>(L.uh[ctx->cur]),
                     f64 ? nullptr : uc, ctx->p<double>(L.eh64), ctx->p<double>(L.h), dax, ctx->nu, ctx->shear_k,
                     comp, vals, &fl->bad, nullptr));
  int32_t bad = 0;
  HIPC(hipMemcpy(&bad, &fl->bad, sizeof(int32_t), hipMemcpyDeviceToHost));
  if (bad) return ctx->fail(ENS_EINVAL, std::string(who) + ": a tangent is parallel to its element's normal");
  return ENS_OK;
}
}  // namespace

int32_t ens_stress(ens_ctx* ctx, const double* axial, int32_t component, double* out) {
  if (!ctx || !out) return ENS_EINVAL;
  GUARD_BEGIN
  const int32_t rc = stress_values(ctx, "ens_stress", axial, component);
  if (rc != ENS_OK) return rc;
  std::vector<double> buf((size_t)ctx->n_el * ctx->ld);
  HIPC(hipMemcpy(buf.data(), ctx->p<void>(ctx->L.stress), sizeof(double) * buf.size(), hipMemcpyDeviceToHost));
  unpad_rows(buf.data(), ctx->n_el, ctx->S, ctx->ld, out, &ctx->eperm, 1);
  return ENS_OK;
  GUARD_END
}

int32_t ens_stress_bands(ens_ctx* ctx, const double* axial, int32_t component, double p_lo, double p_hi,
                         double* mean, double* lo, double* hi) {
  if (!ctx || !mean || !lo || !hi) return ENS_EINVAL;
  GUARD_BEGIN
  if (!(p_lo >= 0.0 && p_lo <= 1.0 && p_hi >= 0.0 && p_hi <= 1.0))
    return ctx->fail(ENS_EINVAL, "ens_stress_bands: quantile levels must lie in [0, 1]");
  if (ctx->S > kBandsMax)
    return ctx->fail(ENS_EUNSUPPORTED, "ens_stress_bands: at most " + std::to_string(kBandsMax) + " samples");
  const int32_t rc = stress_values(ctx, "ens_stress_bands", axial, component);
  if (rc != ENS_OK) return rc;
  const int64_t ne = ctx->n_el;
  double* vals = ctx->p<double>(ctx->L.stress);
  double* b = vals + ne * ctx->ld + 3 * ne;
  HIPC(launch_bands(ne, ctx->ld, ctx->S, vals, p_lo, p_hi, b, b + ne, b + 2 * ne, nullptr));
  std::vector<double> hb(3 * ne);
  HIPC(hipMemcpy(hb.data(), b, sizeof(double) * 3 * ne, hipMemcpyDeviceToHost));
  for (int64_t e = 0; e < ne; ++e) {
    const int64_t o = ctx->eperm[e];
    mean[o] = hb[e];
    lo[o] = hb[ne + e];
    hi[o] = hb[2 * ne + e];
  }
  return ENS_OK;
  GUARD_END
}

int32_t ens_moments(ens_ctx* ctx, double* mean, double* var) {
  if (!ctx || !mean || !var) return ENS_EINVAL;
  if (!(ctx->qoi_mask & ENS_QOI_PEAK_RADIAL)) return ctx->fail(ENS_ESTATE, "ens_moments: QoI not enabled");
  if (!ctx->bound || !ctx->state_init) return ctx->fail(ENS_ESTATE, "ens_moments: no state");
  HIPC(hipSetDevice(ctx->device));
  HIPC(hipDeviceSynchronize());
  {
    const int32_t rc = resolve_qoi(ctx);
    if (rc != ENS_OK) return rc;
  }
  const Layout& L = ctx->L;
  HIPC(launch_moments((int32_t)ctx->n_nodes, ctx->ld, ctx->S, ctx->p<double>(L.q), ctx->p<double>(L.mean),
                      ctx->p<double>(L.var), nullptr, nullptr));
  std::vector<double> hm(ctx->n_nodes), hv(ctx->n_nodes);
  HIPC(hipMemcpy(hm.data(), ctx->p<void>(L.mean), sizeof(double) * ctx->n_nodes, hipMemcpyDeviceToHost));
  HIPC(hipMemcpy(hv.data(), ctx->p<void>(L.var), sizeof(double) * ctx->n_nodes, hipMemcpyDeviceToHost));
  for (int64_t i = 0; i < ctx->n_nodes; ++i) {
    mean[ctx->perm[i]] = hm[i];
    var[ctx->perm[i]] = hv[i];
  }
  return ENS_OK;
}

int32_t ens_moments_noalloc(ens_ctx* ctx, double* mean, double* var) {
  if (!ctx || !mean || !var) return ENS_EINVAL;
  if (!(ctx->qoi_mask & ENS_QOI_PEAK_RADIAL))
    return ctx->fail(ENS_ESTATE, "ens_moments_noalloc: QoI not enabled");
  const size_t need = 2 * sizeof(double) * (size_t)ctx->n_nodes;
  if (need > kScratchBytes)
    return ctx->fail(ENS_EINVAL, "ens_moments_noalloc: " + std::to_string(ctx->n_nodes) +
                                     " nodes exceed the scratch limit of " +
                                     std::to_string(kScratchBytes / (2 * sizeof(double))) +
                                     " nodes (use ens_moments)");
  if (!ctx->bound || !ctx->state_init) return ctx->fail(ENS_ESTATE, "ens_moments_noalloc: no state");
  HIPC(hipSetDevice(ctx->device));
  double* dm = static_cast<double*>(scratch_ptr(ctx->device));
  if (!dm) return ctx->fail(ENS_EDEVICE, "ens_moments_noalloc: scratch address not set up for this device");
  double* dv = dm + ctx->n_nodes;
  HIPC(hipDeviceSynchronize());
  {
    const int32_t rc = resolve_qoi(ctx);
    if (rc != ENS_OK) return rc;
  }
  // every row is written, so nothing needs clearing; rows go straight to
  // the caller's numbering
  const Layout& L = ctx->L;
  HIPC(launch_moments((int32_t)ctx->n_nodes, ctx->ld, ctx->S, ctx->p<double>(L.q), dm, dv,
                      ctx->p<int32_t>(L.perm), nullptr));
  HIPC(hipMemcpy(mean, dm, sizeof(double) * ctx->n_nodes, hipMemcpyDeviceToHost));
  HIPC(hipMemcpy(var, dv, sizeof(double) * ctx->n_nodes, hipMemcpyDeviceToHost));
  return ENS_OK;
}

#ifndef ENSFEM_APPLY_WIDE
#define ENSFEM_APPLY_WIDE 1
#endif
int32_t ens_apply(ens_ctx* ctx, int32_t prec, const void* U_dev, void* R_dev, void* stream) {
  if (!ctx) return ENS_EINVAL;
  if (!ctx->bound) return ctx->fail(ENS_EWORKSPACE, "ens_apply: bind a workspace first");
  if (prec != ENS_F64 && prec != ENS_F32) return ctx->fail(ENS_EINVAL, "ens_apply: prec must be ENS_F64 or ENS_F32");
  if (!U_dev || !R_dev) return ctx->fail(ENS_EINVAL, "ens_apply: null device buffer");
  HIPC(hipSetDevice(ctx->device));
  StepArgs a = base_args(ctx, prec == ENS_F32);
  // the apply alone holds fewer values per sample than the step: a wave
  // can take 4 samples per lane where the padded width allows
  int sb = ctx->SB;
  if (ENSFEM_APPLY_WIDE && sb >= 64 && ctx->ld % 256 == 0) sb = 256;
  a.n_sb = ctx->ld / sb;
  HIPC(launch_apply(a, prec == ENS_F32, sb, use_shared(ctx), U_dev, R_dev, ctx->p<int32_t>(ctx->L.perm),
                    static_cast<hipStream_t>(stream)));
  return ENS_OK;
}

namespace {
struct CkptHeader {
  uint64_t magic;
  int64_t n_dof, ld, S, state_prec, steps, started, u0_zero;
  double dt;
};
constexpr uint64_t kMagic = 0x31764b43464e45ull;  // "ENFCKv1"
}  // namespace

int32_t ens_save(ens_ctx* ctx, void* host, size_t* bytes) {
  if (!ctx || !bytes) return ENS_EINVAL;
  GUARD_BEGIN
  if (!ctx->bound || !ctx->state_init) return ctx->fail(ENS_ESTATE, "ens_save: no state");
  if (ctx->geom_every > 0)
    return ctx->fail(ENS_EUNSUPPORTED, "ens_save: checkpoints do not hold the geometry snapshot");
  const Layout& L = ctx->L;
  const int64_t n = 3 * ctx->n_nodes * (int64_t)ctx->ld, nq = ctx->n_nodes * (int64_t)ctx->ld;
  const bool f64 = ctx->state_prec == ENS_STATE_F64;
  const size_t state_bytes = f64 ? 2 * sizeof(double) * n : 3 * sizeof(float) * n;
  const size_t need = sizeof(CkptHeader) + state_bytes + sizeof(double) * nq;
  if (!host) {
    *bytes = need;
    return ENS_OK;
  }
  if (*bytes < need) return ctx->fail(ENS_EINVAL, "ens_save: buffer too small");
  HIPC(hipSetDevice(ctx->device));
  HIPC(hipDeviceSynchronize());
  {
    const int32_t rc = resolve_qoi(ctx);
    if (rc != ENS_OK) return rc;
  }
  char* o = static_cast<char*>(host);
  CkptHeader hd{kMagic, 3 * ctx->n_nodes, ctx->ld, ctx->S, ctx->state_prec, ctx->steps, ctx->started ? 1 : 0,
                ctx->u0_zero ? 1 : 0, ctx->dt};
  std::memcpy(o, &hd, sizeof hd);
  o += sizeof hd;
  if (f64) {
    HIPC(hipMemcpy(o, ctx->p<void>(L.u[ctx->cur]), sizeof(double) * n, hipMemcpyDeviceToHost));
    o += sizeof(double) * n;
    HIPC(hipMemcpy(o, ctx->p<void>(L.u[1 - ctx->cur]), sizeof(double) * n, hipMemcpyDeviceToHost));
    o += sizeof(double) * n;
  } else {
    HIPC(hipMemcpy(o, ctx->p<void>(L.uh[ctx->cur]), sizeof(float) * n, hipMemcpyDeviceToHost));
    o += sizeof(float) * n;
    if (L.uc && ctx->state_prec == ENS_STATE_F32_KAHAN)
      HIPC(hipMemcpy(o, ctx->p<void>(L.uc), sizeof(float) * n, hipMemcpyDeviceToHost));
    else
      std::memset(o, 0, sizeof(float) * n);
    o += sizeof(float) * n;
    HIPC(hipMemcpy(o, ctx->p<void>(L.v), sizeof(float) * n, hipMemcpyDeviceToHost));
    o += sizeof(float) * n;
  }
  HIPC(hipMemcpy(o, ctx->p<void>(L.q), sizeof(double) * nq, hipMemcpyDeviceToHost));
  *bytes = need;
  return ENS_OK;
  GUARD_END
}

int32_t ens_load(ens_ctx* ctx, const void* host, size_t bytes) {
  if (!ctx || !host) return ENS_EINVAL;
  ctx->gen++;
  GUARD_BEGIN
  if (!ctx->bound) return ctx->fail(ENS_EWORKSPACE, "ens_load: bind a workspace first");
  if (ctx->geom_every > 0)
    return ctx->fail(ENS_EUNSUPPORTED, "ens_load: checkpoints do not hold the geometry snapshot");
  if (bytes < sizeof(CkptHeader)) return ctx->fail(ENS_EINVAL, "ens_load: truncated checkpoint");
  CkptHeader hd;
  std::memcpy(&hd, host, sizeof hd);
  const int64_t n = 3 * ctx->n_nodes * (int64_t)ctx->ld, nq = ctx->n_nodes * (int64_t)ctx->ld;
  if (hd.magic != kMagic || hd.n_dof != 3 * ctx->n_nodes || hd.ld != ctx->ld || hd.S != ctx->S ||
      hd.state_prec != ctx->state_prec)
    return ctx->fail(ENS_EINVAL, "ens_load: checkpoint does not match this context");
  const bool f64 = ctx->state_prec == ENS_STATE_F64;
  const size_t need = sizeof(CkptHeader) + (f64 ? 2 * sizeof(double) * n : 3 * sizeof(float) * n) + sizeof(double) * nq;
  if (bytes < need) return ctx->fail(ENS_EINVAL, "ens_load: truncated checkpoint");
  HIPC(hipSetDevice(ctx->device));
  HIPC(hipDeviceSynchronize());
  const Layout& L = ctx->L;
  const char* o = static_cast<const char*>(host) + sizeof hd;
  ctx->cur = 0;
  if (f64) {
    HIPC(hipMemcpy(ctx->p<void>(L.u[0]), o, sizeof(double) * n, hipMemcpyHostToDevice));
    o += sizeof(double) * n;
    HIPC(hipMemcpy(ctx->p<void>(L.u[1]), o, sizeof(double) * n, hipMemcpyHostToDevice));
    o += sizeof(double) * n;
  } else {
    HIPC(hipMemcpy(ctx->p<void>(L.uh[0]), o, sizeof(float) * n, hipMemcpyHostToDevice));
    o += sizeof(float) * n;
    if (ctx->state_prec == ENS_STATE_F32_KAHAN)
      HIPC(hipMemcpy(ctx->p<void>(L.uc), o, sizeof(float) * n, hipMemcpyHostToDevice));
    o += sizeof(float) * n;
    HIPC(hipMemcpy(ctx->p<void>(L.v), o, sizeof(float) * n, hipMemcpyHostToDevice));
    o += sizeof(float) * n;
  }
  HIPC(hipMemcpy(ctx->p<void>(L.q), o, sizeof(double) * nq, hipMemcpyHostToDevice));
  HIPC(hipMemcpy(ctx->p<void>(L.base), &hd.steps, sizeof(int64_t), hipMemcpyHostToDevice));
  ctx->mask_live = false;
  HIPC(hipMemset(ctx->p<void>(L.qmask), 0, sizeof(uint64_t) * ctx->n_nodes * ((ctx->ld + 63) / 64)));
  HIPC(hipMemset(&ctx->p<Flags>(L.flags)->unstable, 0, sizeof(int32_t)));
  HIPC(hipDeviceSynchronize());
  ctx->steps = hd.steps;
  ctx->started = hd.started != 0;
  ctx->u0_zero = hd.u0_zero != 0;
  ctx->dt = hd.dt;
  ctx->energy_records = 0;
  ctx->energy_steps.assign(kEnergyCap, -1);
  ctx->state_init = true;
  return ENS_OK;
  GUARD_END
}

int32_t ens_set_tuning(ens_ctx* ctx, int32_t sample_block, int32_t sb_inner) {
  if (!ctx) return ENS_EINVAL;
  ctx->gen++;
  if (sample_block != 0 && sample_block != 8 && sample_block != 16 && sample_block != 32 && sample_block != 64 &&
      sample_block != 128 && sample_block != 256)
    return ctx->fail(ENS_EINVAL, "ens_set_tuning: sample block must be 0 (auto), 8, 16, 32, 64, 128 or 256");
  ctx->tune_sb = sample_block;
  ctx->sb_inner = sb_inner ? 1 : 0;
  if (ctx->have_ens) {
    const int sb = pick_sample_block(ctx->S, sample_block);
    const int ld = ((ctx->S + sb - 1) / sb) * sb;
    if (sb != ctx->SB) {
      // the padded width may change: re-pad the fields, drop the binding
      std::vector<double> eh(ctx->n_el * (int64_t)ctx->S), h(eh.size());
      unpad_rows(ctx->eh.data(), ctx->n_el, ctx->S, ctx->ld, eh.data());
      unpad_rows(ctx->h.data(), ctx->n_el, ctx->S, ctx->ld, h.data());
      ctx->SB = sb;
      ctx->ld = ld;
      pad_rows(eh.data(), ctx->n_el, ctx->S, ld, ctx->eh);
      pad_rows(h.data(), ctx->n_el, ctx->S, ld, ctx->h);
      ctx->bound = false;
      ctx->state_init = false;
    }
  }
  return ENS_OK;
}

}  // extern "C"

// ---------------------------------------------------------------------------
// Batching: several contexts stepped by one launch per step (or one per lane
// class), the step loop captured in a hipGraph, tiling chosen by a timing
// autotuner.
// ---------------------------------------------------------------------------

struct ens_batch {
  std::vector<ens_ctx*> ctx;
  int device = 0;
  bool apply_f32 = false, qoi = true;
  int mode = 0;
  // tuning
  int spl = 1, tile_nodes = 4;  // nodes per tile: one per wave of the workgroup (set at creation)
  double tuned_ms = 0.0;
  // device tables (small, owned)
  BatchTile* d_tiles = nullptr;
  int32_t n_tiles = 0, n_wide = 0;  // split: tiles [0, n_wide) are full blocks, the rest tails
  bool split = false;               // one launch per lane class (full, tail) instead of one per step
  bool concurrent = false;          // split: the tail launches on a second stream (st2)
  size_t tiles_cap = 0;
  StepArgs* d_desc = nullptr;
  std::vector<int> desc_cur;
  std::vector<uint64_t> desc_gen;
  // captured chunk of graph_k steps
  hipGraph_t graph = nullptr;
  hipGraphExec_t exec = nullptr;
  int graph_k = 64;
  std::vector<uint64_t> graph_gen;
  int graph_sig[3] = {0, 0, 0};
  hipStream_t st = nullptr;
  hipEvent_t ev_in = nullptr, ev_out = nullptr;
  hipStream_t st2 = nullptr;  // concurrent tails
  hipEvent_t ev_fork = nullptr, ev_join = nullptr;
  std::string err;
  int32_t fail(int32_t code, const std::string& m) {
    err = m;
    return code;
  }
};

namespace {

#define BHIPC(expr)                                                                              \
  do {                                                                                           \
    hipError_t e_ = (expr);                                                                      \
    if (e_ != hipSuccess)                                                                        \
      return b->fail(ENS_EDEVICE, std::string("HIP error: ") + hipGetErrorString(e_) + " at " #expr); \
  } while (0)

void drop_graph(ens_batch* b) {
  if (b->exec) (void)hipGraphExecDestroy(b->exec);
  if (b->graph) (void)hipGraphDestroy(b->graph);
  b->exec = nullptr;
  b->graph = nullptr;
}

// Tiles of `tile_nodes` (= 4, one per wave) consecutive nodes times one
// sample block, mesh by mesh.  With spl = 2 a mesh's samples go in blocks
// of 128 (2 per lane) while 128 remain, a remainder of 96 in one block on
// 48 lanes, then a tail block of 64 or 32; with
// spl = 1 in blocks of 64 and a last one of 32 when the padded width is an
// odd multiple of 32.  Within a mesh the order is node tile by node tile
// with the sample blocks together (or block by block, see
// ENSFEM_BATCH_NODE_MAJOR).  Split: the full blocks first, then the tails
// (one launch each); else tails stay in place.
int32_t build_tiles(ens_batch* b) {
  std::vector<BatchTile> wide, narrow;
  const int blk = 64 * b->spl;
  for (size_t m = 0; m < b->ctx.size(); ++m) {
    const ens_ctx* c = b->ctx[m];
    // a block is wide (the spl launch) when it holds 64 * spl samples, or,
    // at spl = 2, more than 64 (a 96-sample remainder on 48 lanes); the
    // rest (64 or 32 samples) is a tail run at one sample per lane
    auto wide_at = [&](int s0) { return c->ld - s0 >= blk || (b->spl == 2 && c->ld - s0 > 64); };
    std::vector<int> starts;
    for (int s0 = 0; s0 < c->ld; s0 += wide_at(s0) ? std::min(blk, c->ld - s0) : 64) starts.push_back(s0);
    auto put = [&](int64_t n0, int s0) {
      const bool tail = !wide_at(s0);
      const int32_t cnt = (int32_t)std::min<int64_t>(b->tile_nodes, c->n_nodes - n0);
      (tail && b->split ? narrow : wide).push_back(BatchTile{(int32_t)m, (int32_t)n0, cnt | (tail ? kTileTail : 0), s0});
    };
    if (ENSFEM_BATCH_NODE_MAJOR) {
      for (int64_t n0 = 0; n0 < c->n_nodes; n0 += b->tile_nodes)
        for (int s0 : starts) put(n0, s0);
    } else {
      for (int s0 : starts)
        for (int64_t n0 = 0; n0 < c->n_nodes; n0 += b->tile_nodes) put(n0, s0);
    }
  }
  if (!b->split) {
    // one launch: each XCD's eighth of the list (the kernel's slices) runs
    // its full blocks first, then its tails (8.24 against 8.69 ms per step
    // on the 16-tube batch with the two kinds interleaved)
    const size_t n = wide.size();
    for (int x = 0; x < 8; ++x)
      std::stable_partition(wide.begin() + n * x / 8, wide.begin() + n * (x + 1) / 8,
                            [](const BatchTile& t) { return (t.count & kTileTail) == 0; });
  }
  b->n_wide = (int32_t)wide.size();
  b->n_tiles = (int32_t)(wide.size() + narrow.size());
  std::vector<BatchTile> tiles(wide);
  tiles.insert(tiles.end(), narrow.begin(), narrow.end());
  if (tiles.size() > b->tiles_cap) {
    if (b->d_tiles) BHIPC(hipFree(b->d_tiles));
    b->d_tiles = nullptr;
    BHIPC(hipMalloc(&b->d_tiles, sizeof(BatchTile) * tiles.size()));
    b->tiles_cap = tiles.size();
  }
  if (!tiles.empty())
    BHIPC(hipMemcpy(b->d_tiles, tiles.data(), sizeof(BatchTile) * tiles.size(), hipMemcpyHostToDevice));
  drop_graph(b);
  return ENS_OK;
}

// Per-mesh step arguments for both parities, relative to each context's
// current buffer.
int32_t build_desc(ens_batch* b) {
  std::vector<StepArgs> d(2 * b->ctx.size());
  for (size_t m = 0; m < b->ctx.size(); ++m) {
    ens_ctx* c = b->ctx[m];
    for (int par = 0; par < 2; ++par) {
      StepArgs a = base_args(c, b->apply_f32);
      a.dt = c->dt;
      a.a = 0.5 * c->alpha * c->dt;
      set_state_ptrs(c, a, par);
      d[2 * m + par] = a;
    }
    b->desc_cur[m] = c->cur;
    b->desc_gen[m] = c->gen;
  }
  BHIPC(hipMemcpyAsync(b->d_desc, d.data(), sizeof(StepArgs) * d.size(), hipMemcpyHostToDevice, b->st));
  BHIPC(hipStreamSynchronize(b->st));
  return ENS_OK;
}

int32_t check_ready(ens_batch* b) {
  for (size_t m = 0; m < b->ctx.size(); ++m) {
    const ens_ctx* c = b->ctx[m];
    if (!c->bound || !c->state_init || !c->started || !c->have_load)
      return b->fail(ENS_ESTATE, "batch mesh " + std::to_string(m) +
                                     ": bind, init the state and fix dt (ens_step with 0 steps) first");
  }
  return ENS_OK;
}

// Enqueue k steps of every mesh on b->st: per chunk of at most kChunk steps
// the load-factor tables, one launch per step, then the step counters.
// kChunk is even, so step j of a chunk has the parity of j.
static_assert(kChunk % 2 == 0, "chunks must keep the state parity");
int32_t enqueue_steps(ens_batch* b, int64_t k_total) {
  for (int64_t done = 0; done < k_total;) {
    const int k = (int)std::min<int64_t>(k_total - done, kChunk);
    for (ens_ctx* c : b->ctx)
      BHIPC(launch_schedule(c->p<double>(c->L.gtab), c->p<int64_t>(c->L.base), k, c->dt, c->sched, b->st));
    // one launch per step covers both lane classes (the tail blocks on the
    // lower lanes), or, split, one launch for the full blocks and one with a
    // sample per lane for the tails.  Concurrent: the tails of the whole
    // chunk run on a second stream beside the full blocks (their sample
    // columns and rising-bit words are disjoint from the full blocks', so
    // the two chains of steps share nothing but the load factors), joined
    // before the step counters advance.
    const int32_t n_tail = b->n_tiles - b->n_wide;
    const bool two = b->concurrent && b->n_wide > 0 && n_tail > 0;
    hipStream_t ts = b->st;
    if (two) {
      BHIPC(hipEventRecord(b->ev_fork, b->st));
      BHIPC(hipStreamWaitEvent(b->st2, b->ev_fork, 0));
      ts = b->st2;
    }
    for (int j = 0; j < k; ++j) {
      BHIPC(launch_batch_step(b->d_tiles, b->n_wide, b->spl, b->d_desc, j, b->apply_f32, b->mode, b->qoi, b->st));
      BHIPC(launch_batch_step(b->d_tiles + b->n_wide, n_tail, 1, b->d_desc, j, b->apply_f32, b->mode, b->qoi, ts));
    }
    if (two) {
      BHIPC(hipEventRecord(b->ev_join, b->st2));
      BHIPC(hipStreamWaitEvent(b->st, b->ev_join, 0));
    }
    for (ens_ctx* c : b->ctx) BHIPC(launch_advance(c->p<int64_t>(c->L.base), k, b->st));
    done += k;
  }
  return ENS_OK;
}

void after_steps(ens_batch* b, int64_t n) {
  for (ens_ctx* c : b->ctx) {
    c->steps += n;
    if (n & 1) c->cur ^= 1;
    if (b->qoi && n > 0) c->mask_live = true;
  }
}

}  // namespace

extern "C" {

int32_t ens_batch_create(ens_ctx** ctxs, int32_t n, ens_batch** out) {
  if (!ctxs || n < 1 || !out) return ENS_EINVAL;
  *out = nullptr;
  ens_batch* b = new (std::nothrow) ens_batch();
  if (!b) return ENS_EINVAL;
  b->ctx.assign(ctxs, ctxs + n);
  const ens_ctx* c0 = ctxs[0];
  for (int i = 0; i < n; ++i) {
    const ens_ctx* c = ctxs[i];
    std::string why;
    if (!c) why = "null context";
    else if (!c->bound) why = "workspace not bound";
    else if (c->device != c0->device) why = "contexts on different devices";
    else if (c->apply_prec != c0->apply_prec || c->state_prec != c0->state_prec)
      why = "all meshes need the same apply and state precision";
    else if ((c->qoi_mask & ENS_QOI_PEAK_RADIAL) != (c0->qoi_mask & ENS_QOI_PEAK_RADIAL))
      why = "all meshes need the same QoI setting";
    else if (c->energy_every != 0) why = "energy records are not available in batched stepping";
    else if (c->geom_every != 0) why = "the geometry refresh is not available in batched stepping";
    else if (use_shared(c)) why = "batched stepping uses the element-by-element variant only";
    else if (c->ld % 32 != 0)
      why = "padded width must be a multiple of 32 (ens_set_tuning(ctx, 32, 0) or wider before binding)";
    for (int j = 0; j < i && why.empty(); ++j)
      if (ctxs[j] == c) why = "context listed twice";
    if (!why.empty()) {
      delete b;
      if (c) const_cast<ens_ctx*>(c)->err = "ens_batch_create: mesh " + std::to_string(i) + ": " + why;
      return ENS_EINVAL;
    }
  }
  b->device = c0->device;
  b->apply_f32 = c0->apply_prec == ENS_F32;
  b->mode = c0->state_prec;
  b->qoi = (c0->qoi_mask & ENS_QOI_PEAK_RADIAL) != 0;
  b->tile_nodes = kBlock / 64;
  b->spl = 2;
  b->desc_cur.assign(n, -1);
  b->desc_gen.assign(n, ~0ull);
  if (hipSetDevice(b->device) != hipSuccess || hipStreamCreate(&b->st) != hipSuccess ||
      hipStreamCreate(&b->st2) != hipSuccess || hipEventCreateWithFlags(&b->ev_in, hipEventDisableTiming) != hipSuccess ||
      hipEventCreateWithFlags(&b->ev_out, hipEventDisableTiming) != hipSuccess ||
      hipEventCreateWithFlags(&b->ev_fork, hipEventDisableTiming) != hipSuccess ||
      hipEventCreateWithFlags(&b->ev_join, hipEventDisableTiming) != hipSuccess ||
      hipMalloc(&b->d_desc, sizeof(StepArgs) * 2 * n) != hipSuccess) {
    (void)ens_batch_destroy(b);  // releases whatever was created
    return ENS_EDEVICE;
  }
  if (build_tiles(b) != ENS_OK) {
    (void)ens_batch_destroy(b);
    return ENS_EDEVICE;
  }
  *out = b;
  return ENS_OK;
}

int32_t ens_batch_destroy(ens_batch* b) {
  if (!b) return ENS_EINVAL;
  // teardown: errors here have no caller to go to
  (void)hipSetDevice(b->device);
  (void)hipDeviceSynchronize();
  drop_graph(b);
  if (b->d_tiles) (void)hipFree(b->d_tiles);
  if (b->d_desc) (void)hipFree(b->d_desc);
  if (b->ev_in) (void)hipEventDestroy(b->ev_in);
  if (b->ev_out) (void)hipEventDestroy(b->ev_out);
  if (b->ev_fork) (void)hipEventDestroy(b->ev_fork);
  if (b->ev_join) (void)hipEventDestroy(b->ev_join);
  if (b->st2) (void)hipStreamDestroy(b->st2);
  if (b->st) (void)hipStreamDestroy(b->st);
  delete b;
  return ENS_OK;
}

const char* ens_batch_last_error(const ens_batch* b) { return b ? b->err.c_str() : "null batch"; }

int32_t ens_batch_info(ens_batch* b, ens_batch_info_t* out) {
  if (!b || !out) return ENS_EINVAL;
  out->n_meshes = (int32_t)b->ctx.size();
  out->n_tiles = b->n_tiles;
  out->samples_per_lane = b->spl;
  out->tile_nodes = b->tile_nodes;
  out->grid = 0;
  out->graph_steps = b->graph_k;
  out->launches_per_step = (b->n_wide > 0 ? 1 : 0) + (b->n_tiles > b->n_wide ? 1 : 0);
  out->concurrent_tails = b->concurrent && b->n_wide > 0 && b->n_tiles > b->n_wide ? 1 : 0;
  out->tuned_ms_per_step = b->tuned_ms;
  return ENS_OK;
}

int32_t ens_batch_step(ens_batch* b, int64_t n_steps, void* stream) {
  if (!b) return ENS_EINVAL;
  try {
    if (n_steps < 0) return b->fail(ENS_EINVAL, "ens_batch_step: n_steps must be >= 0");
    int32_t rc = check_ready(b);
    if (rc != ENS_OK) return rc;
    BHIPC(hipSetDevice(b->device));
    hipStream_t user = static_cast<hipStream_t>(stream);
    BHIPC(hipEventRecord(b->ev_in, user));
    BHIPC(hipStreamWaitEvent(b->st, b->ev_in, 0));
    bool stale = false;
    for (size_t m = 0; m < b->ctx.size(); ++m)
      if (b->desc_cur[m] != b->ctx[m]->cur || b->desc_gen[m] != b->ctx[m]->gen) stale = true;
    if (stale) {
      rc = build_desc(b);
      if (rc != ENS_OK) return rc;
    }
    std::vector<uint64_t> gen(b->ctx.size());
    for (size_t m = 0; m < b->ctx.size(); ++m) gen[m] = b->ctx[m]->gen;
    const int sig[3] = {b->spl * (b->split ? -1 : 1), b->tile_nodes, b->concurrent ? 1 : 0};
    if (b->exec && (gen != b->graph_gen || std::memcmp(sig, b->graph_sig, sizeof sig) != 0)) drop_graph(b);
    int64_t left = n_steps;
    if (left >= b->graph_k) {
      if (!b->exec) {
        BHIPC(hipStreamBeginCapture(b->st, hipStreamCaptureModeThreadLocal));
        rc = enqueue_steps(b, b->graph_k);
        hipGraph_t g = nullptr;
        const hipError_t e = hipStreamEndCapture(b->st, &g);
        if (rc != ENS_OK) return rc;
        if (e != hipSuccess) return b->fail(ENS_EDEVICE, std::string("graph capture: ") + hipGetErrorString(e));
        b->graph = g;
        BHIPC(hipGraphInstantiate(&b->exec, b->graph, nullptr, nullptr, 0));
        b->graph_gen = gen;
        std::memcpy(b->graph_sig, sig, sizeof sig);
      }
      while (left >= b->graph_k) {  // graph_k is even: parities are unchanged per replay
        BHIPC(hipGraphLaunch(b->exec, b->st));
        after_steps(b, b->graph_k);
        left -= b->graph_k;
      }
    }
    if (left > 0) {
      rc = enqueue_steps(b, (int)left);
      if (rc != ENS_OK) return rc;
      after_steps(b, left);
    }
    BHIPC(hipEventRecord(b->ev_out, b->st));
    BHIPC(hipStreamWaitEvent(user, b->ev_out, 0));
    for (ens_ctx* c : b->ctx) c->last_stream = user;
    return ENS_OK;
  } catch (...) {
    return b->fail(ENS_EINVAL, "ens_batch_step: host failure");
  }
}

int32_t ens_batch_set_tiling(ens_batch* b, int32_t samples_per_lane, int32_t split) {
  if (!b) return ENS_EINVAL;
  try {
    if ((samples_per_lane != 1 && samples_per_lane != 2) || split < 0 || split > 2)
      return b->fail(ENS_EINVAL, "ens_batch_set_tiling: samples_per_lane must be 1 or 2 and split 0, 1 or 2");
    BHIPC(hipSetDevice(b->device));
    b->spl = samples_per_lane;
    b->split = split != 0;
    b->concurrent = split == 2;
    return build_tiles(b);
  } catch (...) {
    return b->fail(ENS_EINVAL, "ens_batch_set_tiling: host failure");
  }
}

int32_t ens_batch_autotune(ens_batch* b, int32_t trial_steps) {
  if (!b) return ENS_EINVAL;
  try {
    if (trial_steps < 1) return b->fail(ENS_EINVAL, "ens_batch_autotune: trial_steps must be >= 1");
    int32_t rc = check_ready(b);
    if (rc != ENS_OK) return rc;
    BHIPC(hipSetDevice(b->device));
    hipEvent_t e0, e1;
    BHIPC(hipEventCreate(&e0));
    BHIPC(hipEventCreate(&e1));
    double best = 1e300;
    int bs = b->spl;
    int bsplit = b->split ? (b->concurrent ? 2 : 1) : 0;
    // 1: one sample per lane; 2: two, one launch; 3: two, a launch per class;
    // 4: as 3 with the tails on a second stream
    for (int mode : {1, 2, 3, 4}) {
      const int spl = mode == 1 ? 1 : 2;
      b->split = mode >= 3;
      b->concurrent = mode == 4;
      b->spl = spl;
      rc = build_tiles(b);
      if (rc == ENS_OK) rc = build_desc(b);
      if (rc == ENS_OK) rc = enqueue_steps(b, 2);  // warm-up, even: parities unchanged
      if (rc != ENS_OK) break;
      after_steps(b, 2);
      hipError_t e = hipEventRecord(e0, b->st);
      if (e == hipSuccess) rc = enqueue_steps(b, trial_steps);
      if (rc != ENS_OK) break;
      if (e == hipSuccess) e = hipEventRecord(e1, b->st);
      if (e == hipSuccess) e = hipEventSynchronize(e1);
      float ms = 0.f;
      if (e == hipSuccess) e = hipEventElapsedTime(&ms, e0, e1);
      if (e != hipSuccess) {
        rc = b->fail(ENS_EDEVICE, std::string("ens_batch_autotune: ") + hipGetErrorString(e));
        break;
      }
      after_steps(b, trial_steps);
      if (ms / trial_steps < best) {
        best = ms / trial_steps;
        bs = spl;
        bsplit = mode == 4 ? 2 : mode == 3 ? 1 : 0;
      }
      if (trial_steps & 1) {
        rc = build_desc(b);
        if (rc != ENS_OK) break;
      }
    }
    (void)hipEventDestroy(e0);
    (void)hipEventDestroy(e1);
    if (rc != ENS_OK) return rc;
    b->spl = bs;
    b->split = bsplit != 0;
    b->concurrent = bsplit == 2;
    b->tuned_ms = best;
    rc = build_tiles(b);
    if (rc != ENS_OK) return rc;
    return build_desc(b);
  } catch (...) {
    return b->fail(ENS_EINVAL, "ens_batch_autotune: host failure");
  }
}

}  // extern "C"
