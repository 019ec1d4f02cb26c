// Internal declarations shared by the HIP sources of libbfc.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

#include <string>
#include <vector>

#include "../../include/bfc.h"

namespace bfc {

// ---------------------------------------------------------------------------
// errors
// ---------------------------------------------------------------------------
void set_error(const std::string& msg);

struct Status {
  bfc_status code = BFC_OK;
  std::string msg;
};

#define BFC_HIP_TRY(expr)                                                   \
  do {                                                                      \
    hipError_t _e = (expr);                                                 \
    if (_e != hipSuccess) {                                                 \
      ::bfc::set_error(std::string(#expr) + ": " + hipGetErrorString(_e));  \
      return (_e == hipErrorOutOfMemory) ? BFC_ENOMEM : BFC_EHIP;           \
    }                                                                       \
  } while (0)

#define BFC_TRY(...)                 \
  do {                               \
    bfc_status _s = (__VA_ARGS__);   \
    if (_s != BFC_OK) return _s;     \
  } while (0)

// ---------------------------------------------------------------------------
// complex helpers (interleaved re/im)
// ---------------------------------------------------------------------------
template <typename T>
struct cx {
  T x, y;
};

template <typename T>
__host__ __device__ inline cx<T> cmul(cx<T> a, cx<T> b) {
  return {a.x * b.x - a.y * b.y, a.x * b.y + a.y * b.x};
}
// acc += a * b
template <typename T>
__host__ __device__ inline void cfma(cx<T>& acc, cx<T> a, cx<T> b) {
  acc.x = fma(a.x, b.x, acc.x);
  acc.x = fma(-a.y, b.y, acc.x);
  acc.y = fma(a.x, b.y, acc.y);
  acc.y = fma(a.y, b.x, acc.y);
}
// acc += conj(a) * b
template <typename T>
__host__ __device__ inline void cfma_conj(cx<T>& acc, cx<T> a, cx<T> b) {
  acc.x = fma(a.x, b.x, acc.x);
  acc.x = fma(a.y, b.y, acc.x);
  acc.y = fma(a.x, b.y, acc.y);
  acc.y = fma(-a.y, b.x, acc.y);
}

// ---------------------------------------------------------------------------
// problem state
// ---------------------------------------------------------------------------
// Entries per subgroup: runs of one inner slice's row (or column) are cut into
// pieces of at most this many entries, one lane each in the Gram kernel.
constexpr int kSubgroup = 8;
constexpr int kSubRec = 4 + kSubgroup;  // int32 values per subgroup record

// Highest rank of the one-wavefront kernels and of every call of the library;
// ranks kNarrowRank+1 .. BFC_MAX_RANK have the sweep, reconstruction and
// residual calls only (fused per-slice kernels, one work item per slice).
constexpr int kNarrowRank = 8;
static_assert(kNarrowRank == BFC_MAX_RANK_FULL, "narrow kernel range");

struct WorkItem {   // a run of subgroups of one inner-core slice, one wavefront
  int32_t tile, sub0, sub1, pad;
};

struct CoreLayout {
  int32_t nblocks = 0;
  int32_t* rows = nullptr;     // entries sorted for this core
  int32_t* cols = nullptr;
  void* vals = nullptr;        // compute precision complex
  int32_t* perm = nullptr;     // input position of every sorted entry
  int32_t* blk_off = nullptr;  // nblocks + 1
  // inner cores only
  int32_t group_by_row = 1;
  int32_t group_extent = 1;    // rows (or columns) per slice tile
  int32_t nruns = 0;           // distinct (slice, row|column) pairs with entries
  int32_t nsub = 0;
  int32_t* sub_off = nullptr;  // nsub + 1
  // nsub records of kSubRec values, read by the FP32 / FP64 Gram at ranks
  // <= kNarrowRank (null otherwise): first entry, entry count, the node of
  // the environment the subgroup shares, 0, then the node of the other
  // environment for each of its kSubgroup entries (-1 past the count), so a
  // lane has all of a subgroup's indices after one round of loads
  int32_t* sub_rec = nullptr;
  int32_t nitems = 0;
  WorkItem* items = nullptr;
  int32_t* tile_items = nullptr;  // nblocks + 1: item range of each slice
  int32_t items_cap = 0;          // WorkItems the items array holds
  std::vector<int32_t> tile_sub;  // host: first subgroup of each slice, nblocks + 1
  // environment node of every sorted entry (nullptr where the environment is
  // a row of Z^1 or of Z^(L+2) itself)
  int32_t* lnode = nullptr;
  int32_t* rnode = nullptr;
  // outer cores at L >= 2 and ranks <= kNarrowRank: for every sorted entry,
  // 2 x its node on the trie level next to the outermost one (right level 1
  // for core 0, left level L for core L+1) plus the bit that picks which of
  // the fiber's two slices of the adjacent inner core (Z^2, Z^(L+1)) turns
  // that node into the entry's environment (null otherwise)
  int32_t* up_node = nullptr;
};

// One level of the environment trie.  Right level p (0 <= p < L) holds the
// distinct right environments of core p, one per (u = ib >> p, column j)
// present in the observed set, ordered by (u, j); left level p (2 <= p <= L+1)
// the distinct left environments of core p, one per (w = jb >> (L-p+1), row i),
// ordered by (w, i).  Each node is one r x r product away from its parent on
// the adjacent level (or from a row of Z^(L+2) / Z^1 at the ends).
struct EnvLevel {
  int32_t count = 0;
  int32_t* node_a = nullptr;   // u (right) or w (left)
  int32_t* node_b = nullptr;   // column j (right) or row i (left)
  int32_t* parent = nullptr;   // node on the adjacent level, or the j / i row
  void* vec = nullptr;         // count x r complex, compute precision
  bool valid = false;          // computed from the current cores
};

// per-kernel timing with HIP events (enabled by bfc_profile_enable)
enum { KIND_OUTER = 0, KIND_INNER_GRAM = 1, KIND_INNER_SOLVE = 2, KIND_RESIDUAL = 3,
       KIND_PREDICT = 4, KIND_ENV = 5, KIND_INNER_IR = 6, KIND_COUNT = 7 };

struct Profiler {
  bool on = false;
  std::vector<hipEvent_t> pool;
  std::vector<std::pair<hipEvent_t, hipEvent_t>> pending[KIND_COUNT];
  double total_ms[KIND_COUNT] = {};
  int64_t launches[KIND_COUNT] = {};
  hipEvent_t take();
};

// Records a start event on construction and a stop event on destruction
// around the kernel launches of one kind, when profiling is on.
struct ProfScope {
  Profiler* pr;
  int kind;
  hipStream_t st;
  hipEvent_t a = nullptr, b = nullptr;
  ProfScope(Profiler* pr_, int kind_, hipStream_t st_);
  ~ProfScope();
};

struct Problem {
  mutable Profiler prof;
  bfc_config cfg{};
  int64_t n = 0;
  int32_t L = 0, r = 0, c = 0;
  int32_t prec = BFC_C128;
  int64_t nnz = 0;
  size_t elem = 16;                  // bytes of one complex compute value
  void* cores = nullptr;             // compute precision
  std::vector<int64_t> core_off;     // complex element offset of each core
  int64_t nparams = 0;
  std::vector<CoreLayout> lay;       // L+2
  void* partials = nullptr;          // inner Gram partial sums
  size_t partials_bytes = 0;
  int32_t* flags = nullptr;          // [0] solve failures since last report
  // refinement of the BF16-Gram solves: per-item partial residual vectors,
  // and per slice the regularization used and the slice before the update
  void* ir_part = nullptr;
  double* ir_lam = nullptr;
  void* ir_old = nullptr;
  void* ir_fac = nullptr;            // BF16-Gram mode: each slice's factor, for the refinement
  double* red = nullptr;             // residual reduction scratch
  // ADAM (bfc_adam_sweep): first moments (complex), second moments (real),
  // both in the cores' layout, and per-item residual vectors; allocated at
  // the first ADAM call
  void* adam_m = nullptr;
  void* adam_v = nullptr;
  void* adam_part = nullptr;
  int32_t adam_part_items = 0;
  void* adf_dir = nullptr;           // ADF directions of an inner core's slices
  void* grad = nullptr;              // per-core gradients (bfc_loss_gradient)
  int32_t* bad_flag = nullptr;       // non-finite value seen by bfc_set_values
  double* batch_res = nullptr;       // bfc_loss_gradient_batch: 2 residual norms per instance
  int32_t batch_res_cap = 0;         // instances batch_res holds
  double* fused_res = nullptr;       // 2 per fiber of the last core: residual norms
  bool fused_res_valid = false;      // fused_res belongs to the current cores
  bool graph_fused_res = false;      // a replay of sweep_graph leaves fused_res valid
  size_t red_len = 0;
  double* red_host = nullptr;        // pinned, 2 doubles
  std::vector<void*> allocs;         // everything hipMalloc'd
  int32_t max_items = 0;
  int32_t item_size = 0;             // subgroups per work item (0: automatic rule)
  int64_t layout_version = 0;        // bumped when work items are rebuilt
  // one full sweep captured as a HIP graph (launched by bfc_sweep when
  // graphs are enabled and per-kernel profiling is off)
  bool use_graph = true;
  hipGraph_t sweep_graph = nullptr;
  hipGraphExec_t sweep_exec = nullptr;
  std::vector<EnvLevel> rlev;        // index p = 0..L-1
  std::vector<EnvLevel> llev;        // index p = 2..L+1 (0, 1 unused)
  int64_t env_bytes = 0;
};

bfc_status dev_alloc(Problem* P, void** ptr, size_t bytes);
// Every device allocation of the library goes through lib_malloc, so that the
// out-of-memory paths can be exercised (bfc_debug_fail_allocation_after).
hipError_t lib_malloc(void** ptr, size_t bytes);
int64_t debug_fail_allocation_after(int64_t count);

// One launch of a batched sweep: a kernel kind at one rank, over tasks (one
// per problem taking part) whose argument structs and block prefix table live
// in device memory.
// BK_OUTER_UP1 / BK_OUTER_UP2: the outer updates of core 0 / core L+1 that
// form their entries' environments from the level above (CoreLayout::up_node)
enum { BK_ENV_RIGHT = 0, BK_ENV_LEFT = 1, BK_OUTER = 2, BK_GRAM_ROW = 3, BK_GRAM_COL = 4,
       BK_SOLVE = 5, BK_RES = 6, BK_RES_FINAL = 7, BK_RES_FUSED = 8, BK_OUTER_UP1 = 9,
       BK_OUTER_UP2 = 10 };
struct BatchLaunch {
  int kind = 0, r = 0;
  void* tasks = nullptr;        // device array of argument structs
  int32_t* block_off = nullptr; // device, ntasks + 1
  int ntasks = 0;
  int64_t blocks = 0;
};

// Independent problems swept together: each launch covers the same kernel
// kind of every problem that needs it at that step of the sweep.
struct Batch {
  std::vector<Problem*> probs;
  std::vector<int64_t> versions;   // layout_version of each problem when planned
  int prec = BFC_C64;
  std::vector<BatchLaunch> sweep;  // one sweep of every problem, in dependency order
  std::vector<BatchLaunch> resid;  // observed-set residual norms of every problem
  std::vector<BatchLaunch> resid_fused;  // the same from the last core's per-fiber sums
  double* res = nullptr;           // device, 2 per problem
  double* res_host = nullptr;      // pinned, 2 per problem
  std::vector<void*> allocs;       // device memory of the plan
  hipGraph_t graph = nullptr;
  hipGraphExec_t exec = nullptr;
};
bfc_status build_batch_plan(Batch* B);
void free_batch_plan(Batch* B);
bfc_status launch_batch(const std::vector<BatchLaunch>& plan, int prec, hipStream_t st);

// geometry helpers (host)
inline int64_t num_params(int64_t n, int L, int r) {
  return 2 * n * r + (int64_t)L * (int64_t(1) << (L + 1)) * r * r;
}

// kernel entry points (defined in the .hip sources)
bfc_status build_layout(Problem* P, const int32_t* d_rows, const int32_t* d_cols,
                        const void* d_vals, hipStream_t st);
bfc_status launch_sweep_core(Problem* P, int core, hipStream_t st);
bfc_status launch_adam_core(Problem* P, int core, int t, double alpha, double beta1,
                            double beta2, double sigma, hipStream_t st);
bfc_status launch_adf_sweep(Problem* P, hipStream_t st);
bfc_status launch_set_values(Problem* P, const void* d_vals, hipStream_t st);
bfc_status enqueue_set_values(Problem* P, const void* d_vals, hipStream_t st);
bfc_status launch_cores_from_f32(Problem* P, const float* src, hipStream_t st);
bfc_status launch_loss_gradient(Problem* P, float scale, void* out, int out_fp64, hipStream_t st);
bfc_status build_items(Problem* P, int core, hipStream_t st);
void plan_items(const Problem* P, int core, int32_t item_size, std::vector<WorkItem>& items,
                std::vector<int32_t>& tile_items);
bfc_status install_items(Problem* P, int core, const std::vector<WorkItem>& items,
                         const std::vector<int32_t>& tile_items, hipStream_t st);
bfc_status dev_free(Problem* P, void* ptr);
bfc_status launch_predict(const Problem* P, int64_t m, const int32_t* rows, const int32_t* cols,
                          void* out, hipStream_t st);
bfc_status launch_residual(const Problem* P, int64_t m, const int32_t* rows, const int32_t* cols,
                           const void* vals, double* out2, hipStream_t st);
bfc_status launch_convert_cores(Problem* P, const void* src_c128, void* dst_c128, bool to_internal,
                                hipStream_t st);
bfc_status launch_random_cores(Problem* P, uint64_t seed, hipStream_t st);
bfc_status launch_residual_observed(Problem* P, double* out2, hipStream_t st);
void invalidate_envs(Problem* P);

}  // namespace bfc
