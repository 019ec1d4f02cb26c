// Layout of an observed set: validation, per-core block keys, stable sort by
// block, block offsets, and (inner cores) the subgroups and work items the
// Gram kernel walks.
//
// Inner core p (the paper's S^(p+1), 1 <= p <= L) has 2^(L+1) slices; slice
// k = ((ib >> (p-1)) << p) | (jb >> (L-p)) owns a contiguous tile of the
// matrix, c 2^(p-1) rows by c 2^(L-p) columns.  Inside a tile the left
// environment of an entry depends on its row only and the right environment
// on its column only, so entries are ordered by (slice, row) when the tile
// has no more rows than columns and by (slice, column) otherwise; runs of
// equal row (column) share one environment.  Runs are cut into subgroups of
// at most kSubgroup entries so that one lane walks one subgroup.
#include <algorithm>
#include <cmath>

#include "bfc_device.h"
#include "bfc_sort.h"

namespace bfc {

namespace {

__global__ void validate_kernel(const int32_t* rows, const int32_t* cols, const double2* vals,
                                int64_t nnz, int64_t n, int32_t* flag) {
  const int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (e >= nnz) return;
  const int32_t i = rows[e], j = cols[e];
  int bad = 0;
  if (i < 0 || i >= n || j < 0 || j >= n) bad |= 1;
  const double2 v = vals[e];
  if (!isfinite(v.x) || !isfinite(v.y)) bad |= 2;
  if (bad) atomicOr(flag, bad);
}

template <typename T>
__global__ void vals_to_compute_kernel(const double2* src, cx<T>* dst, int64_t nnz) {
  const int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (e < nnz) dst[e] = {T(src[e].x), T(src[e].y)};
}

__global__ void core_keys_kernel(const int32_t* rows, const int32_t* cols, int64_t nnz, int c,
                                 int L, int p, uint32_t ext, int byrow, uint32_t* keys,
                                 int32_t* idx) {
  const int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (e >= nnz) return;
  const uint32_t i = (uint32_t)rows[e], j = (uint32_t)cols[e];
  uint32_t key;
  if (p == 0) {
    key = i;
  } else if (p == L + 1) {
    key = j;
  } else {
    const uint32_t tile = slice_key(i / c, j / c, L, p);
    key = tile * ext + (byrow ? i % ext : j % ext);
  }
  keys[e] = key;
  idx[e] = (int32_t)e;
}

template <typename T>
__global__ void gather_entries_kernel(const int32_t* idx, const int32_t* rows, const int32_t* cols,
                                      const cx<T>* vals, int64_t nnz, int32_t* rows_o,
                                      int32_t* cols_o, cx<T>* vals_o) {
  const int64_t k = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (k >= nnz) return;
  const int32_t e = idx[k];
  rows_o[k] = rows[e];
  cols_o[k] = cols[e];
  vals_o[k] = vals[e];
}

__global__ void block_offsets_kernel(const uint32_t* skeys, int64_t nnz, uint32_t ext,
                                     int nblocks, int32_t* blk_off) {
  const int64_t k = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (k >= nnz) return;
  const int64_t tb = skeys[k] / ext;
  const int64_t tp = k ? (int64_t)(skeys[k - 1] / ext) : -1;
  for (int64_t b = tp + 1; b <= tb; ++b) blk_off[b] = (int32_t)k;
  if (k == nnz - 1)
    for (int64_t b = tb + 1; b <= nblocks; ++b) blk_off[b] = (int32_t)nnz;
}

__global__ void run_heads_kernel(const uint32_t* skeys, int64_t nnz, int32_t* head,
                                 int32_t* scan_copy) {
  const int64_t k = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (k >= nnz) return;
  const int32_t h = (k == 0 || skeys[k] != skeys[k - 1]) ? 1 : 0;
  head[k] = h;
  scan_copy[k] = h;
}

// run_scan[k] = number of run heads before k (exclusive scan of head)
__global__ void run_starts_kernel(const int32_t* head, const int32_t* run_scan, int64_t nnz,
                                  int32_t* run_start) {
  const int64_t k = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (k >= nnz) return;
  if (head[k]) run_start[run_scan[k]] = (int32_t)k;
}

__global__ void sub_heads_kernel(const int32_t* head, const int32_t* run_scan,
                                 const int32_t* run_start, int64_t nnz, int32_t* subhead,
                                 int32_t* scan_copy) {
  const int64_t k = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (k >= nnz) return;
  const int32_t rid = run_scan[k] + head[k] - 1;
  const int64_t pos = k - run_start[rid];
  const int32_t h = (pos % kSubgroup) == 0 ? 1 : 0;
  subhead[k] = h;
  scan_copy[k] = h;
}

__global__ void sub_offsets_kernel(const int32_t* subhead, const int32_t* sub_id, int64_t nnz,
                                   int32_t nsub, int32_t* sub_off) {
  const int64_t k = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (k >= nnz) return;
  if (subhead[k]) sub_off[sub_id[k]] = (int32_t)k;
  if (k == nnz - 1) sub_off[nsub] = (int32_t)nnz;
}

// CoreLayout::up_node of an outer core: 2 x the entry's node on the level
// above (ent_up, input order; idx maps sorted to input positions) plus the
// top bit of the other block index (column block for core 0, row block for
// core L+1), which names the slice of the adjacent core.
__global__ void up_node_kernel(const int32_t* idx, const int32_t* ent_up, const int32_t* other,
                               int64_t nnz, int c, int L, int32_t* up) {
  const int64_t k = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (k >= nnz) return;
  up[k] = 2 * ent_up[idx[k]] + (((other[k] / c) >> (L - 1)) & 1);
}

// Subgroup records (CoreLayout::sub_rec): shared_idx names the environment
// node the subgroup's entries share (the left one when grouped by row),
// vary_idx the node of the other environment of every entry.
__global__ void sub_records_kernel(const int32_t* sub_off, int32_t nsub, const int32_t* shared_idx,
                                   const int32_t* vary_idx, int32_t* rec) {
  const int64_t s = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (s >= nsub) return;
  const int32_t e0 = sub_off[s], e1 = sub_off[s + 1];
  int32_t* o = rec + s * kSubRec;
  o[0] = e0;
  o[1] = e1 - e0;
  o[2] = shared_idx[e0];
  o[3] = 0;
#pragma unroll
  for (int q = 0; q < kSubgroup; ++q) o[4 + q] = (e0 + q < e1) ? vary_idx[e0 + q] : -1;
}

__global__ void tile_subs_kernel(const int32_t* blk_off, const int32_t* sub_id, int64_t nnz,
                                 int nb, int32_t nsub, int32_t* tile_sub) {
  const int b = blockIdx.x * blockDim.x + threadIdx.x;
  if (b > nb) return;
  const int32_t k = blk_off[b];
  tile_sub[b] = (k < nnz) ? sub_id[k] : nsub;
}

// Environment-trie levels: right level p keys entries by (ib >> p, j), left
// level p by (jb >> (L-p+1), i); equal keys share one environment vector.
__global__ void level_keys_kernel(const int32_t* rows, const int32_t* cols, int64_t nnz, int c,
                                  int L, int p, int right, uint32_t n, uint32_t* keys,
                                  int32_t* idx) {
  const int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (e >= nnz) return;
  const uint32_t i = (uint32_t)rows[e], j = (uint32_t)cols[e];
  uint32_t key;
  if (right)
    key = ((i / c) >> p) * n + j;
  else
    key = ((j / c) >> (L - p + 1)) * n + i;
  keys[e] = key;
  idx[e] = (int32_t)e;
}

// head/hscan: run heads of the sorted keys and their exclusive scan
__global__ void node_table_kernel(const uint32_t* skeys, const int32_t* idx, const int32_t* head,
                                  const int32_t* hscan, int64_t nnz, uint32_t n, int32_t* node_a,
                                  int32_t* node_b, int32_t* ent_node) {
  const int64_t k = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (k >= nnz) return;
  const int32_t id = hscan[k] + head[k] - 1;
  if (head[k]) {
    node_a[id] = (int32_t)(skeys[k] / n);
    node_b[id] = (int32_t)(skeys[k] % n);
  }
  ent_node[idx[k]] = id;
}

// every entry of a node names the same parent, so concurrent writes agree
__global__ void parent_kernel(const int32_t* ent_child, const int32_t* ent_parent, int64_t nnz,
                              int32_t* parent) {
  const int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (e < nnz) parent[ent_child[e]] = ent_parent[e];
}

__global__ void gather_i32_kernel(const int32_t* idx, const int32_t* src, int64_t nnz,
                                  int32_t* dst) {
  const int64_t k = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (k < nnz) dst[k] = src[idx[k]];
}

inline unsigned grid_for(int64_t n, int t = 256) { return (unsigned)((n + t - 1) / t); }

int bits_for(uint64_t maxval) {
  int b = 0;
  while (b < 64 && (maxval >> b) != 0) ++b;
  return b;
}

struct Scratch {
  std::vector<void*> ptrs;
  ~Scratch() {
    if (!ptrs.empty()) (void)hipDeviceSynchronize();  // after a failure, work may still run
    for (void* p : ptrs) (void)hipFree(p);
  }
  hipError_t get(void** p, size_t bytes) {
    hipError_t e = lib_malloc(p, bytes ? bytes : 16);
    if (e == hipSuccess) ptrs.push_back(*p);
    return e;
  }
};

}  // namespace

// Work items of inner core p: chunks of `item_size` subgroups (automatic
// when 0: at least 128 and enough to keep the item count near 16384), never
// across slices.
void plan_items(const Problem* P, int p, int32_t item_size, std::vector<WorkItem>& items,
                std::vector<int32_t>& tile_items) {
  const CoreLayout& C = P->lay[p];
  int64_t ch = item_size;
  if (P->r > kNarrowRank) {
    ch = INT32_MAX;  // the fused kernels of the wide ranks: one item per slice
  } else if (ch <= 0) {
    const int64_t per_item_target = (int64_t)C.nsub / 16384 + 1;
    ch = std::max<int64_t>(128, ((per_item_target + 63) / 64) * 64);
  }
  items.clear();
  tile_items.assign(C.nblocks + 1, 0);
  const std::vector<int32_t>& hts = C.tile_sub;
  for (int b = 0; b < C.nblocks; ++b) {
    tile_items[b] = (int32_t)items.size();
    for (int64_t s = hts[b]; s < hts[b + 1]; s += ch)
      items.push_back({b, (int32_t)s, (int32_t)std::min<int64_t>(s + ch, hts[b + 1]), 0});
  }
  tile_items[C.nblocks] = (int32_t)items.size();
}

// Copies planned items into core p's arrays (the items array must hold them).
bfc_status install_items(Problem* P, int p, const std::vector<WorkItem>& items,
                         const std::vector<int32_t>& tile_items, hipStream_t st) {
  CoreLayout& C = P->lay[p];
  C.nitems = (int32_t)items.size();
  if (!items.empty())
    BFC_HIP_TRY(hipMemcpyAsync(C.items, items.data(), items.size() * sizeof(WorkItem),
                               hipMemcpyHostToDevice, st));
  BFC_HIP_TRY(hipMemcpyAsync(C.tile_items, tile_items.data(), (C.nblocks + 1) * 4,
                             hipMemcpyHostToDevice, st));
  BFC_HIP_TRY(hipStreamSynchronize(st));
  return BFC_OK;
}

// The items of inner core p at the problem's item size, at layout build.
bfc_status build_items(Problem* P, int p, hipStream_t st) {
  CoreLayout& C = P->lay[p];
  std::vector<WorkItem> items;
  std::vector<int32_t> tile_items;
  plan_items(P, p, P->item_size, items, tile_items);
  if ((int64_t)items.size() > C.items_cap || !C.items) {
    void* fresh = nullptr;
    BFC_TRY(dev_alloc(P, &fresh, std::max<size_t>(1, items.size()) * sizeof(WorkItem)));
    if (C.items) BFC_TRY(dev_free(P, C.items));
    C.items = (WorkItem*)fresh;
    C.items_cap = (int32_t)std::max<size_t>(1, items.size());
  }
  return install_items(P, p, items, tile_items, st);
}

bfc_status build_layout(Problem* P, const int32_t* d_rows, const int32_t* d_cols,
                        const void* d_vals, hipStream_t st) {
  const int64_t nnz = P->nnz;
  const int L = P->L;
  Scratch S;
  int32_t* dflag = nullptr;
  BFC_HIP_TRY(S.get((void**)&dflag, 4));
  BFC_HIP_TRY(hipMemsetAsync(dflag, 0, 4, st));
  validate_kernel<<<grid_for(nnz), 256, 0, st>>>(d_rows, d_cols, (const double2*)d_vals, nnz, P->n,
                                                 dflag);
  BFC_HIP_TRY(hipGetLastError());
  int32_t hflag = 0;
  BFC_HIP_TRY(hipMemcpyAsync(&hflag, dflag, 4, hipMemcpyDeviceToHost, st));
  BFC_HIP_TRY(hipStreamSynchronize(st));
  if (hflag & 1) {
    set_error("bfc_init_cores: an index is outside [0, n)");
    return BFC_EINVAL;
  }
  if (hflag & 2) {
    set_error("bfc_init_cores: a value is NaN or Inf");
    return BFC_ENONFINITE;
  }

  // values in the compute precision, input order
  void* vals_c = nullptr;
  BFC_HIP_TRY(S.get(&vals_c, nnz * P->elem));
  if (P->prec == BFC_C128)
    vals_to_compute_kernel<double><<<grid_for(nnz), 256, 0, st>>>((const double2*)d_vals,
                                                                   (cx<double>*)vals_c, nnz);
  else
    vals_to_compute_kernel<float><<<grid_for(nnz), 256, 0, st>>>((const double2*)d_vals,
                                                                 (cx<float>*)vals_c, nnz);
  BFC_HIP_TRY(hipGetLastError());

  uint32_t* keys = nullptr;
  int32_t* idx = nullptr;
  void* rscr = nullptr;
  int32_t *head = nullptr, *tmp = nullptr, *tmp2 = nullptr, *run_start = nullptr,
          *scan_scr = nullptr;
  BFC_HIP_TRY(S.get((void**)&keys, nnz * 4));
  BFC_HIP_TRY(S.get((void**)&idx, nnz * 4));
  BFC_HIP_TRY(S.get(&rscr, radix_scratch_bytes(nnz)));
  BFC_HIP_TRY(S.get((void**)&head, nnz * 4));
  BFC_HIP_TRY(S.get((void**)&tmp, nnz * 4));
  BFC_HIP_TRY(S.get((void**)&tmp2, nnz * 4));
  BFC_HIP_TRY(S.get((void**)&run_start, nnz * 4));
  BFC_HIP_TRY(S.get((void**)&scan_scr, scan_scratch_elems(nnz) * 4));

  const int64_t n = P->n;
  const int c = P->c;
  if (((uint64_t)n << L) > 0xFFFFFFFFull) {
    set_error("bfc_init_cores: n * 2^L must stay below 2^32");
    return BFC_EINVAL;
  }

  // environment-trie levels: per-entry node ids (input order), node tables
  std::vector<int32_t*> ent_r(L + 2, nullptr), ent_l(L + 2, nullptr);
  P->rlev.assign(L, EnvLevel());
  P->llev.assign(L + 2, EnvLevel());
  auto build_level = [&](int p, bool right, EnvLevel& E, int32_t*& ent) -> bfc_status {
    BFC_HIP_TRY(S.get((void**)&ent, nnz * 4));
    const uint64_t span = right ? ((uint64_t)1 << (L - p)) : ((uint64_t)1 << (p - 1));
    level_keys_kernel<<<grid_for(nnz), 256, 0, st>>>(d_rows, d_cols, nnz, c, L, p, right ? 1 : 0,
                                                     (uint32_t)n, keys, idx);
    BFC_HIP_TRY(hipGetLastError());
    BFC_HIP_TRY(radix_sort_pairs(keys, idx, nnz, bits_for(span * n - 1), rscr, st));
    run_heads_kernel<<<grid_for(nnz), 256, 0, st>>>(keys, nnz, head, tmp);
    BFC_HIP_TRY(exclusive_scan_i32(tmp, nnz, scan_scr, st));
    int32_t last[2];
    BFC_HIP_TRY(hipMemcpyAsync(&last[0], tmp + nnz - 1, 4, hipMemcpyDeviceToHost, st));
    BFC_HIP_TRY(hipMemcpyAsync(&last[1], head + nnz - 1, 4, hipMemcpyDeviceToHost, st));
    BFC_HIP_TRY(hipStreamSynchronize(st));
    E.count = last[0] + last[1];
    BFC_TRY(dev_alloc(P, (void**)&E.node_a, (size_t)E.count * 4));
    BFC_TRY(dev_alloc(P, (void**)&E.node_b, (size_t)E.count * 4));
    BFC_TRY(dev_alloc(P, (void**)&E.parent, (size_t)E.count * 4));
    BFC_TRY(dev_alloc(P, &E.vec, (size_t)E.count * P->r * P->elem));
    P->env_bytes += (int64_t)E.count * (12 + P->r * (int64_t)P->elem);
    node_table_kernel<<<grid_for(nnz), 256, 0, st>>>(keys, idx, head, tmp, nnz, (uint32_t)n,
                                                     E.node_a, E.node_b, ent);
    BFC_HIP_TRY(hipGetLastError());
    return BFC_OK;
  };
  for (int p = L - 1; p >= 0; --p) BFC_TRY(build_level(p, true, P->rlev[p], ent_r[p]));
  for (int p = 2; p <= L + 1; ++p) BFC_TRY(build_level(p, false, P->llev[p], ent_l[p]));
  // parents: right level p -> right level p+1 (level L-1 points at the column
  // j itself); left level p -> left level p-1 (level 2 points at the row i)
  for (int p = 0; p + 1 <= L - 1; ++p)
    parent_kernel<<<grid_for(nnz), 256, 0, st>>>(ent_r[p], ent_r[p + 1], nnz, P->rlev[p].parent);
  if (L >= 1)
    BFC_HIP_TRY(hipMemcpyAsync(P->rlev[L - 1].parent, P->rlev[L - 1].node_b,
                               (size_t)P->rlev[L - 1].count * 4, hipMemcpyDeviceToDevice, st));
  for (int p = 3; p <= L + 1; ++p)
    parent_kernel<<<grid_for(nnz), 256, 0, st>>>(ent_l[p], ent_l[p - 1], nnz, P->llev[p].parent);
  if (L >= 1)
    BFC_HIP_TRY(hipMemcpyAsync(P->llev[2].parent, P->llev[2].node_b,
                               (size_t)P->llev[2].count * 4, hipMemcpyDeviceToDevice, st));
  BFC_HIP_TRY(hipGetLastError());

  P->lay.assign(L + 2, CoreLayout());
  int32_t max_items = 0;
  for (int p = 0; p <= L + 1; ++p) {
    CoreLayout& C = P->lay[p];
    const bool inner = (p >= 1 && p <= L);
    C.nblocks = inner ? (1 << (L + 1)) : (int32_t)n;
    uint32_t ext = 1;
    if (inner) {
      const int64_t R_rows = (int64_t)c << (p - 1);
      const int64_t C_cols = (int64_t)c << (L - p);
      C.group_by_row = R_rows <= C_cols ? 1 : 0;
      ext = (uint32_t)std::min(R_rows, C_cols);
      C.group_extent = (int32_t)ext;
      if ((uint64_t)C.nblocks * ext > 0xFFFFFFFFull) {
        set_error("bfc_init_cores: sizes too large for 32-bit sort keys");
        return BFC_EINVAL;
      }
    }
    const uint64_t maxkey = inner ? (uint64_t)C.nblocks * ext - 1 : (uint64_t)(n - 1);
    core_keys_kernel<<<grid_for(nnz), 256, 0, st>>>(d_rows, d_cols, nnz, c, L, p, ext,
                                                    C.group_by_row, keys, idx);
    BFC_HIP_TRY(hipGetLastError());
    BFC_HIP_TRY(radix_sort_pairs(keys, idx, nnz, bits_for(maxkey), rscr, st));
    BFC_TRY(dev_alloc(P, (void**)&C.rows, nnz * 4));
    BFC_TRY(dev_alloc(P, (void**)&C.cols, nnz * 4));
    BFC_TRY(dev_alloc(P, &C.vals, nnz * P->elem));
    BFC_TRY(dev_alloc(P, (void**)&C.blk_off, (C.nblocks + 1) * 4));
    if (P->prec == BFC_C128)
      gather_entries_kernel<double><<<grid_for(nnz), 256, 0, st>>>(
          idx, d_rows, d_cols, (const cx<double>*)vals_c, nnz, C.rows, C.cols,
          (cx<double>*)C.vals);
    else
      gather_entries_kernel<float><<<grid_for(nnz), 256, 0, st>>>(
          idx, d_rows, d_cols, (const cx<float>*)vals_c, nnz, C.rows, C.cols,
          (cx<float>*)C.vals);
    BFC_HIP_TRY(hipGetLastError());
    BFC_TRY(dev_alloc(P, (void**)&C.perm, nnz * 4));
    BFC_HIP_TRY(hipMemcpyAsync(C.perm, idx, nnz * 4, hipMemcpyDeviceToDevice, st));
    block_offsets_kernel<<<grid_for(nnz), 256, 0, st>>>(keys, nnz, ext, C.nblocks, C.blk_off);
    BFC_HIP_TRY(hipGetLastError());
    // environment nodes of the sorted entries: right level p (p < L) and
    // left level p (p >= 2)
    if (p <= L - 1) {
      BFC_TRY(dev_alloc(P, (void**)&C.rnode, nnz * 4));
      gather_i32_kernel<<<grid_for(nnz), 256, 0, st>>>(idx, ent_r[p], nnz, C.rnode);
    }
    if (p >= 2) {
      BFC_TRY(dev_alloc(P, (void**)&C.lnode, nnz * 4));
      gather_i32_kernel<<<grid_for(nnz), 256, 0, st>>>(idx, ent_l[p], nnz, C.lnode);
    }
    if ((p == 0 || p == L + 1) && L >= 2 && P->r <= kNarrowRank) {
      BFC_TRY(dev_alloc(P, (void**)&C.up_node, nnz * 4));
      up_node_kernel<<<grid_for(nnz), 256, 0, st>>>(idx, p == 0 ? ent_r[1] : ent_l[L],
                                                    p == 0 ? C.cols : C.rows, nnz, c, L,
                                                    C.up_node);
    }
    BFC_HIP_TRY(hipGetLastError());
    if (!inner) continue;

    // subgroups: runs of equal (slice, row|column), cut every kSubgroup entries
    run_heads_kernel<<<grid_for(nnz), 256, 0, st>>>(keys, nnz, head, tmp);
    BFC_HIP_TRY(exclusive_scan_i32(tmp, nnz, scan_scr, st));
    run_starts_kernel<<<grid_for(nnz), 256, 0, st>>>(head, tmp, nnz, run_start);
    sub_heads_kernel<<<grid_for(nnz), 256, 0, st>>>(head, tmp, run_start, nnz, idx, tmp2);
    BFC_HIP_TRY(exclusive_scan_i32(tmp2, nnz, scan_scr, st));
    int32_t last[4];
    BFC_HIP_TRY(hipMemcpyAsync(&last[0], tmp2 + nnz - 1, 4, hipMemcpyDeviceToHost, st));
    BFC_HIP_TRY(hipMemcpyAsync(&last[1], idx + nnz - 1, 4, hipMemcpyDeviceToHost, st));
    BFC_HIP_TRY(hipMemcpyAsync(&last[2], tmp + nnz - 1, 4, hipMemcpyDeviceToHost, st));
    BFC_HIP_TRY(hipMemcpyAsync(&last[3], head + nnz - 1, 4, hipMemcpyDeviceToHost, st));
    BFC_HIP_TRY(hipStreamSynchronize(st));
    C.nsub = last[0] + last[1];
    C.nruns = last[2] + last[3];
    BFC_TRY(dev_alloc(P, (void**)&C.sub_off, ((int64_t)C.nsub + 1) * 4));
    sub_offsets_kernel<<<grid_for(nnz), 256, 0, st>>>(idx, tmp2, nnz, C.nsub, C.sub_off);
    if (P->r <= kNarrowRank && P->prec != BFC_C64_BF16GRAM) {
      // the environment indices the Gram reads: a row of Z^1 at p = 1, a
      // column of Z^(L+2) at p = L, cached trie nodes otherwise
      const int32_t* lidx = (p == 1) ? C.rows : C.lnode;
      const int32_t* ridx = (p == L) ? C.cols : C.rnode;
      BFC_TRY(dev_alloc(P, (void**)&C.sub_rec, (int64_t)C.nsub * kSubRec * 4));
      sub_records_kernel<<<grid_for(C.nsub), 256, 0, st>>>(
          C.sub_off, C.nsub, C.group_by_row ? lidx : ridx, C.group_by_row ? ridx : lidx, C.sub_rec);
    }
    int32_t* tile_sub = head;  // reuse: nblocks + 1 <= nnz is not guaranteed, size check
    if ((int64_t)C.nblocks + 1 > nnz) BFC_HIP_TRY(S.get((void**)&tile_sub, (C.nblocks + 1) * 4));
    tile_subs_kernel<<<grid_for(C.nblocks + 1), 256, 0, st>>>(C.blk_off, tmp2, nnz, C.nblocks,
                                                              C.nsub, tile_sub);
    BFC_HIP_TRY(hipGetLastError());
    C.tile_sub.assign(C.nblocks + 1, 0);
    BFC_HIP_TRY(hipMemcpyAsync(C.tile_sub.data(), tile_sub, (C.nblocks + 1) * 4,
                               hipMemcpyDeviceToHost, st));
    BFC_HIP_TRY(hipStreamSynchronize(st));
    BFC_TRY(dev_alloc(P, (void**)&C.tile_items, (C.nblocks + 1) * 4));
    BFC_TRY(build_items(P, p, st));
    max_items = std::max(max_items, C.nitems);
  }
  P->max_items = max_items;
  BFC_HIP_TRY(hipStreamSynchronize(st));
  return BFC_OK;
}

}  // namespace bfc
