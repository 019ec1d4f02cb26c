// Kernels of the ALS core updates at ranks kNarrowRank+1 .. BFC_MAX_RANK
// (fused per-slice inner update, one-wavefront outer update).
#pragma once

#include "bfc_common.h"

namespace bfc {

// Outer core (Z^1 or Z^(L+2)) update: fiber b's entries are
// blk_off[b] .. blk_off[b+1] of the core's order, env[env_idx[e]] is entry e's
// r-vector environment and vals[e] its value.
template <typename T>
struct WideOuterArgs {
  cx<T>* fibers;
  const cx<T>* env;
  const int32_t* env_idx;
  const cx<T>* vals;
  const int32_t* blk_off;
  int nblocks;
  double reg_rel;
  double reg_floor;
  int prox;
  int32_t* flags;  // [0] solve failures, [1] ladder retries
};

// Inner core update: slice k's subgroups are those of its work items
// (tile_items[k] .. tile_items[k+1]); region holds wide_region_bytes(r)
// bytes per work item.
template <typename T>
struct WideArgs {
  cx<T>* slices;
  const cx<T>* lenv;
  const int32_t* lidx;
  const cx<T>* renv;
  const int32_t* ridx;
  const cx<T>* vals;
  const int32_t* sub_off;
  const WorkItem* items;
  const int32_t* tile_items;
  unsigned char* region;
  double reg_rel;
  double reg_floor;
  int prox;
  int32_t* flags;
};

template <typename T, int R>
bfc_status launch_outer_wide(const WideOuterArgs<T>& a, hipStream_t st);
template <typename T, int R>
bfc_status launch_inner_wide(const WideArgs<T>& a, int nslices, int by_row, hipStream_t st);
size_t wide_region_bytes(int r);

}  // namespace bfc
