// Host-side checks of a problem's layout (the debug checks of the library):
// every invariant the kernels rely on when they index the sorted entries,
// the block offsets, the inner-slice subgroups and work items, and the
// environment trie, recomputed on the host from the entries themselves.
// Nothing here launches a kernel: the device arrays are copied to the host.
#include <algorithm>
#include <cstring>
#include <string>
#include <vector>

#include "bfc_device.h"

struct bfc_problem : public bfc::Problem {};

namespace bfc {
namespace {

template <typename T>
bfc_status fetch(std::vector<T>& out, const void* src, int64_t count) {
  out.resize((size_t)std::max<int64_t>(count, 0));
  if (count > 0)
    BFC_HIP_TRY(hipMemcpy(out.data(), src, sizeof(T) * (size_t)count, hipMemcpyDeviceToHost));
  return BFC_OK;
}

bfc_status bad(const std::string& what) {
  set_error("bfc_validate: " + what);
  return BFC_EINVAL;
}

std::string at(int p, int64_t e) { return " (core " + std::to_string(p) + ", position " +
                                          std::to_string(e) + ")"; }

// Right level p: node (ib >> p, j); left level p: node (jb >> (L-p+1), i).
bfc_status check_level(const Problem* P, const EnvLevel& E, int p, bool right,
                       const EnvLevel* above, std::vector<int32_t>& a, std::vector<int32_t>& b) {
  BFC_TRY(fetch(a, E.node_a, E.count));
  BFC_TRY(fetch(b, E.node_b, E.count));
  std::vector<int32_t> par;
  BFC_TRY(fetch(par, E.parent, E.count));
  const std::string lv = std::string(right ? "right" : "left") + " level " + std::to_string(p);
  for (int64_t k = 0; k < E.count; ++k) {
    if (b[k] < 0 || b[k] >= P->n) return bad(lv + ": node index outside [0, n)");
    if (k > 0 && !(a[k - 1] < a[k] || (a[k - 1] == a[k] && b[k - 1] < b[k])))
      return bad(lv + ": nodes not strictly increasing");
    const bool top = right ? p == P->L - 1 : p == 2;
    if (top) {
      if (par[k] != b[k]) return bad(lv + ": parent of a top node is not its row/column");
    } else {
      if (par[k] < 0 || par[k] >= above->count) return bad(lv + ": parent out of range");
    }
  }
  return BFC_OK;
}

}  // namespace
}  // namespace bfc

using namespace bfc;

extern "C" {

bfc_status bfc_validate(const bfc_problem* p) {
  if (!p) {
    set_error("bfc_validate: null problem");
    return BFC_EINVAL;
  }
  const Problem* P = p;
  const int L = P->L;
  const int64_t nnz = P->nnz, n = P->n, c = P->c;
  BFC_HIP_TRY(hipDeviceSynchronize());
  // the trie: node tables, order, parents (ids checked against the parents below)
  std::vector<std::vector<int32_t>> ra(L), rb(L), la(L + 2), lb(L + 2);
  for (int q = L - 1; q >= 0; --q)
    BFC_TRY(check_level(P, P->rlev[q], q, true, q + 1 < L ? &P->rlev[q + 1] : nullptr, ra[q],
                        rb[q]));
  for (int q = 2; q <= L + 1; ++q)
    BFC_TRY(check_level(P, P->llev[q], q, false, q > 2 ? &P->llev[q - 1] : nullptr, la[q],
                        lb[q]));
  for (int q = 0; q + 1 < L; ++q) {  // right parent: (u >> 1, j) on level q+1
    std::vector<int32_t> par;
    BFC_TRY(fetch(par, P->rlev[q].parent, P->rlev[q].count));
    for (int64_t k = 0; k < P->rlev[q].count; ++k)
      if (ra[q + 1][par[k]] != (ra[q][k] >> 1) || rb[q + 1][par[k]] != rb[q][k])
        return bad("right level " + std::to_string(q) + ": wrong parent");
  }
  for (int q = 3; q <= L + 1; ++q) {  // left parent: (w >> 1, i) on level q-1
    std::vector<int32_t> par;
    BFC_TRY(fetch(par, P->llev[q].parent, P->llev[q].count));
    for (int64_t k = 0; k < P->llev[q].count; ++k)
      if (la[q - 1][par[k]] != (la[q][k] >> 1) || lb[q - 1][par[k]] != lb[q][k])
        return bad("left level " + std::to_string(q) + ": wrong parent");
  }
  // per core: sorted entries, keys, offsets, subgroups, items, node ids
  std::vector<int32_t> rows0, cols0, inv0;
  std::vector<unsigned char> vals0;
  for (int q = 0; q <= L + 1; ++q) {
    const CoreLayout& C = P->lay[q];
    const bool inner = q >= 1 && q <= L;
    std::vector<int32_t> rows, cols, perm, off;
    std::vector<unsigned char> vals;
    BFC_TRY(fetch(rows, C.rows, nnz));
    BFC_TRY(fetch(cols, C.cols, nnz));
    BFC_TRY(fetch(perm, C.perm, nnz));
    BFC_TRY(fetch(vals, C.vals, nnz * (int64_t)P->elem));
    BFC_TRY(fetch(off, C.blk_off, (int64_t)C.nblocks + 1));
    if (C.nblocks != (inner ? (1 << (L + 1)) : n)) return bad("wrong block count" + at(q, 0));
    if (off[0] != 0 || off[C.nblocks] != nnz) return bad("block offsets do not span the entries" + at(q, 0));
    std::vector<char> seen(nnz, 0);
    for (int64_t e = 0; e < nnz; ++e) {
      if (perm[e] < 0 || perm[e] >= nnz || seen[perm[e]]) return bad("not a permutation" + at(q, e));
      seen[perm[e]] = 1;
      if (rows[e] < 0 || rows[e] >= n || cols[e] < 0 || cols[e] >= n)
        return bad("index outside [0, n)" + at(q, e));
    }
    if (q == 0) {
      rows0 = rows;
      cols0 = cols;
      vals0 = vals;
      inv0.assign(nnz, 0);
      for (int64_t e = 0; e < nnz; ++e) inv0[perm[e]] = (int32_t)e;
    } else {
      for (int64_t e = 0; e < nnz; ++e) {
        const int64_t e0 = inv0[perm[e]];
        if (rows[e] != rows0[e0] || cols[e] != cols0[e0] ||
            std::memcmp(&vals[e * P->elem], &vals0[e0 * P->elem], P->elem) != 0)
          return bad("entry differs from the same input entry in core 0" + at(q, e));
      }
    }
    for (int64_t b = 0; b < C.nblocks; ++b) {
      if (off[b] > off[b + 1]) return bad("block offsets decrease" + at(q, off[b]));
      for (int64_t e = off[b]; e < off[b + 1]; ++e) {
        const uint32_t ib = (uint32_t)(rows[e] / c), jb = (uint32_t)(cols[e] / c);
        const int64_t key = q == 0 ? rows[e] : q == L + 1 ? cols[e] : slice_key(ib, jb, L, q);
        if (key != b) return bad("entry in the wrong block" + at(q, e));
        if (inner && e > off[b]) {
          const int32_t prev = C.group_by_row ? rows[e - 1] : cols[e - 1];
          const int32_t cur = C.group_by_row ? rows[e] : cols[e];
          if (prev > cur) return bad("slice not sorted by its grouping index" + at(q, e));
        }
      }
    }
    // environment node of every entry: right level q (q < L), left level q (q >= 2)
    if (q <= L - 1) {
      std::vector<int32_t> nd;
      BFC_TRY(fetch(nd, C.rnode, nnz));
      for (int64_t e = 0; e < nnz; ++e) {
        const int32_t k = nd[e];
        if (k < 0 || k >= P->rlev[q].count) return bad("right node out of range" + at(q, e));
        if (ra[q][k] != (int32_t)((rows[e] / c) >> q) || rb[q][k] != cols[e])
          return bad("entry points at the wrong right node" + at(q, e));
      }
    }
    if (q >= 2) {
      std::vector<int32_t> nd;
      BFC_TRY(fetch(nd, C.lnode, nnz));
      for (int64_t e = 0; e < nnz; ++e) {
        const int32_t k = nd[e];
        if (k < 0 || k >= P->llev[q].count) return bad("left node out of range" + at(q, e));
        if (la[q][k] != (int32_t)((cols[e] / c) >> (L - q + 1)) || lb[q][k] != rows[e])
          return bad("entry points at the wrong left node" + at(q, e));
      }
    }
    // outer cores: each entry's node on the level above the outermost one,
    // and the half bit that picks the slice of the adjacent core
    if (C.up_node) {
      if (inner || L < 2) return bad("level-above nodes on a core without them" + at(q, 0));
      std::vector<int32_t> up;
      BFC_TRY(fetch(up, C.up_node, nnz));
      for (int64_t e = 0; e < nnz; ++e) {
        const int32_t k = up[e] >> 1, half = up[e] & 1;
        if (q == 0) {
          if (k < 0 || k >= P->rlev[1].count) return bad("level-above node out of range" + at(q, e));
          if (ra[1][k] != (int32_t)((rows[e] / c) >> 1) || rb[1][k] != cols[e])
            return bad("entry points at the wrong level-above node" + at(q, e));
          if (half != (int32_t)(((cols[e] / c) >> (L - 1)) & 1))
            return bad("level-above half bit" + at(q, e));
        } else {
          if (k < 0 || k >= P->llev[L].count) return bad("level-above node out of range" + at(q, e));
          if (la[L][k] != (int32_t)((cols[e] / c) >> 1) || lb[L][k] != rows[e])
            return bad("entry points at the wrong level-above node" + at(q, e));
          if (half != (int32_t)(((rows[e] / c) >> (L - 1)) & 1))
            return bad("level-above half bit" + at(q, e));
        }
      }
    } else if ((q == 0 || q == L + 1) && L >= 2 && P->r <= kNarrowRank) {
      return bad("level-above nodes missing" + at(q, 0));
    }
    if (!inner) continue;
    // subgroups: at most kSubgroup entries of one slice sharing the row (or column)
    std::vector<int32_t> so, ti;
    std::vector<WorkItem> items;
    BFC_TRY(fetch(so, C.sub_off, (int64_t)C.nsub + 1));
    BFC_TRY(fetch(ti, C.tile_items, (int64_t)C.nblocks + 1));
    BFC_TRY(fetch(items, C.items, C.nitems));
    if (so[0] != 0 || so[C.nsub] != nnz) return bad("subgroups do not span the entries" + at(q, 0));
    int64_t b = 0;
    for (int64_t s = 0; s < C.nsub; ++s) {
      const int64_t e0 = so[s], e1 = so[s + 1];
      if (e1 <= e0 || e1 - e0 > kSubgroup) return bad("subgroup size outside [1, 8]" + at(q, e0));
      while (b < C.nblocks && off[b + 1] <= e0) ++b;
      if (e1 > off[b + 1]) return bad("subgroup crosses slices" + at(q, e0));
      for (int64_t e = e0 + 1; e < e1; ++e)
        if ((C.group_by_row ? rows[e] != rows[e0] : cols[e] != cols[e0]))
          return bad("subgroup mixes rows (or columns)" + at(q, e));
      if (C.tile_sub[b] > s || C.tile_sub[b + 1] <= s) return bad("slice subgroup range" + at(q, e0));
    }
    // subgroup records of the narrow-rank FP32 / FP64 Gram: offsets and
    // environment indices as the per-entry arrays give them
    if (C.sub_rec) {
      std::vector<int32_t> rec, ln, rn;
      BFC_TRY(fetch(rec, C.sub_rec, (int64_t)C.nsub * kSubRec));
      if (q >= 2) BFC_TRY(fetch(ln, C.lnode, nnz));
      if (q <= L - 1) BFC_TRY(fetch(rn, C.rnode, nnz));
      // the index the Gram reads: a row of Z^1 at q = 1, a column of
      // Z^(L+2) at q = L, a trie node otherwise
      auto lsrc = [&](int64_t e) { return q == 1 ? rows[e] : ln[e]; };
      auto rsrc = [&](int64_t e) { return q == L ? cols[e] : rn[e]; };
      for (int64_t s = 0; s < C.nsub; ++s) {
        const int32_t* o = rec.data() + s * kSubRec;
        const int64_t e0 = so[s], e1 = so[s + 1];
        if (o[0] != e0 || o[1] != e1 - e0) return bad("subgroup record offsets" + at(q, e0));
        if (o[2] != (C.group_by_row ? lsrc(e0) : rsrc(e0)))
          return bad("subgroup record shared node" + at(q, e0));
        for (int k = 0; k < kSubgroup; ++k) {
          const int64_t e = e0 + k;
          const int32_t want = e < e1 ? (C.group_by_row ? rsrc(e) : lsrc(e)) : -1;
          if (o[4 + k] != want) return bad("subgroup record entry node" + at(q, e0));
        }
      }
    } else if (P->r <= kNarrowRank && P->prec != BFC_C64_BF16GRAM) {
      return bad("subgroup records missing" + at(q, 0));
    }
    if (ti[0] != 0 || ti[C.nblocks] != C.nitems) return bad("items do not span the slices" + at(q, 0));
    for (int64_t t = 0; t < C.nblocks; ++t) {
      int64_t next = C.tile_sub[t];
      for (int64_t it = ti[t]; it < ti[t + 1]; ++it) {
        if (items[it].tile != t || items[it].sub0 != next || items[it].sub1 <= items[it].sub0)
          return bad("work items do not tile the slice's subgroups" + at(q, it));
        next = items[it].sub1;
      }
      if (next != C.tile_sub[t + 1]) return bad("work items miss subgroups" + at(q, t));
    }
  }
  return BFC_OK;
}

int64_t bfc_debug_fail_allocation_after(int64_t count) {
  return debug_fail_allocation_after(count);
}

}  // extern "C"
