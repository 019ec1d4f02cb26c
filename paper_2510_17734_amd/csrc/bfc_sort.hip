// Device prefix sums and a stable LSD radix sort of (uint32 key, int32 value)
// pairs, used once per observed set to order the entries of every core by
// block.  Stability makes the order (and so every later floating-point sum)
// independent of scheduling.
#include "bfc_sort.h"

namespace bfc {

namespace {

constexpr int kScanThreads = 256;
constexpr int kScanItems = 16;
constexpr int kScanTile = kScanThreads * kScanItems;  // 4096

// Exclusive scan of each 4096-element tile in place; tile totals to sums.
__global__ __launch_bounds__(kScanThreads) void scan_tiles_kernel(int32_t* data, int64_t len,
                                                                  int32_t* sums) {
  __shared__ int32_t part[kScanThreads];
  const int64_t base = (int64_t)blockIdx.x * kScanTile + (int64_t)threadIdx.x * kScanItems;
  int32_t v[kScanItems];
  int32_t run = 0;
#pragma unroll
  for (int k = 0; k < kScanItems; ++k) {
    const int64_t idx = base + k;
    v[k] = idx < len ? data[idx] : 0;
    run += v[k];
  }
  part[threadIdx.x] = run;
  __syncthreads();
  // Hillis-Steele inclusive scan over the thread totals
  for (int off = 1; off < kScanThreads; off <<= 1) {
    int32_t add = threadIdx.x >= off ? part[threadIdx.x - off] : 0;
    __syncthreads();
    part[threadIdx.x] += add;
    __syncthreads();
  }
  int32_t pre = threadIdx.x ? part[threadIdx.x - 1] : 0;
#pragma unroll
  for (int k = 0; k < kScanItems; ++k) {
    const int64_t idx = base + k;
    if (idx < len) data[idx] = pre;
    pre += v[k];
  }
  if (sums && threadIdx.x == kScanThreads - 1) sums[blockIdx.x] = part[kScanThreads - 1];
}

__global__ void scan_add_kernel(int32_t* data, int64_t len, const int32_t* offs) {
  const int64_t idx = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (idx < len) data[idx] += offs[idx / kScanTile];
}

constexpr int kSortThreads = 256;
constexpr int kSortRounds = 16;
constexpr int kSortTile = kSortThreads * kSortRounds;  // 4096 elements per block
constexpr int kWaves = kSortThreads / 64;

__global__ __launch_bounds__(kSortThreads) void radix_hist_kernel(const uint32_t* keys, int64_t n,
                                                                   int shift, int32_t* hist,
                                                                   int nblk) {
  __shared__ int32_t cnt[256];
  cnt[threadIdx.x] = 0;
  __syncthreads();
  const int64_t base = (int64_t)blockIdx.x * kSortTile;
  for (int k = 0; k < kSortRounds; ++k) {
    const int64_t idx = base + (int64_t)k * kSortThreads + threadIdx.x;
    if (idx < n) atomicAdd(&cnt[(keys[idx] >> shift) & 255u], 1);
  }
  __syncthreads();
  hist[(int64_t)threadIdx.x * nblk + blockIdx.x] = cnt[threadIdx.x];
}

// Stable scatter: inside a block, elements keep their (round, thread) order.
__global__ __launch_bounds__(kSortThreads) void radix_scatter_kernel(
    const uint32_t* keys_in, const int32_t* vals_in, uint32_t* keys_out, int32_t* vals_out,
    int64_t n, int shift, const int32_t* offs, int nblk) {
  __shared__ int32_t wcnt[kWaves][256];
  __shared__ int32_t run[256];
  const int tid = threadIdx.x;
  const int lane = tid & 63;
  const int wave = tid >> 6;
  run[tid] = offs[(int64_t)tid * nblk + blockIdx.x];
  for (int w = 0; w < kWaves; ++w) wcnt[w][tid] = 0;
  __syncthreads();
  const uint64_t lt = (lane == 0) ? 0ull : (~0ull >> (64 - lane));
  const int64_t base = (int64_t)blockIdx.x * kSortTile;
  for (int k = 0; k < kSortRounds; ++k) {
    const int64_t idx = base + (int64_t)k * kSortThreads + tid;
    const bool valid = idx < n;
    uint32_t key = 0;
    int32_t val = 0;
    if (valid) {
      key = keys_in[idx];
      val = vals_in[idx];
    }
    const uint32_t dg = (key >> shift) & 255u;
    uint64_t peers = __ballot(valid);
#pragma unroll
    for (int b = 0; b < 8; ++b) {
      const bool bit = (dg >> b) & 1u;
      const uint64_t m = __ballot(valid && bit);
      peers &= bit ? m : ~m;
    }
    const int wrank = __popcll(peers & lt);
    if (valid && wrank == 0) wcnt[wave][dg] = __popcll(peers);
    __syncthreads();
    if (valid) {
      int32_t pos = run[dg] + wrank;
      for (int w = 0; w < wave; ++w) pos += wcnt[w][dg];
      keys_out[pos] = key;
      vals_out[pos] = val;
    }
    __syncthreads();
    int32_t tot = 0;
    for (int w = 0; w < kWaves; ++w) {
      tot += wcnt[w][tid];
      wcnt[w][tid] = 0;
    }
    run[tid] += tot;
    __syncthreads();
  }
}

}  // namespace

// Exclusive prefix sum of data[0..len) in place.  scratch must hold
// scan_scratch_elems(len) int32 values.
hipError_t exclusive_scan_i32(int32_t* data, int64_t len, int32_t* scratch, hipStream_t st) {
  if (len <= 0) return hipSuccess;
  const int64_t tiles = (len + kScanTile - 1) / kScanTile;
  if (tiles == 1) {
    scan_tiles_kernel<<<1, kScanThreads, 0, st>>>(data, len, nullptr);
    return hipGetLastError();
  }
  int32_t* sums = scratch;
  scan_tiles_kernel<<<(unsigned)tiles, kScanThreads, 0, st>>>(data, len, sums);
  hipError_t e = hipGetLastError();
  if (e != hipSuccess) return e;
  e = exclusive_scan_i32(sums, tiles, scratch + tiles, st);
  if (e != hipSuccess) return e;
  scan_add_kernel<<<(unsigned)((len + 255) / 256), 256, 0, st>>>(data, len, sums);
  return hipGetLastError();
}

int64_t scan_scratch_elems(int64_t len) {
  int64_t total = 0;
  while (len > kScanTile) {
    len = (len + kScanTile - 1) / kScanTile;
    total += len;
  }
  return total + 1;
}

int64_t radix_scratch_bytes(int64_t n) {
  const int64_t nblk = (n + kSortTile - 1) / kSortTile;
  const int64_t hist = 256 * nblk;
  return (2 * n + 2 * n + hist + scan_scratch_elems(hist)) * 4 + 1024;
}

// Stable sort of (keys, vals) by the low `bits` bits of keys.  Results end up
// in keys/vals; scratch holds radix_scratch_bytes(n) bytes.
hipError_t radix_sort_pairs(uint32_t* keys, int32_t* vals, int64_t n, int bits, void* scratch,
                            hipStream_t st) {
  if (n <= 1 || bits <= 0) return hipSuccess;
  const int64_t nblk = (n + kSortTile - 1) / kSortTile;
  uint8_t* s = (uint8_t*)scratch;
  uint32_t* k2 = (uint32_t*)s;
  int32_t* v2 = (int32_t*)(s + n * 4);
  int32_t* hist = (int32_t*)(s + n * 8);
  int32_t* scan_scr = hist + 256 * nblk;
  uint32_t* ka = keys;
  int32_t* va = vals;
  uint32_t* kb = k2;
  int32_t* vb = v2;
  const int passes = (bits + 7) / 8;
  hipError_t e;
  for (int pass = 0; pass < passes; ++pass) {
    const int shift = pass * 8;
    radix_hist_kernel<<<(unsigned)nblk, kSortThreads, 0, st>>>(ka, n, shift, hist, (int)nblk);
    if ((e = hipGetLastError()) != hipSuccess) return e;
    if ((e = exclusive_scan_i32(hist, 256 * nblk, scan_scr, st)) != hipSuccess) return e;
    radix_scatter_kernel<<<(unsigned)nblk, kSortThreads, 0, st>>>(ka, va, kb, vb, n, shift, hist,
                                                                   (int)nblk);
    if ((e = hipGetLastError()) != hipSuccess) return e;
    uint32_t* tk = ka; ka = kb; kb = tk;
    int32_t* tv = va; va = vb; vb = tv;
  }
  if (ka != keys) {
    if ((e = hipMemcpyAsync(keys, ka, n * 4, hipMemcpyDeviceToDevice, st)) != hipSuccess) return e;
    if ((e = hipMemcpyAsync(vals, va, n * 4, hipMemcpyDeviceToDevice, st)) != hipSuccess) return e;
  }
  return hipSuccess;
}

}  // namespace bfc
