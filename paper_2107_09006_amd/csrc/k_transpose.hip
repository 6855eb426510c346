// CSR transpose of A on the device (the A^T of the products A^T y, of the
// assembly and of the adjoint).
//
// The entries are sorted by column with a least-significant-digit radix sort
// on the column index (8-bit digits, as many passes as the column count
// needs), carrying each entry's index in A as its value.  Every pass is a
// stable counting sort, so inside a column the entries keep A's order, that
// is ascending rows.  A pass:
//   1. k_digit_hist: per tile of RS_TILE keys a 256-bin digit histogram,
//      stored digit-major (hist[digit * ntiles + tile]);
//   2. an exclusive scan of that array: the first output position of every
//      (digit, tile) pair;
//   3. k_digit_scatter: each tile ranks its keys among equal digits in input
//      order (wave ballots on the digit bits, per-wave counts in LDS) and
//      writes key and value to their positions.
// The row pointer of A^T is the exclusive scan of the column counts; the row
// of each entry is found by binary search in A's row pointer.
#include <mutex>
#include <string>

#include "kernels.hpp"

namespace lsq2l {

constexpr int RS_THREADS = 256;                 // threads of a sort workgroup
constexpr int RS_ITEMS = 16;                    // keys per thread and tile
constexpr int RS_TILE = RS_THREADS * RS_ITEMS;  // keys per tile
constexpr int RS_BINS = 256;
constexpr int SCAN_THREADS = 256, SCAN_ITEMS = 8, SCAN_TILE = SCAN_THREADS * SCAN_ITEMS;

// ---------------------------------------------------------------------------
// exclusive scan of int32 counts (in place), three phases
// ---------------------------------------------------------------------------
// Sum of v over the 256 threads of a block, and the exclusive prefix of each
// thread (fixed order: waves reduce by shuffles, then the four wave totals).
__device__ inline int block_excl_scan_256(int v, int* sh, int* total) {
  const int lane = threadIdx.x % 64, w = threadIdx.x / 64;
  int x = v;
#pragma unroll
  for (int o = 1; o < 64; o <<= 1) {
    const int y = __shfl_up(x, o, 64);
    if (lane >= o) x += y;
  }
  if (lane == 63) sh[w] = x;
  __syncthreads();
  int wbase = 0, tot = 0;
#pragma unroll
  for (int q = 0; q < RS_THREADS / 64; ++q) {
    if (q < w) wbase += sh[q];
    tot += sh[q];
  }
  __syncthreads();
  *total = tot;
  return wbase + x - v;
}

__global__ void __launch_bounds__(SCAN_THREADS)
k_scan_tiles(int64_t n, const int32_t* __restrict__ in, int32_t* __restrict__ tile_sum) {
  __shared__ int sh[4];
  const int64_t base = (int64_t)blockIdx.x * SCAN_TILE + (int64_t)threadIdx.x * SCAN_ITEMS;
  int s = 0;
#pragma unroll
  for (int q = 0; q < SCAN_ITEMS; ++q)
    if (base + q < n) s += in[base + q];
  int tot = 0;
  (void)block_excl_scan_256(s, sh, &tot);
  if (threadIdx.x == 0) tile_sum[blockIdx.x] = tot;
}

// exclusive scan of the tile sums by one workgroup, in chunks of 256
__global__ void __launch_bounds__(SCAN_THREADS)
k_scan_sums(int32_t ntiles, int32_t* __restrict__ tile_sum) {
  __shared__ int sh[4];
  int carry = 0;
  for (int32_t b0 = 0; b0 < ntiles; b0 += SCAN_THREADS) {
    const int32_t t = b0 + threadIdx.x;
    const int v = t < ntiles ? tile_sum[t] : 0;
    int tot = 0;
    const int ex = block_excl_scan_256(v, sh, &tot);
    if (t < ntiles) tile_sum[t] = carry + ex;
    carry += tot;
  }
}

__global__ void __launch_bounds__(SCAN_THREADS)
k_scan_apply(int64_t n, int32_t* __restrict__ v, const int32_t* __restrict__ tile_sum) {
  __shared__ int sh[4];
  const int64_t base = (int64_t)blockIdx.x * SCAN_TILE + (int64_t)threadIdx.x * SCAN_ITEMS;
  int x[SCAN_ITEMS];
  int s = 0;
#pragma unroll
  for (int q = 0; q < SCAN_ITEMS; ++q) {
    x[q] = base + q < n ? v[base + q] : 0;
    s += x[q];
  }
  int tot = 0;
  int run = tile_sum[blockIdx.x] + block_excl_scan_256(s, sh, &tot);
#pragma unroll
  for (int q = 0; q < SCAN_ITEMS; ++q)
    if (base + q < n) {
      v[base + q] = run;
      run += x[q];
    }
}

static int64_t scan_tiles(int64_t n) { return (n + SCAN_TILE - 1) / SCAN_TILE; }

// in-place exclusive scan of v[0..n); work: scan_tiles(n) int32
static void exclusive_scan(hipStream_t st, int64_t n, int32_t* v, int32_t* work) {
  if (n == 0) return;
  const unsigned nt = (unsigned)scan_tiles(n);
  k_scan_tiles<<<nt, SCAN_THREADS, 0, st>>>(n, v, work);
  k_scan_sums<<<1, SCAN_THREADS, 0, st>>>((int32_t)nt, work);
  k_scan_apply<<<nt, SCAN_THREADS, 0, st>>>(n, v, work);
}

// ---------------------------------------------------------------------------
// radix sort passes
// ---------------------------------------------------------------------------
// key of entry k in the first pass is colind[k] and its value k; later passes
// read the previous pass's output
__global__ void __launch_bounds__(RS_THREADS)
k_digit_hist(int64_t nnz, const int32_t* __restrict__ keys, int shift,
             int32_t* __restrict__ hist, int32_t ntiles) {
  __shared__ int cnt[RS_BINS];
  cnt[threadIdx.x] = 0;
  __syncthreads();
  const int64_t base = (int64_t)blockIdx.x * RS_TILE;
  for (int q = 0; q < RS_ITEMS; ++q) {
    const int64_t k = base + (int64_t)q * RS_THREADS + threadIdx.x;
    if (k < nnz) atomicAdd(&cnt[(keys[k] >> shift) & (RS_BINS - 1)], 1);
  }
  __syncthreads();
  hist[(int64_t)threadIdx.x * ntiles + blockIdx.x] = cnt[threadIdx.x];
}

// Stable scatter of one tile.  Round q takes keys base + q * 256 + t (thread
// t); in a round the lanes of wave w rank their key among the lanes of the
// wave with the same digit (8 ballots), the waves' digit counts are added in
// wave order, and a running count per digit carries the rounds.  Input
// order = (round, wave, lane), so equal digits keep their order.
__global__ void __launch_bounds__(RS_THREADS)
k_digit_scatter(int64_t nnz, const int32_t* __restrict__ keys, const int32_t* __restrict__ vals,
                int shift, const int32_t* __restrict__ hist, int32_t ntiles,
                int32_t* __restrict__ okeys, int32_t* __restrict__ ovals) {
  constexpr int NW = RS_THREADS / 64;
  __shared__ int run[RS_BINS];            // keys of each digit placed by earlier rounds
  __shared__ int wcnt[NW][RS_BINS];       // this round's count per wave and digit
  const int tid = threadIdx.x, lane = tid % 64, w = tid / 64;
  run[tid] = hist[(int64_t)tid * ntiles + blockIdx.x];
  const int64_t base = (int64_t)blockIdx.x * RS_TILE;
  const unsigned long long below = (lane == 0) ? 0ull : (~0ull >> (64 - lane));
  for (int q = 0; q < RS_ITEMS; ++q) {
    const int64_t k = base + (int64_t)q * RS_THREADS + tid;
    const bool valid = k < nnz;
    const int key = valid ? keys[k] : 0;
    const int val = valid ? (vals ? vals[k] : (int32_t)k) : 0;
    const int dg = (key >> shift) & (RS_BINS - 1);
#pragma unroll
    for (int p = 0; p < NW; ++p) wcnt[p][tid] = 0;
    __syncthreads();
    // lanes of this wave with a valid key of the same digit
    unsigned long long peers = __ballot(valid);
#pragma unroll
    for (int b = 0; b < 8; ++b) {
      const unsigned long long m = __ballot((dg >> b) & 1);
      peers &= ((dg >> b) & 1) ? m : ~m;
    }
    const int rank = __popcll(peers & below);
    // the lowest peer lane publishes the wave's count of this digit
    if (valid && rank == 0) wcnt[w][dg] = __popcll(peers);
    __syncthreads();
    if (valid) {
      int pos = run[dg] + rank;
      for (int p = 0; p < w; ++p) pos += wcnt[p][dg];
      okeys[pos] = key;
      ovals[pos] = val;
    }
    __syncthreads();
    int add = 0;
#pragma unroll
    for (int p = 0; p < NW; ++p) add += wcnt[p][tid];
    run[tid] += add;
    __syncthreads();
  }
}

// column counts; a column outside [0, n) is skipped (the caller reports it)
__global__ void k_col_count(int64_t nnz, const int32_t* __restrict__ colind, int32_t n,
                            int32_t* __restrict__ cnt) {
  const int64_t k = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (k < nnz) {
    const int32_t c = colind[k];
    if (c >= 0 && c < n) atomicAdd(&cnt[c], 1);
  }
}

__global__ void k_zero_fill_i32(int64_t n, int32_t v, int32_t* __restrict__ out) {
  const int64_t k = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (k < n) out[k] = v;
}

// trow[k] = the row of A holding entry tperm[k] (upper bound in rowptr);
// tvals[k] = vals[tperm[k]]
__global__ void k_rows_of(int64_t nnz, int32_t m, const int32_t* __restrict__ rowptr,
                          const int32_t* __restrict__ tperm, const double* __restrict__ vals,
                          int32_t* __restrict__ trow, double* __restrict__ tvals) {
  const int64_t k = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (k >= nnz) return;
  const int32_t e = tperm[k];
  int32_t lo = 0, hi = m - 1;             // largest r with rowptr[r] <= e
  while (lo < hi) {
    const int32_t mid = (lo + hi + 1) >> 1;
    if (rowptr[mid] <= e) lo = mid; else hi = mid - 1;
  }
  trow[k] = lo;
  if (tvals) tvals[k] = vals[e];
}

static int key_bits(int32_t n) {
  int b = 1;
  while (b < 31 && ((int64_t)1 << b) < n) ++b;
  return b;
}

static int passes_for(int32_t n) { return (key_bits(n) + 7) / 8; }

size_t transpose_temp_bytes(int64_t nnz, int32_t n) {
  const int64_t ntiles = (nnz + RS_TILE - 1) / RS_TILE;
  const int64_t hist = ntiles * RS_BINS;
  const int64_t scan = std::max(scan_tiles(hist), scan_tiles((int64_t)n + 1)) + 1;
  const int64_t pp = passes_for(n) >= 2 ? 2 * nnz : 0;   // ping-pong keys and values
  const int64_t words = hist + scan + pp;
  return (size_t)((words * 4 + 255) / 256 * 256);
}

hipError_t launch_transpose(hipStream_t st, int32_t m, int32_t n, int64_t nnz, const int32_t* rowptr,
                            const int32_t* colind, const double* vals, int32_t* trowptr,
                            int32_t* trow, double* tvals, int32_t* tperm, void* temp,
                            size_t temp_bytes) {
  if (temp_bytes < transpose_temp_bytes(nnz, n)) return hipErrorInvalidValue;
  const int64_t ntiles = (nnz + RS_TILE - 1) / RS_TILE;
  const int64_t nhist = ntiles * RS_BINS;
  int32_t* hist = (int32_t*)temp;
  int32_t* scanw = hist + nhist;
  int32_t* pk = scanw + std::max(scan_tiles(nhist), scan_tiles((int64_t)n + 1)) + 1;
  int32_t* pv = pk + nnz;
  // column counts -> row pointer of A^T
  k_zero_fill_i32<<<(unsigned)((n + 1 + 255) / 256), 256, 0, st>>>((int64_t)n + 1, 0, trowptr);
  if (nnz > 0)
    k_col_count<<<(unsigned)((nnz + 255) / 256), 256, 0, st>>>(nnz, colind, n, trowptr);
  exclusive_scan(st, (int64_t)n + 1, trowptr, scanw);
  if (nnz == 0) return hipGetLastError();
  // radix passes; the last one writes (trow, tperm), earlier ones alternate
  // so that the sequence ends there
  const int P = passes_for(n);
  const int32_t* ik = colind;
  const int32_t* iv = nullptr;             // first pass: values are the entry indices
  for (int p = 0; p < P; ++p) {
    const bool to_out = ((P - 1 - p) % 2) == 0;
    int32_t* ok = to_out ? trow : pk;
    int32_t* ov = to_out ? tperm : pv;
    k_digit_hist<<<(unsigned)ntiles, RS_THREADS, 0, st>>>(nnz, ik, 8 * p, hist, (int32_t)ntiles);
    exclusive_scan(st, nhist, hist, scanw);
    k_digit_scatter<<<(unsigned)ntiles, RS_THREADS, 0, st>>>(nnz, ik, iv, 8 * p, hist,
                                                             (int32_t)ntiles, ok, ov);
    ik = ok;
    iv = ov;
  }
  k_rows_of<<<(unsigned)((nnz + 255) / 256), 256, 0, st>>>(nnz, m, rowptr, tperm, vals, trow, tvals);
  return hipGetLastError();
}

// Row i of the row-permuted copy is row perm[i] of A (one thread per row;
// prowptr holds the permuted row starts).
__global__ void k_permute_rows(int32_t m, const int32_t* __restrict__ perm,
                               const int32_t* __restrict__ rowptr, const int32_t* __restrict__ colind,
                               const double* __restrict__ vals, const int32_t* __restrict__ prowptr,
                               int32_t* __restrict__ pcolind, double* __restrict__ pvals) {
  const int32_t i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= m) return;
  const int32_t r = perm[i];
  int32_t d = prowptr[i];
  for (int32_t k = rowptr[r]; k < rowptr[r + 1]; ++k, ++d) {
    pcolind[d] = colind[k];
    pvals[d] = vals[k];
  }
}

void launch_permute_rows(hipStream_t st, int32_t m, const int32_t* perm, const int32_t* rowptr,
                         const int32_t* colind, const double* vals, const int32_t* prowptr,
                         int32_t* pcolind, double* pvals) {
  if (m == 0) return;
  k_permute_rows<<<(m + 255) / 256, 256, 0, st>>>(m, perm, rowptr, colind, vals, prowptr, pcolind, pvals);
}

// flag[0] = 1 if a column index lies outside [0, n) (the sort's counters and
// positions assume valid columns)
__global__ void k_check_cols(int64_t nnz, const int32_t* __restrict__ colind, int32_t n,
                             int32_t* __restrict__ flag) {
  const int64_t k = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (k < nnz && (colind[k] < 0 || colind[k] >= n)) flag[0] = 1;
}

void launch_check_cols(hipStream_t st, int64_t nnz, const int32_t* colind, int32_t n, int32_t* flag) {
  k_zero_fill_i32<<<1, 64, 0, st>>>(1, 0, flag);
  if (nnz == 0) return;
  k_check_cols<<<(unsigned)((nnz + 255) / 256), 256, 0, st>>>(nnz, colind, n, flag);
}

// ---------------------------------------------------------------------------
// Input of the setup: the CSR arrays of all instances concatenated into the
// handle's copy of A (row pointers narrowed to int32 and shifted by the
// instance's first entry, columns shifted by its first column), checked on
// the way.  A failed check records the smallest failing (global) row of its
// kind in bad[kind] (atomicMin; INT64_MAX when none): CSR_FIRST rowptr[0] !=
// 0, CSR_LAST rowptr[m] != nnz, CSR_MONO a row start below the previous one
// or above nnz, CSR_RANGE a column outside [0, n), CSR_ORDER columns not
// strictly increasing.  Reads never leave an instance's arrays, whatever
// they hold.
// ---------------------------------------------------------------------------
// the instance holding global index g of the table field (r0 or e0)
__device__ inline int instance_of(const InstDesc* __restrict__ d, int S, int64_t g, bool by_rows) {
  int lo = 0, hi = S - 1;
  while (lo < hi) {
    const int mid = (lo + hi + 1) >> 1;
    if ((by_rows ? d[mid].r0 : d[mid].e0) <= g) lo = mid;
    else hi = mid - 1;
  }
  return lo;
}

__global__ void k_concat_rows(int S, const InstDesc* __restrict__ d, int64_t M,
                              int32_t* __restrict__ rp, unsigned long long* __restrict__ bad) {
  const int64_t g = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (g >= M) return;
  const int k = instance_of(d, S, g, true);
  const InstDesc D = d[k];
  const int64_t r = g - D.r0;
  const int64_t lo = D.rowptr[r], hi = D.rowptr[r + 1];
  if (r == 0 && lo != 0) atomicMin(&bad[CSR_FIRST], (unsigned long long)g);
  if (r == D.m - 1 && hi != D.nnz) atomicMin(&bad[CSR_LAST], (unsigned long long)g);
  if (hi < lo || hi > D.nnz) atomicMin(&bad[CSR_MONO], (unsigned long long)g);
  rp[g + 1] = (int32_t)(D.e0 + min(max(hi, (int64_t)0), D.nnz));
  if (g == 0) rp[0] = 0;
}

__global__ void k_concat_entries(int S, const InstDesc* __restrict__ d, int64_t NNZ,
                                 int32_t* __restrict__ ci, double* __restrict__ vals) {
  const int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (e >= NNZ) return;
  const int k = instance_of(d, S, e, false);
  const InstDesc D = d[k];
  const int64_t q = e - D.e0;
  ci[e] = D.colind[q] + (int32_t)D.c0;
  vals[e] = D.vals[q];
}

// columns of every row (rp as written by k_concat_rows: inside each
// instance's entries even for a corrupt rowptr)
__global__ void k_check_rows(int S, const InstDesc* __restrict__ d, int64_t M,
                             const int32_t* __restrict__ rp, const int32_t* __restrict__ ci,
                             unsigned long long* __restrict__ bad) {
  const int64_t g = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (g >= M) return;
  const int k = instance_of(d, S, g, true);
  const InstDesc D = d[k];
  const int32_t a = rp[g], b = rp[g + 1];
  const int64_t c0 = D.c0, c1 = D.c0 + D.n;
  for (int32_t e = a; e < b; ++e) {
    const int32_t c = ci[e];
    if (c < c0 || c >= c1) { atomicMin(&bad[CSR_RANGE], (unsigned long long)g); return; }
    if (e > a && c <= ci[e - 1]) { atomicMin(&bad[CSR_ORDER], (unsigned long long)g); return; }
  }
}

__global__ void k_fill_u64(int n, unsigned long long v, unsigned long long* __restrict__ out) {
  const int k = blockIdx.x * blockDim.x + threadIdx.x;
  if (k < n) out[k] = v;
}

void launch_concat(hipStream_t st, int S, const InstDesc* d, int64_t M, int64_t NNZ, int32_t* rp,
                   int32_t* ci, double* vals, unsigned long long* bad) {
  k_fill_u64<<<1, 64, 0, st>>>(CSR_KINDS, ~0ull, bad);
  k_concat_rows<<<(unsigned)((M + 255) / 256), 256, 0, st>>>(S, d, M, rp, bad);
  if (NNZ > 0)
    k_concat_entries<<<(unsigned)((NNZ + 255) / 256), 256, 0, st>>>(S, d, NNZ, ci, vals);
  k_check_rows<<<(unsigned)((M + 255) / 256), 256, 0, st>>>(S, d, M, rp, ci, bad);
}

// ---------------------------------------------------------------------------
// Transpose without allocation: the sort's work arrays live in a file-scope
// device array, `scratch`, of TRANSPOSE_SCRATCH_BYTES, which every GPU the
// library runs on holds until the process ends.  Its device address is taken
// once per device with hipGetSymbolAddress (the array's name in host code is
// only a host-side stand-in) and kept per device.
// ---------------------------------------------------------------------------
namespace {
constexpr size_t TRANSPOSE_SCRATCH_BYTES = (size_t)104 << 20;
constexpr int MAX_DEVICES = 64;
}  // namespace

static __device__ __align__(256) unsigned char scratch[TRANSPOSE_SCRATCH_BYTES];

namespace {
std::mutex g_scratch_mu;
void* g_scratch_ptr[MAX_DEVICES] = {};

// device address of `scratch` on the current device
hipError_t scratch_address(void** out) {
  int dev = 0;
  hipError_t e = hipGetDevice(&dev);
  if (e != hipSuccess) return e;
  if (dev < 0 || dev >= MAX_DEVICES) return hipErrorInvalidDevice;
  std::lock_guard<std::mutex> g(g_scratch_mu);
  if (!g_scratch_ptr[dev]) {
    void* p = nullptr;
    e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
    if (e != hipSuccess) return e;
    g_scratch_ptr[dev] = p;
  }
  *out = g_scratch_ptr[dev];
  return hipSuccess;
}
}  // namespace

}  // namespace lsq2l

extern "C" lsq2l_status lsq2l_transpose_noalloc(int32_t m, int32_t n, int32_t nnz,
                                                const int32_t* rowptr, const int32_t* colind,
                                                const double* vals, int32_t* trowptr,
                                                int32_t* trow, double* tvals, int32_t* tperm,
                                                void* hip_stream) {
  using namespace lsq2l;
  if (m < 0 || n < 0 || nnz < 0 || !rowptr || !trowptr || (nnz > 0 && (!colind || !trow)) ||
      (nnz > 0 && tvals && !vals)) {
    set_error("bad sizes or NULL required pointer");
    return LSQ2L_EINVAL;
  }
  const size_t tb = transpose_temp_bytes(nnz, n);
  const size_t perm_bytes = tperm ? 0 : ((size_t)nnz * sizeof(int32_t) + 255) / 256 * 256;
  if (tb + perm_bytes + 256 > TRANSPOSE_SCRATCH_BYTES) {
    set_error("transpose without allocation: n = " + std::to_string(n) + ", nnz = " +
              std::to_string(nnz) + " need " + std::to_string(tb + perm_bytes + 256) +
              " bytes of work space, above the " + std::to_string(TRANSPOSE_SCRATCH_BYTES) +
              " bytes held per device");
    return LSQ2L_EINVAL;
  }
  const hipStream_t st = (hipStream_t)hip_stream;
  void* base = nullptr;
  hipError_t e = scratch_address(&base);
  if (e != hipSuccess) {
    set_error(std::string("transpose without allocation: hipGetSymbolAddress: ") + hipGetErrorString(e));
    return LSQ2L_EHIP;
  }
  int32_t* perm = tperm ? tperm : (int32_t*)((char*)base + tb);
  int32_t* flag = (int32_t*)((char*)base + tb + perm_bytes);
  int32_t hflag = 0;
  launch_check_cols(st, nnz, colind, n, flag);
  e = hipMemcpyAsync(&hflag, flag, sizeof(int32_t), hipMemcpyDeviceToHost, st);
  if (e == hipSuccess) e = hipStreamSynchronize(st);
  if (e == hipSuccess && hflag == 0)
    e = launch_transpose(st, m, n, nnz, rowptr, colind, vals, trowptr, trow, tvals, perm, base, tb);
  if (e == hipSuccess) e = hipStreamSynchronize(st);
  if (e != hipSuccess) {
    set_error(std::string("transpose without allocation: ") + hipGetErrorString(e));
    return LSQ2L_EHIP;
  }
  if (hflag) {
    set_error("transpose: a column index lies outside [0, n)");
    return LSQ2L_EINVAL;
  }
  return LSQ2L_OK;
}

