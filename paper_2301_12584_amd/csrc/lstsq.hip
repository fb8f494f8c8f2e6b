// The sketched least-squares assembly of STS-CP (Section 3.3; Appendix A.9
// for the solve's pieces; Appendix A.13 for the reduction of the sampled
// spMTTKRP to an SpMM) and the exact fit (Section 4.3).
//
//   fiber index : per mode j the COO entries sorted by the other modes'
//                 indices (increasing mode order), then i_j -- the mode-j
//                 fibers, i.e. the rows of mat(T, j)^T, are contiguous; an
//                 offset table over the leading other mode narrows lookups.
//                 Entries with equal coordinates are merged into one stored
//                 entry whose float64 value is their sum (duplicates mean a
//                 sum), so a fiber holds each i_j at most once.
//   lookup      : per sample, the entry range of its fiber (offset table,
//                 then binary search on the remaining modes).
//   merge       : samples drawn more than once select the same fiber and
//                 the same row a_d; their weights w_d^2 are summed in a
//                 hash table keyed by the fiber, and only the first such
//                 sample expands the fiber (the rows of the sampling matrix
//                 are i.i.d. draws, Section 2.1; repeated rows add).  This
//                 bounds the SpMM by the stored entries.
//   SpMM        : Y[i_j(e), :] += (sum w^2 / w_d) x_e (w_d a_d) over the
//                 entries of each distinct sampled fiber, split into chunks
//                 of CH entries so that heavy fibers spread over many
//                 wavefronts (float64 atomics on Y).
//   solve       : U_j = Y M^+ (M^+ in LDS, float64 products), per-column
//                 sums of squares reduced deterministically, sigma, and the
//                 renormalisation of U_j.
//   fit         : <T, T~> over the stored entries and sigma^T (*G_k) sigma.
#include <rocprim/device/device_radix_sort.hpp>
#include <rocprim/device/device_reduce_by_key.hpp>
#include <rocprim/device/device_scan.hpp>
#include <rocprim/iterator/counting_iterator.hpp>
#include <rocprim/iterator/discard_iterator.hpp>
#include <rocprim/iterator/transform_iterator.hpp>

#include "device_common.h"
#include "krps_internal.h"

namespace krps {

namespace {

constexpr int CH = 64;  // fiber entries per SpMM work item (one per lane)

__global__ void fill_u32_kernel(uint32_t* __restrict__ p, int64_t n) {
  for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n;
       i += (int64_t)gridDim.x * blockDim.x)
    p[i] = 0u;
}

__global__ void iota_kernel(uint32_t* __restrict__ p, int64_t n) {
  for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n;
       i += (int64_t)gridDim.x * blockDim.x)
    p[i] = (uint32_t)i;
}

__global__ void gather_key_kernel(uint32_t* __restrict__ keys, const int32_t* __restrict__ idx,
                                  const uint32_t* __restrict__ perm, int N, int col, int64_t n) {
  for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n;
       i += (int64_t)gridDim.x * blockDim.x)
    keys[i] = (uint32_t)idx[(int64_t)perm[i] * N + col];
}

// head[e] = 1 where the sorted entry e starts a run of equal coordinates.
__global__ void head_kernel(uint32_t* __restrict__ head, const int32_t* __restrict__ idx,
                            const uint32_t* __restrict__ perm, int N, int64_t n) {
  for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n;
       i += (int64_t)gridDim.x * blockDim.x) {
    bool h = i == 0;
    if (!h) {
      const int32_t* __restrict__ a = idx + (int64_t)perm[i] * N;
      const int32_t* __restrict__ b = idx + (int64_t)perm[i - 1] * N;
      for (int k = 0; k < N; ++k) h = h || a[k] != b[k];
    }
    head[i] = h ? 1u : 0u;
  }
}

// Columns of the merged sorted copy for one mode: the head of each run of
// equal coordinates (run number rid[e] - 1) writes its indices.
__global__ void coalesce_cols_kernel(int32_t* __restrict__ cols, const int32_t* __restrict__ idx,
                                     const uint32_t* __restrict__ perm,
                                     const uint32_t* __restrict__ head,
                                     const uint32_t* __restrict__ rid, int N, int64_t n,
                                     int64_t nu) {
  for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n;
       i += (int64_t)gridDim.x * blockDim.x) {
    if (head[i] == 0) continue;
    const int64_t q = (int64_t)rid[i] - 1;
    const int64_t p = perm[i];
    for (int k = 0; k < N; ++k) cols[(int64_t)k * nu + q] = idx[p * N + k];
  }
}

// Value of sorted entry i as float64 (the input of the run sums).
struct SortedValue {
  const float* val;
  const uint32_t* perm;
  __host__ __device__ double operator()(uint32_t i) const { return (double)val[perm[i]]; }
};

// off[v] = first entry whose leading key is >= v, for v in [0, dim].
__global__ void offsets_kernel(int64_t* __restrict__ off, const int32_t* __restrict__ key,
                               int64_t n, int64_t dim) {
  for (int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; e <= n;
       e += (int64_t)gridDim.x * blockDim.x) {
    const int64_t prev = e == 0 ? -1 : key[e - 1];
    const int64_t cur = e == n ? dim : key[e];
    for (int64_t v = prev + 1; v <= cur; ++v) off[v] = e;
  }
}

// ||T||^2 over the merged entries (each coordinate stored once): block
// partials out[1 + b], then their sum in a fixed order into out[0], so the
// norm repeats bit for bit.
constexpr int NORM_BLOCKS = 1024;

__global__ void norm2_kernel(const double* __restrict__ vals, int64_t n,
                             double* __restrict__ out) {
  __shared__ double red[256];
  double acc = 0;
  for (int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; e < n;
       e += (int64_t)gridDim.x * blockDim.x)
    acc += vals[e] * vals[e];
  red[threadIdx.x] = acc;
  __syncthreads();
  for (int o = blockDim.x / 2; o > 0; o >>= 1) {
    if ((int)threadIdx.x < o) red[threadIdx.x] += red[threadIdx.x + o];
    __syncthreads();
  }
  if (threadIdx.x == 0) out[1 + blockIdx.x] = red[0];
}

__global__ void norm2_final_kernel(double* __restrict__ out) {
  if (threadIdx.x != 0) return;
  double sum = 0.0;
  for (int b = 0; b < NORM_BLOCKS; ++b) sum += out[1 + b];
  out[0] = sum;
}

}  // namespace

// ------------------------------------------------------------------ tensor

size_t sort_temp_bytes(int64_t nnz) {
  size_t bytes = 0, sb = 0, rb = 0;
  (void)rocprim::radix_sort_pairs(nullptr, bytes, (uint32_t*)nullptr, (uint32_t*)nullptr,
                                  (uint32_t*)nullptr, (uint32_t*)nullptr, (uint32_t)nnz, 0, 32);
  (void)rocprim::inclusive_scan(nullptr, sb, (const uint32_t*)nullptr, (uint32_t*)nullptr,
                                (size_t)nnz, rocprim::plus<uint32_t>());
  auto vin = rocprim::make_transform_iterator(rocprim::make_counting_iterator<uint32_t>(0),
                                              SortedValue{nullptr, nullptr});
  (void)rocprim::reduce_by_key(nullptr, rb, (const uint32_t*)nullptr, vin, (size_t)nnz,
                               rocprim::make_discard_iterator(), (double*)nullptr,
                               rocprim::make_discard_iterator(), rocprim::plus<double>(),
                               rocprim::equal_to<uint32_t>());
  size_t m = bytes > sb ? bytes : sb;
  return m > rb ? m : rb;
}

static int bits_of(int64_t dim) {
  int b = 1;
  while ((int64_t(1) << b) < dim) ++b;
  return b;
}

hipError_t build_fiber_index(hipStream_t st, int N, const int64_t* dims, int64_t nnz,
                             const int32_t* idx, const float* val, int j, int32_t* cols,
                             double* vals, int64_t* off, uint32_t* k0, uint32_t* k1, uint32_t* p0,
                             uint32_t* p1, void* temp, size_t temp_bytes, int64_t* nu) {
  const int grid = 4096, block = 256;
  hipLaunchKernelGGL(iota_kernel, dim3(grid), dim3(block), 0, st, p0, nnz);
  // LSD: least significant key first (i_j), then the other modes from the
  // last to the first; each pass is a stable sort of the current order
  int order[KRPS_MAX_MODES + 1];
  int no = 0;
  order[no++] = j;
  for (int k = N - 1; k >= 0; --k)
    if (k != j) order[no++] = k;
  for (int pass = 0; pass < no; ++pass) {
    const int col = order[pass];
    hipLaunchKernelGGL(gather_key_kernel, dim3(grid), dim3(block), 0, st, k0, idx, p0, N, col, nnz);
    size_t tb = temp_bytes;
    hipError_t e = rocprim::radix_sort_pairs(temp, tb, k0, k1, p0, p1, (uint32_t)nnz, 0,
                                             bits_of(dims[col]), st);
    if (e != hipSuccess) return e;
    uint32_t* t = p0;
    p0 = p1;
    p1 = t;
  }
  // runs of equal coordinates -> one stored entry each (k0: heads, k1: run
  // number, 1-based); each run's value is its float64 sum in sorted order
  hipLaunchKernelGGL(head_kernel, dim3(grid), dim3(block), 0, st, k0, idx, p0, N, nnz);
  size_t tb = temp_bytes;
  hipError_t e = rocprim::inclusive_scan(temp, tb, k0, k1, (size_t)nnz,
                                         rocprim::plus<uint32_t>(), st);
  if (e != hipSuccess) return e;
  if (*nu < 0) {  // the count of distinct coordinates is the same in every mode
    uint32_t last = 0;
    e = hipMemcpyAsync(&last, k1 + nnz - 1, 4, hipMemcpyDeviceToHost, st);
    if (e == hipSuccess) e = hipStreamSynchronize(st);
    if (e != hipSuccess) return e;
    *nu = (int64_t)last;
  }
  auto vin = rocprim::make_transform_iterator(rocprim::make_counting_iterator<uint32_t>(0),
                                              SortedValue{val, p0});
  tb = temp_bytes;
  e = rocprim::reduce_by_key(temp, tb, (const uint32_t*)k1, vin, (size_t)nnz,
                             rocprim::make_discard_iterator(), vals,
                             rocprim::make_discard_iterator(), rocprim::plus<double>(),
                             rocprim::equal_to<uint32_t>(), st);
  if (e != hipSuccess) return e;
  hipLaunchKernelGGL(coalesce_cols_kernel, dim3(grid), dim3(block), 0, st, cols, idx, p0, k0, k1,
                     N, nnz, *nu);
  int lead = j == 0 ? 1 : 0;
  if (N == 1) lead = 0;
  hipLaunchKernelGGL(offsets_kernel, dim3(grid), dim3(block), 0, st, off,
                     cols + (int64_t)lead * *nu, *nu, dims[lead]);
  return hipGetLastError();
}

hipError_t launch_norm2(hipStream_t st, const double* vals, int64_t n, double* out) {
  hipLaunchKernelGGL(norm2_kernel, dim3(NORM_BLOCKS), dim3(256), 0, st, vals, n, out);
  hipLaunchKernelGGL(norm2_final_kernel, dim3(1), dim3(64), 0, st, out);
  return hipGetLastError();
}

size_t norm2_bytes() { return (size_t)(NORM_BLOCKS + 1) * 8; }

// ---------------------------------------------------------------- hot rows
//
// The HOT_ROWS rows of each mode that hold the most stored entries: the
// SpMM accumulates their updates in LDS per workgroup and adds them to Y
// once per workgroup, so the most popular rows of a power-law mode do not
// serialise the float64 atomics on a few addresses.

namespace {

// Entries per row.  A power-law mode sends a large share of all entries to
// a handful of rows, so each workgroup first counts in a small LDS hash
// table (the popular rows arrive early and take its slots) and falls back to
// global atomics for rows it finds no slot for; the table is added to the
// global counts at the end.
constexpr int HC_SLOTS = 2048, HC_PROBES = 8;

__global__ __launch_bounds__(256) void hot_count_kernel(const int32_t* __restrict__ col, int64_t n,
                                                        uint32_t* __restrict__ count) {
  __shared__ int32_t key[HC_SLOTS];
  __shared__ uint32_t cnt[HC_SLOTS];
  for (int q = threadIdx.x; q < HC_SLOTS; q += blockDim.x) {
    key[q] = -1;
    cnt[q] = 0;
  }
  __syncthreads();
  for (int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; e < n;
       e += (int64_t)gridDim.x * blockDim.x) {
    const int32_t v = col[e];
    uint32_t h = (uint32_t)v * 2654435761u;
    bool done = false;
    for (int p = 0; p < HC_PROBES && !done; ++p) {
      const int q = (int)((h >> 21) + p) & (HC_SLOTS - 1);
      int32_t k = key[q];
      if (k == -1) {
        const int32_t old = atomicCAS(&key[q], -1, v);
        k = old == -1 ? v : old;
      }
      if (k == v) {
        atomicAdd(&cnt[q], 1u);
        done = true;
      }
    }
    if (!done) atomicAdd(&count[v], 1u);
  }
  __syncthreads();
  for (int q = threadIdx.x; q < HC_SLOTS; q += blockDim.x)
    if (cnt[q] != 0) atomicAdd(&count[key[q]], cnt[q]);
}

__global__ void hot_clear_kernel(uint32_t* __restrict__ count, uint32_t* __restrict__ index,
                                 int16_t* __restrict__ slot, int64_t dim) {
  for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < dim;
       i += (int64_t)gridDim.x * blockDim.x) {
    count[i] = 0;
    index[i] = (uint32_t)i;
    slot[i] = -1;
  }
}

__global__ void hot_pick_kernel(const uint32_t* __restrict__ sorted_index, int nhot,
                                int32_t* __restrict__ rows, int16_t* __restrict__ slot) {
  for (int s = threadIdx.x; s < nhot; s += blockDim.x) {
    const uint32_t i = sorted_index[s];
    rows[s] = (int32_t)i;
    slot[i] = (int16_t)s;
  }
}

}  // namespace

size_t hot_temp_bytes(int64_t dim) {
  size_t bytes = 0;
  (void)rocprim::radix_sort_pairs_desc(nullptr, bytes, (uint32_t*)nullptr, (uint32_t*)nullptr,
                                       (uint32_t*)nullptr, (uint32_t*)nullptr, (uint32_t)dim, 0,
                                       32);
  return bytes;
}

hipError_t build_hot_rows(hipStream_t st, const int32_t* col, int64_t n, int64_t dim, int nhot,
                          uint32_t* c0, uint32_t* c1, uint32_t* i0, uint32_t* i1, void* temp,
                          size_t temp_bytes, int32_t* rows, int16_t* slot) {
  hipLaunchKernelGGL(hot_clear_kernel, dim3(1024), dim3(256), 0, st, c0, i0, slot, dim);
  hipLaunchKernelGGL(hot_count_kernel, dim3(4096), dim3(256), 0, st, col, n, c0);
  size_t tb = temp_bytes;
  hipError_t e = rocprim::radix_sort_pairs_desc(temp, tb, c0, c1, i0, i1, (uint32_t)dim, 0, 32,
                                                st);
  if (e != hipSuccess) return e;
  hipLaunchKernelGGL(hot_pick_kernel, dim3(1), dim3(256), 0, st, i1, nhot, rows, slot);
  return hipGetLastError();
}

// ------------------------------------------------------------------ lookup

namespace {

// Entry range of the fiber of sample d in the mode-j index: offsets over
// the leading other mode, then lexicographic binary search on the rest.
__global__ void lookup_kernel(FiberArgs a) {
  const int N = a.N;
  for (int64_t d = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; d < a.J;
       d += (int64_t)gridDim.x * blockDim.x) {
    const int32_t* __restrict__ sidx = a.sample_idx + d * N;
    int64_t lo = 0, hi = 0;
    if (N > 1) {
      const int v = sidx[a.lead];
      lo = a.off[v];
      hi = a.off[v + 1];
      // remaining other modes, in increasing order
      for (int k = a.lead + 1; k < N; ++k) {
        if (k == a.j) continue;
        const int32_t* __restrict__ c = a.cols + (int64_t)k * a.nnz;
        const int key = sidx[k];
        int64_t l = lo, r = hi;
        while (l < r) {  // first >= key
          const int64_t m = (l + r) >> 1;
          if (c[m] < key) l = m + 1; else r = m;
        }
        int64_t l2 = l, r2 = hi;
        while (l2 < r2) {  // first > key
          const int64_t m = (l2 + r2) >> 1;
          if (c[m] <= key) l2 = m + 1; else r2 = m;
        }
        lo = l;
        hi = l2;
      }
    } else {
      lo = 0;
      hi = a.nnz;
    }
    a.lo[d] = lo;
    a.hi[d] = hi;
  }
}

constexpr unsigned long long EMPTY_KEY = ~0ull;

__global__ void merge_clear_kernel(FiberArgs a) {
  for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < a.H;
       i += (int64_t)gridDim.x * blockDim.x) {
    a.hkey[i] = EMPTY_KEY;
    a.hW[i] = 0.0;  // also the int64 zero of the fixed-point high words
    if (a.hWlo != nullptr) a.hWlo[i] = 0;
    a.hrep[i] = INT32_MAX;
  }
}

// Deterministic mode: the per-fiber sums of w_d^2 are fixed point with
// 2^-S units, S = 93 - ceil(log2 B) for B = sum_d w_d^2 (>= every fiber's
// sum; reduced here in a fixed order), kept as two int64 words (the high
// word counts 2^32 units): about 93 significant bits, with every partial
// sum exact, so their order does not matter.
__global__ __launch_bounds__(1024) void w2_scale_kernel(FiberArgs a) {
  __shared__ double red[1024];
  double acc = 0.0;
  for (int64_t d = threadIdx.x; d < a.J; d += blockDim.x) {
    const double wd = a.w[d];
    acc += wd * wd;
  }
  red[threadIdx.x] = acc;
  __syncthreads();
  for (int h = 512; h > 0; h >>= 1) {
    if ((int)threadIdx.x < h) red[threadIdx.x] += red[threadIdx.x + h];
    __syncthreads();
  }
  if (threadIdx.x == 0) {
    const double B = red[0] * (1.0 + 1e-9);
    const int S = B > 0.0 ? 93 - (ilogb(B) + 1) : 0;
    a.wscale[0] = ldexp(1.0, S);
    a.wscale[1] = ldexp(1.0, -S);
  }
}

__device__ __forceinline__ int wave_min(int v) {
#pragma unroll
  for (int o = 32; o > 0; o >>= 1) {
    const int u = __shfl_xor(v, o);
    v = u < v ? u : v;
  }
  return v;
}

// Inserts every sample with a nonempty fiber into the hash table keyed by
// the fiber's first entry: the slot accumulates sum w_d^2 and the smallest
// d.  Lanes of a wavefront holding the same key are combined first (one
// leader per key), so a fiber drawn thousands of times costs few atomics.
// H >= 2 J, so an empty slot is always found within H probes.
__global__ __launch_bounds__(256) void merge_insert_kernel(FiberArgs a) {
  const int lane = threadIdx.x & 63;
  const int64_t wave = ((int64_t)blockIdx.x * blockDim.x + threadIdx.x) >> 6;
  const int64_t nwaves = ((int64_t)gridDim.x * blockDim.x) >> 6;
  for (int64_t base = wave * 64; base < a.J; base += nwaves * 64) {
    const int64_t d = base + lane;
    bool active = false;
    int64_t key = 0;
    double w2 = 0.0;
    if (d < a.J) {
      key = a.lo[d];
      const double wd = a.w[d];
      // a sample of weight 0 (see the walk) expands nothing
      active = a.hi[d] > key && wd > 0.0;
      w2 = wd * wd;
    }
    int myslot = -1;
    for (;;) {
      const unsigned long long m = __ballot(active);
      if (m == 0) break;
      const int leader = __ffsll((long long)m) - 1;
      const int64_t lkey = __shfl(key, leader);
      const bool mine = active && key == lkey;
      const double v = wave_sum(mine ? w2 : 0.0);
      const int dmin = wave_min(mine ? (int)d : INT32_MAX);
      int slot = 0;
      if (lane == leader) {
        uint64_t h = ((uint64_t)lkey * 0x9E3779B97F4A7C15ull) >> (64 - a.hbits);
        for (int64_t probe = 0; probe < a.H; ++probe) {
          const unsigned long long prev =
              atomicCAS(&a.hkey[h], EMPTY_KEY, (unsigned long long)lkey);
          if (prev == EMPTY_KEY || prev == (unsigned long long)lkey) break;
          h = (h + 1) & (uint64_t)(a.H - 1);
        }
        slot = (int)h;
        if (a.hWlo != nullptr) {
          // t = v 2^S < 2^93 split exactly into 2^32 units and the rest
          const double t = v * a.wscale[0];
          const double hi = floor(t * 0x1p-32);
          const double lo = floor(t - hi * 0x1p32);
          atomicAdd((unsigned long long*)&a.hW[slot], (unsigned long long)(long long)hi);
          atomicAdd((unsigned long long*)&a.hWlo[slot], (unsigned long long)(long long)lo);
        } else {
          atomicAdd(&a.hW[slot], v);
        }
        atomicMin(&a.hrep[slot], dmin);
      }
      slot = __shfl(slot, leader);
      if (mine) {
        myslot = slot;
        active = false;
      }
    }
    if (d < a.J) a.slot[d] = myslot;
  }
}

// The first sample of each distinct fiber expands it with coefficient
// (sum w^2) / w_d applied to its stored row w_d a_d; the others expand
// nothing.
__global__ void merge_finish_kernel(FiberArgs a) {
  for (int64_t d = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; d < a.J;
       d += (int64_t)gridDim.x * blockDim.x) {
    const int s = a.slot[d];
    int64_t c = 0;
    double coef = 0.0;
    if (s >= 0 && a.hrep[s] == (int)d) {
      c = (a.hi[d] - a.lo[d] + CH - 1) / CH;
      double W = a.hW[s];
      if (a.hWlo != nullptr) {
        const long long hi = __double_as_longlong(a.hW[s]);
        W = ((double)hi * 0x1p32 + (double)a.hWlo[s]) * a.wscale[1];
      }
      coef = W / a.w[d];
    }
    a.cnt[d] = c;
    a.coef[d] = coef;
    a.rflag[d] = c > 0 ? 1 : 0;
  }
}

// The samples that expand a fiber, in sample order: rep[k] and the first
// work item rstart[k] of the k-th of them (rstart[nrep] = all items).
__global__ void compact_kernel(FiberArgs a) {
  for (int64_t d = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; d <= a.J;
       d += (int64_t)gridDim.x * blockDim.x) {
    if (d == a.J) {
      a.rstart[a.rpos[a.J]] = a.start[a.J];
    } else if (a.cnt[d] > 0) {
      const int64_t k = a.rpos[d];
      a.rep[k] = (int32_t)d;
      a.rstart[k] = a.start[d];
    }
  }
}

// Entries the SpMM expands: the sizes of the distinct sampled fibers,
// summed by one block in a fixed order (a measurement, read by callers).
__global__ __launch_bounds__(1024) void expanded_kernel(FiberArgs a) {
  __shared__ int64_t red[16];
  int64_t sum = 0;
  for (int64_t d = threadIdx.x; d < a.J; d += blockDim.x)
    if (a.cnt[d] > 0) sum += a.hi[d] - a.lo[d];
  for (int o = 32; o > 0; o >>= 1) sum += __shfl_down(sum, o, 64);
  if ((threadIdx.x & 63) == 0) red[threadIdx.x >> 6] = sum;
  __syncthreads();
  if (threadIdx.x == 0) {
    int64_t t = 0;
    for (int w = 0; w < (int)(blockDim.x >> 6); ++w) t += red[w];
    *a.expanded = t;
  }
}

// Exclusive scan of cnt[0..J) into start[0..J] (start[J] = the total) in
// three launches: tiles of 1024 (wave scans, then the 16 wave totals),
// the tile totals, and the tile offsets added back.
constexpr int SCAN_TILE = 1024;

__device__ __forceinline__ int64_t wave_incl_scan_i64(int64_t x, int lane) {
#pragma unroll
  for (int o = 1; o < 64; o <<= 1) {
    const int64_t y = __shfl_up(x, o, 64);
    if (lane >= o) x += y;
  }
  return x;
}

__global__ __launch_bounds__(SCAN_TILE) void scan_tiles_kernel(const int64_t* __restrict__ cnt,
                                                               int64_t* __restrict__ start,
                                                               int64_t* __restrict__ bsum,
                                                               int64_t J) {
  __shared__ int64_t wsum[SCAN_TILE / 64];
  const int t = threadIdx.x, lane = t & 63, wave = t >> 6;
  const int64_t i = (int64_t)blockIdx.x * SCAN_TILE + t;
  const int64_t v = i < J ? cnt[i] : 0;
  int64_t x = wave_incl_scan_i64(v, lane);
  if (lane == 63) wsum[wave] = x;
  __syncthreads();
  if (wave == 0) {
    const int64_t w = lane < SCAN_TILE / 64 ? wsum[lane] : 0;
    const int64_t wi = wave_incl_scan_i64(w, lane);
    if (lane < SCAN_TILE / 64) wsum[lane] = wi - w;  // exclusive
    if (lane == SCAN_TILE / 64 - 1) bsum[blockIdx.x] = wi;
  }
  __syncthreads();
  x += wsum[wave];
  if (i < J) start[i] = x - v;
}

// Exclusive scan of the nb tile totals in place; bsum[nb] = the total.
__global__ __launch_bounds__(1024) void scan_bsum_kernel(int64_t* __restrict__ bsum, int64_t nb) {
  __shared__ int64_t part[1024];
  const int t = threadIdx.x;
  const int64_t per = (nb + 1023) / 1024;
  const int64_t b = t * per, e = b + per < nb ? b + per : nb;
  int64_t s = 0;
  for (int64_t i = b; i < e; ++i) s += bsum[i];
  part[t] = s;
  __syncthreads();
  for (int o = 1; o < 1024; o <<= 1) {
    const int64_t v = t >= o ? part[t - o] : 0;
    __syncthreads();
    part[t] += v;
    __syncthreads();
  }
  int64_t run = t == 0 ? 0 : part[t - 1];
  for (int64_t i = b; i < e; ++i) {
    const int64_t c = bsum[i];
    bsum[i] = run;
    run += c;
  }
  if (t == 1023) bsum[nb] = part[1023];
}

__global__ __launch_bounds__(SCAN_TILE) void scan_add_kernel(int64_t* __restrict__ start,
                                                             const int64_t* __restrict__ bsum,
                                                             int64_t J, int64_t nb) {
  const int64_t i = (int64_t)blockIdx.x * SCAN_TILE + threadIdx.x;
  if (i < J) start[i] += bsum[blockIdx.x];
  if (i == 0) start[J] = bsum[nb];
}

void launch_scan(hipStream_t st, const int64_t* cnt, int64_t* start, int64_t* bsum, int64_t J) {
  const int64_t nb = J > 0 ? (J + SCAN_TILE - 1) / SCAN_TILE : 1;
  hipLaunchKernelGGL(scan_tiles_kernel, dim3((unsigned)nb), dim3(SCAN_TILE), 0, st, cnt, start,
                     bsum, J);
  hipLaunchKernelGGL(scan_bsum_kernel, dim3(1), dim3(1024), 0, st, bsum, nb);
  hipLaunchKernelGGL(scan_add_kernel, dim3((unsigned)nb), dim3(SCAN_TILE), 0, st, start, bsum, J,
                     nb);
}

// Y[i_j(e), :] += coef_d x_e rows[d, :].  A wavefront takes SPMM_IPW
// consecutive work items (chunks of <= CH entries of one distinct sampled
// fiber): one binary search over the compacted item starts for the first,
// then a linear advance.  The chunk's entries are read by the lanes in one
// go and broadcast one by one; lanes run over the R columns.
constexpr int SPMM_IPW = 4;
// Workgroups of 16 wavefronts, as many per CU (256 CUs, 160 KB of LDS
// each) as their HOT_LDS_BYTES of hot-row accumulators allow.
constexpr int SPMM_BLOCKS = 256 * (int)((size_t(160) << 10) / HOT_LDS_BYTES);

template <typename T, typename YT>
__global__ __launch_bounds__(1024) void spmm_kernel(FiberArgs a, const T* __restrict__ rows,
                                                   YT* __restrict__ Y) {
  extern __shared__ double hot_acc[];  // [nhot][R]
  const int lane = threadIdx.x & 63;
  const int R = a.R;
  for (int q = threadIdx.x; q < a.nhot * R; q += blockDim.x) hot_acc[q] = 0.0;
  __syncthreads();
  const int64_t nrep = a.rpos[a.J];
  const int64_t total = a.rstart[nrep];
  const int64_t nw = (int64_t)gridDim.x * (blockDim.x >> 6);
  const int32_t* __restrict__ ij = a.cols + (int64_t)a.j * a.nnz;
  for (int64_t c0 = ((int64_t)blockIdx.x * (blockDim.x >> 6) + (threadIdx.x >> 6)) * SPMM_IPW;
       c0 < total; c0 += nw * SPMM_IPW) {
    int64_t l = 0, r = nrep;  // last k with rstart[k] <= c0
    while (r - l > 1) {
      const int64_t m = (l + r) >> 1;
      if (a.rstart[m] <= c0) l = m; else r = m;
    }
    int64_t k = l;
    const int64_t c1 = c0 + SPMM_IPW < total ? c0 + SPMM_IPW : total;
    for (int64_t c = c0; c < c1; ++c) {
      while (k + 1 < nrep && a.rstart[k + 1] <= c) ++k;
      const int64_t d = a.rep[k];
      const int64_t e0 = a.lo[d] + (c - a.rstart[k]) * CH;
      const int64_t e1 = e0 + CH < a.hi[d] ? e0 + CH : a.hi[d];
      const double cd = a.coef[d];
      const T r0 = lane < R ? rows[d * R + lane] : T(0);
      const T r1 = lane + 64 < R ? rows[d * R + lane + 64] : T(0);
      // lane t holds entry e0 + t (CH == 64) and its row's hot slot, so
      // the loop below does no dependent loads
      const int64_t et = e0 + lane < e1 ? e0 + lane : e1 - 1;
      const double xv = cd * a.vals[et];
      const int iv = ij[et];
      const int hv = a.hot_slot[iv];
      const int n = (int)(e1 - e0);
      for (int t = 0; t < n; ++t) {
        // t is wave-uniform: read lane t's values straight into scalar
        // registers (no LDS permute on the loop's critical path)
        const double coef = __hiloint2double(__builtin_amdgcn_readlane(__double2hiint(xv), t),
                                             __builtin_amdgcn_readlane(__double2loint(xv), t));
        const int64_t i = __builtin_amdgcn_readlane(iv, t);
        const int hs = __builtin_amdgcn_readlane(hv, t);
        if (hs >= 0 && hs < a.nhot) {
          double* acc = hot_acc + hs * R;
          if (lane < R) atomicAdd(&acc[lane], coef * (double)r0);
          if (lane + 64 < R) atomicAdd(&acc[lane + 64], coef * (double)r1);
        } else {
          if (lane < R) atomicAdd(&Y[i * R + lane], (YT)(coef * (double)r0));
          if (lane + 64 < R) atomicAdd(&Y[i * R + lane + 64], (YT)(coef * (double)r1));
        }
      }
    }
  }
  __syncthreads();
  for (int q = threadIdx.x; q < a.nhot * R; q += blockDim.x) {
    const double v = hot_acc[q];
    if (v != 0.0) atomicAdd(&Y[(int64_t)a.hot_rows[q / R] * R + q % R], (YT)v);
  }
}

// Deterministic SpMM (fixed point).  Every term coef x_e rows[d][c] is
// rounded to an integer multiple of 2^-s and summed with int64 atomics,
// whose result does not depend on their order.  s is the largest exponent
// with B 2^s <= 2^62 for a bound B >= every row's sum of |terms| (the sum
// over all terms of |coef_d x_e| max_c |rows[d][c]|), so no partial sum
// overflows; each term then carries at most 2^-(s+1) <= B 2^-63 of
// rounding.  B is reduced in a fixed order: each wavefront walks the same
// work items in every run, each block sums its waves in order, and one
// thread sums the blocks in order.
constexpr int DET_BLOCKS = 1024;
constexpr int DET_IPW = 8;

template <typename T>
__global__ __launch_bounds__(256) void spmm_bound_kernel(FiberArgs a, const T* __restrict__ rows,
                                                         double* __restrict__ partial) {
  __shared__ double wsum[4];
  const int lane = threadIdx.x & 63;
  const int wave = threadIdx.x >> 6;
  const int R = a.R;
  const int64_t nrep = a.rpos[a.J];
  const int64_t total = a.rstart[nrep];
  const int64_t nw = (int64_t)gridDim.x * (blockDim.x >> 6);
  double acc = 0.0;
  for (int64_t c0 = ((int64_t)blockIdx.x * (blockDim.x >> 6) + wave) * DET_IPW; c0 < total;
       c0 += nw * DET_IPW) {
    int64_t l = 0, r = nrep;  // last k with rstart[k] <= c0
    while (r - l > 1) {
      const int64_t m = (l + r) >> 1;
      if (a.rstart[m] <= c0) l = m; else r = m;
    }
    int64_t k = l;
    const int64_t c1 = c0 + DET_IPW < total ? c0 + DET_IPW : total;
    for (int64_t c = c0; c < c1; ++c) {
      while (k + 1 < nrep && a.rstart[k + 1] <= c) ++k;
      const int64_t d = a.rep[k];
      const int64_t e = a.lo[d] + (c - a.rstart[k]) * CH + lane;
      double x = e < a.hi[d] ? fabs(a.vals[e]) : 0.0;
      double m = 0.0;
      for (int q = lane; q < R; q += 64) m = fmax(m, fabs((double)rows[d * R + q]));
#pragma unroll
      for (int o = 32; o > 0; o >>= 1) {
        x += __shfl_xor(x, o, 64);
        m = fmax(m, __shfl_xor(m, o, 64));
      }
      acc += fabs(a.coef[d]) * m * x;  // the same value in every lane
    }
  }
  if (lane == 0) wsum[wave] = acc;
  __syncthreads();
  if (threadIdx.x == 0) partial[blockIdx.x] = ((wsum[0] + wsum[1]) + wsum[2]) + wsum[3];
}

// scale[0] = 2^s, scale[1] = 2^-s from the block bounds.
__global__ void spmm_scale_kernel(const double* __restrict__ partial, int n,
                                  double* __restrict__ scale) {
  if (threadIdx.x != 0 || blockIdx.x != 0) return;
  double B = 0.0;
  for (int i = 0; i < n; ++i) B += partial[i];
  B *= 1.0 + 1e-9;  // the bound's own rounding
  int s = 0;
  if (B > 0.0) s = 62 - (ilogb(B) + 1);  // 2^(ilogb + 1) > B
  scale[0] = ldexp(1.0, s);
  scale[1] = ldexp(1.0, -s);
}

template <typename T>
__global__ __launch_bounds__(1024) void spmm_det_kernel(FiberArgs a, const T* __restrict__ rows,
                                                       const double* __restrict__ scale,
                                                       unsigned long long* __restrict__ Y) {
  extern __shared__ unsigned long long hot_q[];  // [nhot][R]
  const int lane = threadIdx.x & 63;
  const int R = a.R;
  const double sc = scale[0];
  for (int q = threadIdx.x; q < a.nhot * R; q += blockDim.x) hot_q[q] = 0ull;
  __syncthreads();
  const int64_t nrep = a.rpos[a.J];
  const int64_t total = a.rstart[nrep];
  const int64_t nw = (int64_t)gridDim.x * (blockDim.x >> 6);
  const int32_t* __restrict__ ij = a.cols + (int64_t)a.j * a.nnz;
  for (int64_t c0 = ((int64_t)blockIdx.x * (blockDim.x >> 6) + (threadIdx.x >> 6)) * SPMM_IPW;
       c0 < total; c0 += nw * SPMM_IPW) {
    int64_t l = 0, r = nrep;  // last k with rstart[k] <= c0
    while (r - l > 1) {
      const int64_t m = (l + r) >> 1;
      if (a.rstart[m] <= c0) l = m; else r = m;
    }
    int64_t k = l;
    const int64_t c1 = c0 + SPMM_IPW < total ? c0 + SPMM_IPW : total;
    for (int64_t c = c0; c < c1; ++c) {
      while (k + 1 < nrep && a.rstart[k + 1] <= c) ++k;
      const int64_t d = a.rep[k];
      const int64_t e0 = a.lo[d] + (c - a.rstart[k]) * CH;
      const int64_t e1 = e0 + CH < a.hi[d] ? e0 + CH : a.hi[d];
      const double cd = a.coef[d];
      const double r0 = lane < R ? (double)rows[d * R + lane] : 0.0;
      const double r1 = lane + 64 < R ? (double)rows[d * R + lane + 64] : 0.0;
      const int64_t et = e0 + lane < e1 ? e0 + lane : e1 - 1;
      const double xv = cd * a.vals[et];
      const int iv = ij[et];
      const int hv = a.hot_slot[iv];
      const int n = (int)(e1 - e0);
      for (int t = 0; t < n; ++t) {
        const double coef = __hiloint2double(__builtin_amdgcn_readlane(__double2hiint(xv), t),
                                             __builtin_amdgcn_readlane(__double2loint(xv), t));
        const int64_t i = __builtin_amdgcn_readlane(iv, t);
        const int hs = __builtin_amdgcn_readlane(hv, t);
        const unsigned long long q0 = (unsigned long long)(long long)rint(coef * r0 * sc);
        const unsigned long long q1 = (unsigned long long)(long long)rint(coef * r1 * sc);
        if (hs >= 0 && hs < a.nhot) {
          unsigned long long* acc = hot_q + hs * R;
          if (lane < R) atomicAdd(&acc[lane], q0);
          if (lane + 64 < R) atomicAdd(&acc[lane + 64], q1);
        } else {
          if (lane < R) atomicAdd(&Y[i * R + lane], q0);
          if (lane + 64 < R) atomicAdd(&Y[i * R + lane + 64], q1);
        }
      }
    }
  }
  __syncthreads();
  for (int q = threadIdx.x; q < a.nhot * R; q += blockDim.x) {
    const unsigned long long v = hot_q[q];
    if (v != 0ull) atomicAdd(&Y[(int64_t)a.hot_rows[q / R] * R + q % R], v);
  }
}

// The listed rows of Y from fixed point to float64, in place.
__global__ __launch_bounds__(256) void fix_to_double_kernel(double* __restrict__ Y, int R,
                                                            const int32_t* __restrict__ list,
                                                            const int64_t* __restrict__ count,
                                                            const double* __restrict__ scale) {
  const int lane = threadIdx.x & 63;
  const int64_t n = *count;
  const double inv = scale[1];
  const int64_t nw = (int64_t)gridDim.x * (blockDim.x >> 6);
  for (int64_t p = (int64_t)blockIdx.x * (blockDim.x >> 6) + (threadIdx.x >> 6); p < n; p += nw) {
    double* y = Y + (int64_t)list[p] * R;
    for (int c = lane; c < R; c += 64) {
      const long long v = (long long)__double_as_longlong(y[c]);
      y[c] = (double)v * inv;
    }
  }
}

// The rows of mode j that the sampled fibers' entries reach: mark[i] = 1.
// Traverses the compacted work items as the SpMM does, one item per
// wavefront (lane t takes the item's entry t).
constexpr int MARK_IPW = 8;

__global__ __launch_bounds__(256) void mark_rows_kernel(FiberArgs a, int32_t* __restrict__ mark) {
  const int lane = threadIdx.x & 63;
  const int64_t nrep = a.rpos[a.J];
  const int64_t total = a.rstart[nrep];
  const int64_t nw = (int64_t)gridDim.x * (blockDim.x >> 6);
  const int32_t* __restrict__ ij = a.cols + (int64_t)a.j * a.nnz;
  for (int64_t c0 = ((int64_t)blockIdx.x * (blockDim.x >> 6) + (threadIdx.x >> 6)) * MARK_IPW;
       c0 < total; c0 += nw * MARK_IPW) {
    int64_t l = 0, r = nrep;  // last k with rstart[k] <= c0
    while (r - l > 1) {
      const int64_t m = (l + r) >> 1;
      if (a.rstart[m] <= c0) l = m; else r = m;
    }
    int64_t k = l;
    const int64_t c1 = c0 + MARK_IPW < total ? c0 + MARK_IPW : total;
    for (int64_t c = c0; c < c1; ++c) {
      while (k + 1 < nrep && a.rstart[k + 1] <= c) ++k;
      const int64_t d = a.rep[k];
      const int64_t e = a.lo[d] + (c - a.rstart[k]) * CH + lane;
      if (e < a.hi[d] && lane < CH) mark[ij[e]] = 1;
    }
  }
}

// Marked rows per tile of SCAN_TILE rows.
__global__ __launch_bounds__(SCAN_TILE) void mark_count_kernel(const int32_t* __restrict__ mark,
                                                               int64_t n,
                                                               int64_t* __restrict__ bsum) {
  const int64_t i = (int64_t)blockIdx.x * SCAN_TILE + threadIdx.x;
  const int c = __syncthreads_count(i < n && mark[i] != 0);
  if (threadIdx.x == 0) bsum[blockIdx.x] = c;
}

// list[bsum[tile] + rank within the tile] = i for every marked row i (rows
// in increasing order); block 0 also copies the total to *count.
__global__ __launch_bounds__(SCAN_TILE) void mark_compact_kernel(const int32_t* __restrict__ mark,
                                                                 int64_t n, int64_t nb,
                                                                 const int64_t* __restrict__ bsum,
                                                                 int32_t* __restrict__ list,
                                                                 int64_t* __restrict__ count) {
  __shared__ int wsum[SCAN_TILE / 64];
  const int t = threadIdx.x, lane = t & 63, wave = t >> 6;
  const int64_t i = (int64_t)blockIdx.x * SCAN_TILE + t;
  const bool f = i < n && mark[i] != 0;
  const uint64_t b = __ballot(f);
  const int pre = __popcll(b & ((uint64_t(1) << lane) - 1));
  if (lane == 0) wsum[wave] = __popcll(b);
  __syncthreads();
  int off = 0;
  for (int q = 0; q < wave; ++q) off += wsum[q];
  if (f) list[bsum[blockIdx.x] + off + pre] = (int32_t)i;
  if (blockIdx.x == 0 && t == 0) *count = bsum[nb];
}

// Y[list[p], :] = 0 for p < *count; a wavefront per row.
template <typename YT>
__global__ __launch_bounds__(256) void zero_rows_kernel(YT* __restrict__ Y, int R,
                                                        const int32_t* __restrict__ list,
                                                        const int64_t* __restrict__ count) {
  const int lane = threadIdx.x & 63;
  const int64_t n = *count;
  const int64_t nw = (int64_t)gridDim.x * (blockDim.x >> 6);
  for (int64_t p = (int64_t)blockIdx.x * (blockDim.x >> 6) + (threadIdx.x >> 6); p < n; p += nw) {
    YT* y = Y + (int64_t)list[p] * R;
    for (int c = lane; c < R; c += 64) y[c] = YT(0);
  }
}

}  // namespace

hipError_t launch_lookup(hipStream_t st, const FiberArgs& a) {
  int64_t blocks = (a.J + 255) / 256;
  if (blocks > 4096) blocks = 4096;
  if (blocks < 1) blocks = 1;
  hipLaunchKernelGGL(lookup_kernel, dim3((unsigned)blocks), dim3(256), 0, st, a);
  int64_t hb = (a.H + 255) / 256;
  if (hb > 4096) hb = 4096;
  hipLaunchKernelGGL(merge_clear_kernel, dim3((unsigned)hb), dim3(256), 0, st, a);
  if (a.hWlo != nullptr) hipLaunchKernelGGL(w2_scale_kernel, dim3(1), dim3(1024), 0, st, a);
  hipLaunchKernelGGL(merge_insert_kernel, dim3((unsigned)blocks), dim3(256), 0, st, a);
  hipLaunchKernelGGL(merge_finish_kernel, dim3((unsigned)blocks), dim3(256), 0, st, a);
  launch_scan(st, a.cnt, a.start, a.bsum, a.J);
  launch_scan(st, a.rflag, a.rpos, a.bsum, a.J);
  int64_t cb = (a.J + 1 + 255) / 256;
  if (cb > 4096) cb = 4096;
  hipLaunchKernelGGL(compact_kernel, dim3((unsigned)cb), dim3(256), 0, st, a);
  if (a.expanded != nullptr)
    hipLaunchKernelGGL(expanded_kernel, dim3(1), dim3(1024), 0, st, a);
  return hipGetLastError();
}

size_t row_bsum_bytes(int64_t I) { return (size_t)((I + SCAN_TILE - 1) / SCAN_TILE + 2) * 8; }

hipError_t launch_rows(hipStream_t st, const FiberArgs& a, int64_t I, int32_t* mark, int64_t* bsum,
                       int32_t* list, int64_t* count, void* Y, bool y32) {
  const int64_t nb = I > 0 ? (I + SCAN_TILE - 1) / SCAN_TILE : 1;
  hipLaunchKernelGGL(fill_u32_kernel, dim3((unsigned)std::min<int64_t>(nb * 4, 8192)), dim3(256), 0,
                     st, (uint32_t*)mark, I);
  hipLaunchKernelGGL(mark_rows_kernel, dim3(2048), dim3(256), 0, st, a, mark);
  hipLaunchKernelGGL(mark_count_kernel, dim3((unsigned)nb), dim3(SCAN_TILE), 0, st, mark, I, bsum);
  hipLaunchKernelGGL(scan_bsum_kernel, dim3(1), dim3(1024), 0, st, bsum, nb);
  hipLaunchKernelGGL(mark_compact_kernel, dim3((unsigned)nb), dim3(SCAN_TILE), 0, st, mark, I, nb,
                     bsum, list, count);
  if (y32)
    hipLaunchKernelGGL(zero_rows_kernel<float>, dim3(2048), dim3(256), 0, st, (float*)Y, a.R, list,
                       count);
  else
    hipLaunchKernelGGL(zero_rows_kernel<double>, dim3(2048), dim3(256), 0, st, (double*)Y, a.R,
                       list, count);
  return hipGetLastError();
}

hipError_t launch_spmm_det(hipStream_t st, krps_precision p, const FiberArgs& a, const void* rows,
                           void* Y, const int32_t* list, const int64_t* count, double* det) {
  // det: DET_BLOCKS block bounds, then the scale pair
  double* scale = det + DET_BLOCKS;
  FiberArgs b = a;
  b.nhot = hot_rows_used(a.nhot, a.R);
  const size_t lds = (size_t)b.nhot * b.R * 8;
  if (p == KRPS_BF16X2) {
    hipLaunchKernelGGL(spmm_bound_kernel<float>, dim3(DET_BLOCKS), dim3(256), 0, st, a,
                       (const float*)rows, det);
    hipLaunchKernelGGL(spmm_scale_kernel, dim3(1), dim3(64), 0, st, det, DET_BLOCKS, scale);
    hipLaunchKernelGGL(spmm_det_kernel<float>, dim3(SPMM_BLOCKS), dim3(1024), lds, st, b,
                       (const float*)rows, scale, (unsigned long long*)Y);
  } else {
    hipLaunchKernelGGL(spmm_bound_kernel<double>, dim3(DET_BLOCKS), dim3(256), 0, st, a,
                       (const double*)rows, det);
    hipLaunchKernelGGL(spmm_scale_kernel, dim3(1), dim3(64), 0, st, det, DET_BLOCKS, scale);
    hipLaunchKernelGGL(spmm_det_kernel<double>, dim3(SPMM_BLOCKS), dim3(1024), lds, st, b,
                       (const double*)rows, scale, (unsigned long long*)Y);
  }
  hipLaunchKernelGGL(fix_to_double_kernel, dim3(2048), dim3(256), 0, st, (double*)Y, a.R, list,
                     count, scale);
  return hipGetLastError();
}

size_t spmm_det_bytes() { return (size_t)(DET_BLOCKS + 4) * 8; }

hipError_t launch_spmm(hipStream_t st, krps_precision p, const FiberArgs& a, const void* rows,
                       void* Y) {
  FiberArgs b = a;
  b.nhot = hot_rows_used(a.nhot, a.R);
  const size_t lds = (size_t)b.nhot * b.R * 8;
  // the split path's rows are float32 and its Y is float32 (half the
  // atomic traffic); the float64 and float32 paths form Y in float64
  if (p == KRPS_FP64)
    hipLaunchKernelGGL((spmm_kernel<double, double>), dim3(SPMM_BLOCKS), dim3(1024), lds, st, b,
                       (const double*)rows, (double*)Y);
  else
    hipLaunchKernelGGL((spmm_kernel<float, float>), dim3(SPMM_BLOCKS), dim3(1024), lds, st, b,
                       (const float*)rows, (float*)Y);
  return hipGetLastError();
}

// --------------------------------------------------------- fills and solve

namespace {

template <typename T>
__global__ void fill_kernel(T* __restrict__ p, int64_t n, T v) {
  for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n;
       i += (int64_t)gridDim.x * blockDim.x)
    p[i] = v;
}

// Y M^+ over the rows list[0 .. *count) (the rows of Y that the SpMM can
// reach; every other row of Y M^+ is zero), a persistent sweep of 64-row
// tiles.  The block's 256 threads
// are 16 row groups x 16 column groups; a thread accumulates 4 rows x
// RC/16 columns (columns tc + 16 j) in float64 registers, with K taken in
// chunks of 32 through LDS (Y tile [64][33], M^+ chunk [32][RC]).
// Pass 1 (sigma == nullptr) only keeps the per-column sums of squares of
// the products and reduces them per block into partial[block][c]; pass 2
// recomputes the products and writes U = (Y M^+)[:, c] / sigma[c],
// rounded once to the factor type.
constexpr int GT_ROWS = 64, GT_KC = 32;

template <typename T, int RC, typename YT>
__global__ __launch_bounds__(256) void gemm_colsum_kernel(const YT* __restrict__ Y,
                                                          const double* __restrict__ Mp,
                                                          T* __restrict__ out,
                                                          const int32_t* __restrict__ list,
                                                          const int64_t* __restrict__ count, int R,
                                                          double* __restrict__ partial,
                                                          const double* __restrict__ sigma) {
  constexpr int TCW = RC / 16;
  __shared__ int64_t rix[GT_ROWS];  // row of Y per tile row, -1 past the end
  __shared__ double Ys[GT_ROWS][GT_KC + 1];
  __shared__ double Ms[GT_KC][RC];
  __shared__ double red[16][RC];
  const int tc = threadIdx.x % 16;
  const int tr = threadIdx.x / 16;
  double inv[TCW], sq[TCW];
#pragma unroll
  for (int j = 0; j < TCW; ++j) {
    const int c = tc + 16 * j;
    inv[j] = (sigma != nullptr && c < R && sigma[c] > 0) ? 1.0 / sigma[c] : 0.0;
    sq[j] = 0.0;
  }
  const int64_t nrow = *count;
  const int64_t ntile = (nrow + GT_ROWS - 1) / GT_ROWS;
  for (int64_t tile = blockIdx.x; tile < ntile; tile += gridDim.x) {
    __syncthreads();
    if (threadIdx.x < GT_ROWS) {
      const int64_t p = tile * GT_ROWS + threadIdx.x;
      rix[threadIdx.x] = p < nrow ? (int64_t)list[p] : -1;
    }
    double acc[4][TCW];
#pragma unroll
    for (int i = 0; i < 4; ++i)
#pragma unroll
      for (int j = 0; j < TCW; ++j) acc[i][j] = 0.0;
    for (int k0 = 0; k0 < R; k0 += GT_KC) {
      __syncthreads();
      for (int e = threadIdx.x; e < GT_ROWS * GT_KC; e += 256) {
        const int i = e / GT_KC, kk = e % GT_KC;
        const int64_t r = rix[i];
        Ys[i][kk] = (r >= 0 && k0 + kk < R) ? (double)Y[r * R + k0 + kk] : 0.0;
      }
      for (int e = threadIdx.x; e < GT_KC * RC; e += 256) {
        const int kk = e / RC, c = e % RC;
        Ms[kk][c] = (k0 + kk < R && c < R) ? Mp[(int64_t)(k0 + kk) * R + c] : 0.0;
      }
      __syncthreads();
#pragma unroll 4
      for (int kk = 0; kk < GT_KC; ++kk) {
        double a[4], b[TCW];
#pragma unroll
        for (int i = 0; i < 4; ++i) a[i] = Ys[tr * 4 + i][kk];
#pragma unroll
        for (int j = 0; j < TCW; ++j) b[j] = Ms[kk][tc + 16 * j];
#pragma unroll
        for (int i = 0; i < 4; ++i)
#pragma unroll
          for (int j = 0; j < TCW; ++j) acc[i][j] += a[i] * b[j];
      }
    }
#pragma unroll
    for (int i = 0; i < 4; ++i) {
      const int64_t r = rix[tr * 4 + i];
      if (r < 0) continue;
#pragma unroll
      for (int j = 0; j < TCW; ++j) {
        const int c = tc + 16 * j;
        if (c >= R) continue;
        if (sigma == nullptr)
          sq[j] += acc[i][j] * acc[i][j];
        else
          out[r * R + c] = (T)(acc[i][j] * inv[j]);
      }
    }
  }
  if (sigma != nullptr) return;
  __syncthreads();
#pragma unroll
  for (int j = 0; j < TCW; ++j) red[tr][tc + 16 * j] = sq[j];
  __syncthreads();
  for (int c = threadIdx.x; c < R; c += 256) {
    double t = 0;
    for (int q = 0; q < 16; ++q) t += red[q][c];
    partial[(int64_t)blockIdx.x * R + c] = t;
  }
}

// Column sums of squares of a factor (for the initial normalisation).
template <typename T, int RB>
__global__ __launch_bounds__(256) void colsum_kernel(const T* __restrict__ U, int64_t I, int R,
                                                     double* __restrict__ partial) {
  __shared__ double red[256];
  constexpr int ROWS = 256 / RB;
  const int c = threadIdx.x % RB;
  const int rs = threadIdx.x / RB;
  double sq = 0;
  for (int64_t r = (int64_t)blockIdx.x * ROWS + rs; r < I; r += (int64_t)gridDim.x * ROWS)
    if (c < R) {
      const double v = (double)U[r * R + c];
      sq += v * v;
    }
  red[threadIdx.x] = sq;
  __syncthreads();
  if (rs == 0 && c < R) {
    double s = 0;
    for (int q = 0; q < ROWS; ++q) s += red[q * RB + c];
    partial[(int64_t)blockIdx.x * R + c] = s;
  }
}

// sigma[c] = sqrt(sum_b partial[b][c]); one block per column.
__global__ __launch_bounds__(256) void sigma_kernel(const double* __restrict__ partial, int nb,
                                                    int R, double* __restrict__ sigma) {
  __shared__ double red[256];
  const int c = blockIdx.x;
  double s = 0;
  for (int b = threadIdx.x; b < nb; b += blockDim.x) s += partial[(int64_t)b * R + c];
  red[threadIdx.x] = s;
  __syncthreads();
  for (int o = blockDim.x / 2; o > 0; o >>= 1) {
    if ((int)threadIdx.x < o) red[threadIdx.x] += red[threadIdx.x + o];
    __syncthreads();
  }
  if (threadIdx.x == 0) sigma[c] = sqrt(red[0]);
}

template <typename T>
__global__ void normalize_kernel(T* __restrict__ U, int64_t I, int R,
                                 const double* __restrict__ sigma) {
  const int64_t n = I * R;
  for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n;
       i += (int64_t)gridDim.x * blockDim.x) {
    const double s = sigma[i % R];
    U[i] = s > 0 ? (T)((double)U[i] / s) : T(0);
  }
}

}  // namespace

constexpr int SOLVE_BLOCKS = 2048;

size_t solve_partial_bytes(int R) { return (size_t)SOLVE_BLOCKS * R * 8; }

hipError_t launch_fill(hipStream_t st, krps_precision p, void* ptr, int64_t n) {
  if (n <= 0) return hipSuccess;
  int64_t blocks = (n + 255) / 256;
  if (blocks > 8192) blocks = 8192;
  if (p == KRPS_FP64)
    hipLaunchKernelGGL(fill_kernel<double>, dim3((unsigned)blocks), dim3(256), 0, st, (double*)ptr,
                       n, 0.0);
  else
    hipLaunchKernelGGL(fill_kernel<float>, dim3((unsigned)blocks), dim3(256), 0, st, (float*)ptr,
                       n, 0.0f);
  return hipGetLastError();
}

__global__ void set_u64_kernel(uint64_t* __restrict__ p, uint64_t v) { *p = v; }

hipError_t launch_set_u64(hipStream_t st, uint64_t* ptr, uint64_t v) {
  hipLaunchKernelGGL(set_u64_kernel, dim3(1), dim3(1), 0, st, ptr, v);
  return hipGetLastError();
}

hipError_t launch_fill_f64(hipStream_t st, double* ptr, int64_t n) {
  if (n <= 0) return hipSuccess;
  hipLaunchKernelGGL(fill_kernel<double>, dim3(64), dim3(256), 0, st, ptr, n, 0.0);
  return hipGetLastError();
}

template <typename T, int RC, typename YT>
static hipError_t run_gemm(hipStream_t st, const YT* Y, const double* Mp, void* out,
                           const int32_t* list, const int64_t* count, int R, double* partial,
                           double* sigma) {
  hipLaunchKernelGGL((gemm_colsum_kernel<T, RC, YT>), dim3(SOLVE_BLOCKS), dim3(256), 0, st, Y, Mp,
                     (T*)out, list, count, R, partial, (const double*)nullptr);
  hipLaunchKernelGGL(sigma_kernel, dim3(R), dim3(256), 0, st, partial, SOLVE_BLOCKS, R, sigma);
  hipLaunchKernelGGL((gemm_colsum_kernel<T, RC, YT>), dim3(SOLVE_BLOCKS), dim3(256), 0, st, Y, Mp,
                     (T*)out, list, count, R, partial, (const double*)sigma);
  return hipGetLastError();
}

// U = Y M^+ with its column norms sigma taken out: two passes over the
// listed rows of Y (norms, then the normalised write) so that U is rounded
// once; U is cleared first, since its other rows are zero.
hipError_t launch_solve_gemm(hipStream_t st, krps_precision p, const void* Y, const double* Mp,
                             void* U, int64_t I, const int32_t* list, const int64_t* count, int R,
                             double* partial, double* sigma) {
  hipError_t e = launch_fill(st, p, U, I * R);
  if (e != hipSuccess) return e;
  const double* Yd = (const double*)Y;
  const float* Yf = (const float*)Y;  // the split path's Y
  if (p == KRPS_FP64) {
    if (R <= 32) return run_gemm<double, 32>(st, Yd, Mp, U, list, count, R, partial, sigma);
    if (R <= 64) return run_gemm<double, 64>(st, Yd, Mp, U, list, count, R, partial, sigma);
    return run_gemm<double, 128>(st, Yd, Mp, U, list, count, R, partial, sigma);
  }
  if (p == KRPS_BF16X2) {
    if (R <= 32) return run_gemm<float, 32>(st, Yf, Mp, U, list, count, R, partial, sigma);
    if (R <= 64) return run_gemm<float, 64>(st, Yf, Mp, U, list, count, R, partial, sigma);
    return run_gemm<float, 128>(st, Yf, Mp, U, list, count, R, partial, sigma);
  }
  if (R <= 32) return run_gemm<float, 32>(st, Yd, Mp, U, list, count, R, partial, sigma);
  if (R <= 64) return run_gemm<float, 64>(st, Yd, Mp, U, list, count, R, partial, sigma);
  return run_gemm<float, 128>(st, Yd, Mp, U, list, count, R, partial, sigma);
}

hipError_t launch_colnorm(hipStream_t st, krps_precision p, const void* U, int64_t I, int R,
                          double* partial, double* sigma) {
  if (p == KRPS_FP64) {
    if (R <= 64)
      hipLaunchKernelGGL((colsum_kernel<double, 64>), dim3(SOLVE_BLOCKS), dim3(256), 0, st,
                         (const double*)U, I, R, partial);
    else
      hipLaunchKernelGGL((colsum_kernel<double, 128>), dim3(SOLVE_BLOCKS), dim3(256), 0, st,
                         (const double*)U, I, R, partial);
  } else {
    if (R <= 64)
      hipLaunchKernelGGL((colsum_kernel<float, 64>), dim3(SOLVE_BLOCKS), dim3(256), 0, st,
                         (const float*)U, I, R, partial);
    else
      hipLaunchKernelGGL((colsum_kernel<float, 128>), dim3(SOLVE_BLOCKS), dim3(256), 0, st,
                         (const float*)U, I, R, partial);
  }
  hipLaunchKernelGGL(sigma_kernel, dim3(R), dim3(256), 0, st, partial, SOLVE_BLOCKS, R, sigma);
  return hipGetLastError();
}

hipError_t launch_normalize(hipStream_t st, krps_precision p, void* U, int64_t I, int R,
                            const double* sigma) {
  int64_t blocks = (I * R + 255) / 256;
  if (blocks > 8192) blocks = 8192;
  if (p == KRPS_FP64)
    hipLaunchKernelGGL(normalize_kernel<double>, dim3((unsigned)blocks), dim3(256), 0, st,
                       (double*)U, I, R, sigma);
  else
    hipLaunchKernelGGL(normalize_kernel<float>, dim3((unsigned)blocks), dim3(256), 0, st,
                       (float*)U, I, R, sigma);
  return hipGetLastError();
}

// ---------------------------------------------------------------------- fit

namespace {

// <T, T~> partial sums, sum_e v_e sum_r sigma_r prod_k U_k[i_k(e), r]: a team
// of L lanes per stored entry, lane l taking columns l, l + L, ... so that each
// factor row is read as contiguous runs across the team.  The sum over r is
// linear, so every lane accumulates its own columns over all of its entries
// and the block reduces once at the end.
template <typename T, int L>
__global__ __launch_bounds__(256) void fit_inner_kernel(FitArgs a, double* __restrict__ partial) {
  __shared__ double red[256];
  double acc = 0;
  const int R = a.R;
  const int lane = threadIdx.x % L;
  const int64_t team = ((int64_t)blockIdx.x * blockDim.x + threadIdx.x) / L;
  const int64_t nteam = (int64_t)gridDim.x * blockDim.x / L;
  for (int64_t e = team; e < a.nnz; e += nteam) {
    int64_t row[KRPS_MAX_MODES];
#pragma unroll
    for (int k = 0; k < KRPS_MAX_MODES; ++k)
      row[k] = k < a.N ? (int64_t)a.cols[(int64_t)k * a.nnz + e] * R : 0;
    double part = 0;
    for (int c = lane; c < R; c += L) {
      double pr = a.sigma[c];
#pragma unroll
      for (int k = 0; k < KRPS_MAX_MODES; ++k)
        if (k < a.N) pr *= (double)((const T*)a.U[k])[row[k] + c];
      part += pr;
    }
    acc += a.vals[e] * part;
  }
  red[threadIdx.x] = acc;
  __syncthreads();
  for (int o = blockDim.x / 2; o > 0; o >>= 1) {
    if ((int)threadIdx.x < o) red[threadIdx.x] += red[threadIdx.x + o];
    __syncthreads();
  }
  if (threadIdx.x == 0) partial[blockIdx.x] = red[0];
}

// The same sum when R is a multiple of the 16-byte vector width VW (4
// floats or 2 doubles): lane l of an entry's team of L lanes reads columns
// VW l .. VW l + VW - 1 (then + VW L ...) of every row with one 16-byte
// load, and a wavefront serves 64 / L entries at once.
template <typename T, int L>
__global__ __launch_bounds__(256) void fit_inner_vec_kernel(FitArgs a,
                                                            double* __restrict__ partial) {
  constexpr int VW = 16 / (int)sizeof(T);
  typedef T vec __attribute__((ext_vector_type(VW)));
  __shared__ double red[256];
  double acc = 0;
  const int R = a.R;
  const int lane = threadIdx.x % L;
  const int64_t team = ((int64_t)blockIdx.x * blockDim.x + threadIdx.x) / L;
  const int64_t nteam = (int64_t)gridDim.x * blockDim.x / L;
  for (int64_t e = team; e < a.nnz; e += nteam) {
    int64_t row[KRPS_MAX_MODES];
#pragma unroll
    for (int k = 0; k < KRPS_MAX_MODES; ++k)
      row[k] = k < a.N ? (int64_t)a.cols[(int64_t)k * a.nnz + e] * R : 0;
    double part = 0;
    for (int c = lane * VW; c < R; c += L * VW) {
      double pr[VW];
#pragma unroll
      for (int v = 0; v < VW; ++v) pr[v] = a.sigma[c + v];
#pragma unroll
      for (int k = 0; k < KRPS_MAX_MODES; ++k)
        if (k < a.N) {
          const vec u = *(const vec*)((const T*)a.U[k] + row[k] + c);
#pragma unroll
          for (int v = 0; v < VW; ++v) pr[v] *= (double)u[v];
        }
#pragma unroll
      for (int v = 0; v < VW; ++v) part += pr[v];
    }
    acc += a.vals[e] * part;
  }
  red[threadIdx.x] = acc;
  __syncthreads();
  for (int o = blockDim.x / 2; o > 0; o >>= 1) {
    if ((int)threadIdx.x < o) red[threadIdx.x] += red[threadIdx.x + o];
    __syncthreads();
  }
  if (threadIdx.x == 0) partial[blockIdx.x] = red[0];
}

// out[0] = sum of partials (<T, T~>), out[1] = sigma^T ((*)_k G_k) sigma.
__global__ __launch_bounds__(256) void fit_final_kernel(FitArgs a, const double* __restrict__ partial,
                                                        int nb, double* __restrict__ out) {
  __shared__ double red[256];
  double s = 0;
  for (int b = threadIdx.x; b < nb; b += blockDim.x) s += partial[b];
  red[threadIdx.x] = s;
  __syncthreads();
  for (int o = blockDim.x / 2; o > 0; o >>= 1) {
    if ((int)threadIdx.x < o) red[threadIdx.x] += red[threadIdx.x + o];
    __syncthreads();
  }
  const double inner = red[0];
  __syncthreads();
  const int R = a.R;
  double m = 0;
  for (int i = threadIdx.x; i < R * R; i += blockDim.x) {
    double g = 1.0;
    for (int k = 0; k < a.N; ++k) g *= a.G[k][i];
    m += a.sigma[i / R] * g * a.sigma[i % R];
  }
  red[threadIdx.x] = m;
  __syncthreads();
  for (int o = blockDim.x / 2; o > 0; o >>= 1) {
    if ((int)threadIdx.x < o) red[threadIdx.x] += red[threadIdx.x + o];
    __syncthreads();
  }
  if (threadIdx.x == 0) {
    out[0] = inner;
    out[1] = red[0];
  }
}

}  // namespace

constexpr int FIT_BLOCKS = 2048;
size_t fit_partial_bytes() { return FIT_BLOCKS * 8; }

template <typename T>
static void launch_fit_vec(hipStream_t st, const FitArgs& a, double* partial) {
  constexpr int VW = 16 / (int)sizeof(T);
  // team width: the power of two >= R / VW, between 2 and a wavefront
  const int n = a.R / VW;
  const int L = n > 32 ? 64 : n > 16 ? 32 : n > 8 ? 16 : n > 4 ? 8 : n > 2 ? 4 : 2;
  const dim3 g(FIT_BLOCKS), b(256);
  switch (L) {
    case 64: hipLaunchKernelGGL((fit_inner_vec_kernel<T, 64>), g, b, 0, st, a, partial); break;
    case 32: hipLaunchKernelGGL((fit_inner_vec_kernel<T, 32>), g, b, 0, st, a, partial); break;
    case 16: hipLaunchKernelGGL((fit_inner_vec_kernel<T, 16>), g, b, 0, st, a, partial); break;
    case 8: hipLaunchKernelGGL((fit_inner_vec_kernel<T, 8>), g, b, 0, st, a, partial); break;
    case 4: hipLaunchKernelGGL((fit_inner_vec_kernel<T, 4>), g, b, 0, st, a, partial); break;
    default: hipLaunchKernelGGL((fit_inner_vec_kernel<T, 2>), g, b, 0, st, a, partial); break;
  }
}

hipError_t launch_fit(hipStream_t st, krps_precision p, const FitArgs& a, double* partial,
                      double* out) {
  // 16-byte row loads when every row starts on a 16-byte boundary (the
  // factors are allocated so; R a multiple of the vector width)
  bool vec_ok = true;
  for (int k = 0; k < a.N; ++k) vec_ok = vec_ok && ((uintptr_t)a.U[k] % 16 == 0);
  if (vec_ok && p == KRPS_FP64 && a.R % 2 == 0) {
    launch_fit_vec<double>(st, a, partial);
    hipLaunchKernelGGL(fit_final_kernel, dim3(1), dim3(256), 0, st, a, partial, FIT_BLOCKS, out);
    return hipGetLastError();
  }
  if (vec_ok && p != KRPS_FP64 && a.R % 4 == 0) {
    launch_fit_vec<float>(st, a, partial);
    hipLaunchKernelGGL(fit_final_kernel, dim3(1), dim3(256), 0, st, a, partial, FIT_BLOCKS, out);
    return hipGetLastError();
  }
  // team width: the power of two >= R, between 8 and a wavefront
  const int L = a.R > 32 ? 64 : a.R > 16 ? 32 : a.R > 8 ? 16 : 8;
  const dim3 g(FIT_BLOCKS), b(256);
  if (p == KRPS_FP64) {
    if (L == 64) hipLaunchKernelGGL((fit_inner_kernel<double, 64>), g, b, 0, st, a, partial);
    else if (L == 32) hipLaunchKernelGGL((fit_inner_kernel<double, 32>), g, b, 0, st, a, partial);
    else if (L == 16) hipLaunchKernelGGL((fit_inner_kernel<double, 16>), g, b, 0, st, a, partial);
    else hipLaunchKernelGGL((fit_inner_kernel<double, 8>), g, b, 0, st, a, partial);
  } else {
    if (L == 64) hipLaunchKernelGGL((fit_inner_kernel<float, 64>), g, b, 0, st, a, partial);
    else if (L == 32) hipLaunchKernelGGL((fit_inner_kernel<float, 32>), g, b, 0, st, a, partial);
    else if (L == 16) hipLaunchKernelGGL((fit_inner_kernel<float, 16>), g, b, 0, st, a, partial);
    else hipLaunchKernelGGL((fit_inner_kernel<float, 8>), g, b, 0, st, a, partial);
  }
  hipLaunchKernelGGL(fit_final_kernel, dim3(1), dim3(256), 0, st, a, partial, FIT_BLOCKS, out);
  return hipGetLastError();
}

}  // namespace krps

// ------------------------------------------------- generic sketched solve
//
// min_X || S A X - S B ||_F from the sampled rows a_d of A, their
// probabilities q_d and the sampled rows b_d of B (Section 2.1): with
// w_d = 1/sqrt(J q_d), X = M^+ Z, M = sum_d w_d^2 a_d a_d^T (R x R) and
// Z = sum_d w_d^2 a_d b_d^T (R x n).

namespace krps {

namespace {

constexpr int LS_CHUNKS = 64;  // J chunks of the Z partial sums

// SA[d] = w_d a_d and SBw[d] = w_d b_d in float64.
template <typename T>
__global__ void ls_scale_kernel(const T* __restrict__ rows, const T* __restrict__ sb,
                                const double* __restrict__ prob, int64_t J, int R, int64_t n,
                                double* __restrict__ SA, double* __restrict__ SBw) {
  const int64_t w = R + n;
  for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < J * w;
       i += (int64_t)gridDim.x * blockDim.x) {
    const int64_t d = i / w, c = i % w;
    const double wd = 1.0 / sqrt((double)J * prob[d]);
    if (c < R)
      SA[d * R + c] = wd * (double)rows[d * R + c];
    else
      SBw[d * n + (c - R)] = wd * (double)sb[d * n + (c - R)];
  }
}

// partial[chunk][r][c] = sum over the chunk's samples of SA[d][r] SBw[d][c].
__global__ void ls_atb_kernel(const double* __restrict__ SA, const double* __restrict__ SBw,
                              int64_t J, int R, int64_t n, double* __restrict__ partial) {
  const int64_t per = (J + LS_CHUNKS - 1) / LS_CHUNKS;
  const int chunk = blockIdx.y;
  const int64_t d0 = chunk * per, d1 = d0 + per < J ? d0 + per : J;
  for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < (int64_t)R * n;
       i += (int64_t)gridDim.x * blockDim.x) {
    const int64_t r = i / n, c = i % n;
    double acc = 0;
    for (int64_t d = d0; d < d1; ++d) acc += SA[d * R + r] * SBw[d * n + c];
    partial[(int64_t)chunk * R * n + i] = acc;
  }
}

// Z = the sum of the chunk partials, in chunk order.
__global__ void ls_z_kernel(const double* __restrict__ partial, int R, int64_t n,
                            double* __restrict__ Z) {
  for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < (int64_t)R * n;
       i += (int64_t)gridDim.x * blockDim.x) {
    double z = 0;
    for (int ch = 0; ch < LS_CHUNKS; ++ch) z += partial[(int64_t)ch * R * n + i];
    Z[i] = z;
  }
}

// X = M^+ Z.
__global__ void ls_mul_kernel(const double* __restrict__ Mp, const double* __restrict__ Z, int R,
                              int64_t n, double* __restrict__ X) {
  for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < (int64_t)R * n;
       i += (int64_t)gridDim.x * blockDim.x) {
    const int64_t r = i / n, c = i % n;
    double x = 0;
    for (int k = 0; k < R; ++k) x += Mp[(int64_t)r * R + k] * Z[(int64_t)k * n + c];
    X[i] = x;
  }
}

}  // namespace

size_t lstsq_partial_bytes(int R, int64_t n) { return (size_t)LS_CHUNKS * R * n * 8; }

hipError_t launch_ls_scale(hipStream_t st, krps_precision p, const void* rows, const void* sb,
                           const double* prob, int64_t J, int R, int64_t n, double* SA,
                           double* SBw) {
  int64_t blocks = (J * (R + n) + 255) / 256;
  if (blocks > 8192) blocks = 8192;
  if (blocks < 1) blocks = 1;
  if (p == KRPS_FP64)
    hipLaunchKernelGGL(ls_scale_kernel<double>, dim3((unsigned)blocks), dim3(256), 0, st,
                       (const double*)rows, (const double*)sb, prob, J, R, n, SA, SBw);
  else
    hipLaunchKernelGGL(ls_scale_kernel<float>, dim3((unsigned)blocks), dim3(256), 0, st,
                       (const float*)rows, (const float*)sb, prob, J, R, n, SA, SBw);
  return hipGetLastError();
}

hipError_t launch_ls_solve(hipStream_t st, const double* SA, const double* SBw, int64_t J, int R,
                           int64_t n, const double* Mp, double* partial, double* Z, double* X) {
  int64_t bx = ((int64_t)R * n + 255) / 256;
  if (bx > 1024) bx = 1024;
  hipLaunchKernelGGL(ls_atb_kernel, dim3((unsigned)bx, LS_CHUNKS), dim3(256), 0, st, SA, SBw, J, R,
                     n, partial);
  hipLaunchKernelGGL(ls_z_kernel, dim3((unsigned)bx), dim3(256), 0, st, partial, R, n, Z);
  hipLaunchKernelGGL(ls_mul_kernel, dim3((unsigned)bx), dim3(256), 0, st, Mp, Z, R, n, X);
  return hipGetLastError();
}

}  // namespace krps

// ------------------------------------------------- range-finder initialisation
//
// U_j = mat(T, j) S with a Gaussian sketch S that is generated, never
// stored, for the fibers that hold entries (the initialisation the paper
// uses for its sparsest tensor, Section 4.3).  Row of S for a fiber with
// other-mode indices (i_a, i_b, i_c, i_d) (increasing mode order, missing
// ones 0), column pair q: Philox4x64-10 (Salmon et al., SC'11) of counter
// (i_a | i_b << 32, i_c | i_d << 32, q, 0) under key (seed, j); the first
// two output words give open-interval uniforms ((x >> 11) + 0.5) 2^-53 and
// Box-Muller gives columns 2q (cosine) and 2q + 1 (sine).

namespace krps {

namespace {

// Entry z of column r of the sketch row (w0, w1).
__device__ __forceinline__ double sketch_entry(uint64_t w0, uint64_t w1, int r, uint64_t seed,
                                               int j) {
  uint64_t c[4] = {w0, w1, (uint64_t)(r >> 1), 0};
  philox4x64_10(c, seed, (uint64_t)j);
  const double u1 = u01_of_word(c[0]);
  const double u2 = u01_of_word(c[1]);
  const double rad = sqrt(-2.0 * log(u1));
  const double ang = 2.0 * M_PI * u2;
  return (r & 1) ? rad * sin(ang) : rad * cos(ang);
}

// Y[i_j(e), r] += x_e S[fiber(e), r]: one wavefront per stored entry at a
// time, lanes over the columns (r and r + 64).
__global__ __launch_bounds__(256) void range_finder_kernel(const int32_t* __restrict__ cols,
                                                           const double* __restrict__ vals,
                                                           int64_t nu, int N, int j, int R,
                                                           uint64_t seed, double* __restrict__ Y) {
  const int lane = threadIdx.x & 63;
  const int64_t nw = ((int64_t)gridDim.x * blockDim.x) >> 6;
  for (int64_t e = ((int64_t)blockIdx.x * blockDim.x + threadIdx.x) >> 6; e < nu; e += nw) {
    uint64_t w[4] = {0, 0, 0, 0};
    int m = 0;
    for (int k = 0; k < N; ++k)
      if (k != j) w[m++] = (uint64_t)(uint32_t)cols[(int64_t)k * nu + e];
    const uint64_t w0 = w[0] | (w[1] << 32), w1 = w[2] | (w[3] << 32);
    const int64_t i = cols[(int64_t)j * nu + e];
    const double x = vals[e];
    if (lane < R) atomicAdd(&Y[i * R + lane], x * sketch_entry(w0, w1, lane, seed, j));
    if (lane + 64 < R)
      atomicAdd(&Y[i * R + lane + 64], x * sketch_entry(w0, w1, lane + 64, seed, j));
  }
}

template <typename T>
__global__ void store_factor_kernel(const double* __restrict__ Y, T* __restrict__ U, int64_t n) {
  for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n;
       i += (int64_t)gridDim.x * blockDim.x)
    U[i] = (T)Y[i];
}

}  // namespace

hipError_t launch_range_finder(hipStream_t st, krps_precision p, const int32_t* cols,
                               const double* vals, int64_t nu, int N, int j, int R, uint64_t seed,
                               int64_t I, double* Y, void* U) {
  hipError_t e = launch_fill_f64(st, Y, I * R);
  if (e != hipSuccess) return e;
  hipLaunchKernelGGL(range_finder_kernel, dim3(4096), dim3(256), 0, st, cols, vals, nu, N, j, R,
                     seed, Y);
  int64_t blocks = (I * R + 255) / 256;
  if (blocks > 8192) blocks = 8192;
  if (p == KRPS_FP64)
    hipLaunchKernelGGL(store_factor_kernel<double>, dim3((unsigned)blocks), dim3(256), 0, st, Y,
                       (double*)U, I * R);
  else
    hipLaunchKernelGGL(store_factor_kernel<float>, dim3((unsigned)blocks), dim3(256), 0, st, Y,
                       (float*)U, I * R);
  return hipGetLastError();
}

}  // namespace krps

// ------------------------------------------------------ exact MTTKRP
//
// The exact ALS step of mode j (Algorithm 6 with the full least-squares
// problem): Y = mat(T, j) (U_N (.) ... (.) U_1 without U_j), i.e.
// Y[i_j(e), :] += x_e (*)_{k != j} U_k[i_k(e), :] over every stored entry.

namespace krps {
namespace {

// mark[i_j(e)] = 1 for every stored entry.
__global__ __launch_bounds__(256) void mark_all_kernel(const int32_t* __restrict__ ij, int64_t n,
                                                       int32_t* __restrict__ mark) {
  for (int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; e < n;
       e += (int64_t)gridDim.x * blockDim.x)
    mark[ij[e]] = 1;
}

// A wavefront takes MTTKRP_CHUNK consecutive entries of mode j's copy
// (sorted by the other modes' indices, so the entries of a fiber are
// consecutive and share their Khatri-Rao row, formed once per fiber);
// lanes run over the R columns (two per lane above 64).  The rows of mode
// j with the most entries are accumulated per workgroup in LDS, as in the
// sampled SpMM.
constexpr int MTTKRP_CHUNK = 256;

template <typename T>
__global__ __launch_bounds__(1024) void mttkrp_kernel(MttkrpArgs a, double* __restrict__ Y) {
  extern __shared__ double hot_acc[];  // [nhot][R]
  const int lane = threadIdx.x & 63;
  const int R = a.R;
  for (int q = threadIdx.x; q < a.nhot * R; q += blockDim.x) hot_acc[q] = 0.0;
  __syncthreads();
  const int32_t* __restrict__ ij = a.cols + (int64_t)a.j * a.nnz;
  const int64_t nw = (int64_t)gridDim.x * (blockDim.x >> 6);
  for (int64_t e0 = ((int64_t)blockIdx.x * (blockDim.x >> 6) + (threadIdx.x >> 6)) * MTTKRP_CHUNK;
       e0 < a.nnz; e0 += nw * MTTKRP_CHUNK) {
    const int64_t e1 = e0 + MTTKRP_CHUNK < a.nnz ? e0 + MTTKRP_CHUNK : a.nnz;
    double k0 = 0.0, k1 = 0.0;  // the current fiber's Khatri-Rao row (columns lane, lane + 64)
    int32_t prev[KRPS_MAX_MODES];
#pragma unroll
    for (int k = 0; k < KRPS_MAX_MODES; ++k) prev[k] = -1;
    for (int64_t e = e0; e < e1; ++e) {
      bool same = true;
#pragma unroll
      for (int k = 0; k < KRPS_MAX_MODES; ++k)
        if (k < a.N && k != a.j) {
          const int32_t c = a.cols[(int64_t)k * a.nnz + e];
          same = same && c == prev[k];
          prev[k] = c;
        }
      if (!same) {
        k0 = 1.0;
        k1 = 1.0;
#pragma unroll
        for (int k = 0; k < KRPS_MAX_MODES; ++k)
          if (k < a.N && k != a.j) {
            const T* u = (const T*)a.U[k] + (int64_t)prev[k] * R;
            if (lane < R) k0 *= (double)u[lane];
            if (lane + 64 < R) k1 *= (double)u[lane + 64];
          }
      }
      const double x = a.vals[e];
      const int32_t i = ij[e];
      const int hs = a.hot_slot[i];
      if (hs >= 0 && hs < a.nhot) {
        double* acc = hot_acc + hs * R;
        if (lane < R) atomicAdd(&acc[lane], x * k0);
        if (lane + 64 < R) atomicAdd(&acc[lane + 64], x * k1);
      } else {
        if (lane < R) atomicAdd(&Y[(int64_t)i * R + lane], x * k0);
        if (lane + 64 < R) atomicAdd(&Y[(int64_t)i * R + lane + 64], x * k1);
      }
    }
  }
  __syncthreads();
  for (int q = threadIdx.x; q < a.nhot * R; q += blockDim.x) {
    const double v = hot_acc[q];
    if (v != 0.0) atomicAdd(&Y[(int64_t)a.hot_rows[q / R] * R + q % R], v);
  }
}

}  // namespace

hipError_t launch_mttkrp(hipStream_t st, krps_precision p, const MttkrpArgs& a, int64_t I,
                         int32_t* mark, int64_t* bsum, int32_t* list, int64_t* count, double* Y) {
  const int64_t nb = I > 0 ? (I + SCAN_TILE - 1) / SCAN_TILE : 1;
  const int32_t* ij = a.cols + (int64_t)a.j * a.nnz;
  hipLaunchKernelGGL(fill_u32_kernel, dim3((unsigned)std::min<int64_t>(nb * 4, 8192)), dim3(256), 0,
                     st, (uint32_t*)mark, I);
  hipLaunchKernelGGL(mark_all_kernel, dim3(4096), dim3(256), 0, st, ij, a.nnz, mark);
  hipLaunchKernelGGL(mark_count_kernel, dim3((unsigned)nb), dim3(SCAN_TILE), 0, st, mark, I, bsum);
  hipLaunchKernelGGL(scan_bsum_kernel, dim3(1), dim3(1024), 0, st, bsum, nb);
  hipLaunchKernelGGL(mark_compact_kernel, dim3((unsigned)nb), dim3(SCAN_TILE), 0, st, mark, I, nb,
                     bsum, list, count);
  hipLaunchKernelGGL(zero_rows_kernel<double>, dim3(2048), dim3(256), 0, st, Y, a.R, list, count);
  MttkrpArgs b = a;
  b.nhot = hot_rows_used(a.nhot, a.R);
  const size_t lds = (size_t)b.nhot * b.R * 8;
  if (p == KRPS_FP64)
    hipLaunchKernelGGL(mttkrp_kernel<double>, dim3(SPMM_BLOCKS), dim3(1024), lds, st, b, Y);
  else
    hipLaunchKernelGGL(mttkrp_kernel<float>, dim3(SPMM_BLOCKS), dim3(1024), lds, st, b, Y);
  return hipGetLastError();
}

}  // namespace krps
