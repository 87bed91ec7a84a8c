// finalize.hip -- from the elimination's column chunks to the solve layout:
// canonical CSC of F (label order, rows ascending), its CSR transpose (rows
// ordered by column, so every row sum has a fixed order), rows grouped by
// elimination level for the triangular solves, D^+, FP32 copies, statistics.
#include "device.hpp"
#include "internal.hpp"

namespace parac {

static inline unsigned nblk(int64_t n, int t) { return (unsigned)((n + t - 1) / t > 0 ? (n + t - 1) / t : 1); }

// lanes per column in the column copies below, so that a column's reads and
// writes are contiguous
constexpr int kColLanes = 16;

__global__ void k_compact_csc(int64_t ntot, const int64_t *__restrict__ colstart,
                              const int32_t *__restrict__ colcnt, const int32_t *__restrict__ frow,
                              const double *__restrict__ fval, const int64_t *__restrict__ colptr,
                              int32_t *rowind, double *val) {
  const int64_t t = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  const int64_t k = t / kColLanes;
  const int q = (int)(t % kColLanes);
  if (k >= ntot) return;
  const int64_t s = colstart[k], o = colptr[k];
  const int c = colcnt[k];
  for (int e = q; e < c; e += kColLanes) {
    rowind[o + e] = frow[s + e];
    val[o + e] = fval[s + e];
  }
}

hipError_t launch_compact_csc(int64_t ntot, const int64_t *colstart, const int32_t *colcnt,
                              const int32_t *frow, const double *fval, const int64_t *colptr,
                              int32_t *rowind, double *val, hipStream_t s) {
  hipLaunchKernelGGL(k_compact_csc, dim3(nblk(ntot * kColLanes, 256)), dim3(256), 0, s, ntot,
                     colstart, colcnt, frow, fval, colptr, rowind, val);
  return hipGetLastError();
}

__global__ void k_row_count(int64_t nnz, const int32_t *__restrict__ rowind, int32_t *rowcnt) {
  int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (e < nnz) atomicAdd(&rowcnt[rowind[e]], 1);
}

hipError_t launch_row_count(int64_t nnz, const int32_t *rowind, int32_t *rowcnt, hipStream_t s) {
  if (nnz == 0) return hipSuccess;
  hipLaunchKernelGGL(k_row_count, dim3(nblk(nnz, 256)), dim3(256), 0, s, nnz, rowind, rowcnt);
  return hipGetLastError();
}

__global__ void k_transpose(int64_t ntot, const int64_t *__restrict__ colptr,
                            const int32_t *__restrict__ rowind, const double *__restrict__ val,
                            const int64_t *__restrict__ rowptr_f, int32_t *cursor,
                            int32_t *colind_f, double *val_f) {
  // the order within a row is arbitrary here; k_sort_rows sorts it
  const int64_t t = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  const int64_t k = t / kColLanes;
  const int q = (int)(t % kColLanes);
  if (k >= ntot) return;
  for (int64_t e = colptr[k] + q; e < colptr[k + 1]; e += kColLanes) {
    int32_t i = rowind[e];
    int64_t pos = rowptr_f[i] + atomicAdd(&cursor[i], 1);
    colind_f[pos] = (int32_t)k;
    val_f[pos] = val[e];
  }
}

hipError_t launch_transpose(int64_t ntot, const int64_t *colptr, const int32_t *rowind,
                            const double *val, const int64_t *rowptr_f, int32_t *cursor,
                            int32_t *colind_f, double *val_f, hipStream_t s) {
  hipLaunchKernelGGL(k_transpose, dim3(nblk(ntot * kColLanes, 256)), dim3(256), 0, s, ntot, colptr,
                     rowind, val, rowptr_f, cursor, colind_f, val_f);
  return hipGetLastError();
}

// rows of up to 64 entries: insertion sort by column, one lane per row; the
// longer ones are listed for the wave-per-row pass
__global__ void k_sort_rows(int64_t ntot, const int64_t *__restrict__ rowptr_f, int32_t *colind_f,
                            double *val_f, int32_t *long_rows, int32_t *n_long) {
  int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= ntot) return;
  int64_t b = rowptr_f[i], e = rowptr_f[i + 1];
  if (e - b > 64) {
    long_rows[atomicAdd(n_long, 1)] = (int32_t)i;
    return;
  }
  for (int64_t p = b + 1; p < e; ++p) {
    int32_t c = colind_f[p];
    double v = val_f[p];
    int64_t q = p - 1;
    while (q >= b && colind_f[q] > c) {
      colind_f[q + 1] = colind_f[q];
      val_f[q + 1] = val_f[q];
      --q;
    }
    colind_f[q + 1] = c;
    val_f[q + 1] = v;
  }
}

// long rows: one wave per row, stable radix sort on the column label bits,
// ping-ponging with the scratch arrays tmp_c / tmp_v at the row's own offsets
__global__ __launch_bounds__(256) void k_sort_long_rows(const int64_t *__restrict__ rowptr_f,
                                                        int32_t *colind_f, double *val_f,
                                                        const int32_t *__restrict__ long_rows,
                                                        const int32_t *__restrict__ n_long,
                                                        int32_t *tmp_c, double *tmp_v,
                                                        int nbits) {
  __shared__ int hist[4][256];
  int *h = hist[threadIdx.x >> 6];
  const int l = lane();
  const int wid = (int)(((int64_t)blockIdx.x * blockDim.x + threadIdx.x) >> 6);
  const int nw = (int)((gridDim.x * (int64_t)blockDim.x) >> 6);
  const int cnt = *n_long;
  int shifts[4], np = 0;
  for (int b = 0; b < nbits && np < 4; b += 8) shifts[np++] = b;
  for (int r = wid; r < cnt; r += nw) {
    const int32_t row = long_rows[r];
    const int64_t b = rowptr_f[row];
    const int len = (int)(rowptr_f[row + 1] - b);
    const bool in_a = wave_radix_sort<int32_t, double>(colind_f + b, val_f + b, tmp_c + b,
                                                       tmp_v + b, len, shifts, np, h);
    if (!in_a) {
      for (int i = l; i < len; i += kWave) {
        colind_f[b + i] = tmp_c[b + i];
        val_f[b + i] = tmp_v[b + i];
      }
    }
    fence_wave_local();
  }
}

hipError_t launch_sort_rows(int64_t ntot, const int64_t *rowptr_f, int32_t *colind_f,
                            double *val_f, int32_t *long_rows, int32_t *n_long, hipStream_t s) {
  hipLaunchKernelGGL(k_sort_rows, dim3(nblk(ntot, 256)), dim3(256), 0, s, ntot, rowptr_f, colind_f,
                     val_f, long_rows, n_long);
  return hipGetLastError();
}

hipError_t launch_sort_long_rows(const int64_t *rowptr_f, int32_t *colind_f, double *val_f,
                                 const int32_t *long_rows, const int32_t *n_long, int32_t *tmp_c,
                                 double *tmp_v, int64_t ntot, hipStream_t s) {
  int nbits = 0;
  while (nbits < 31 && ((int64_t)1 << nbits) < ntot) ++nbits;
  hipLaunchKernelGGL(k_sort_long_rows, dim3(1024), dim3(256), 0, s, rowptr_f, colind_f, val_f,
                     long_rows, n_long, tmp_c, tmp_v, nbits);
  return hipGetLastError();
}

// --------------------------------------------------------------------------
// rows grouped by level; one atomic per wave and distinct level
// --------------------------------------------------------------------------
__device__ __forceinline__ int wave_aggregate_add(bool valid, int key, int32_t *ctr, int &mine) {
  uint64_t act = __ballot(valid);
  mine = 0;
  while (act) {
    const int leader = __ffsll((long long)act) - 1;
    const int kl = shfl(key, leader);
    const uint64_t peers = __ballot(valid && key == kl) & act;
    int base = 0;
    if (lane() == leader) base = atomicAdd(&ctr[kl], __popcll(peers));
    base = shfl(base, leader);
    if ((peers >> lane()) & 1ull) mine = base + __popcll(peers & lanemask_lt());
    act &= ~peers;
  }
  return 0;
}

// Rows are grouped by level with block-local histograms in LDS (levels below
// kHist; the heavily populated low levels then cost one global atomic per
// block instead of one per row); rarer higher levels use wave-aggregated
// global atomics.  Positions within a level are arbitrary: rows of one level
// are independent.
constexpr int kHist = 4096;
constexpr int kLvT = 1024, kLvItems = 4;

__global__ __launch_bounds__(kLvT) void k_level_count(int64_t nrows, const int32_t *__restrict__ lev,
                                                      int32_t *lcount) {
  __shared__ int32_t h[kHist];
  for (int t = threadIdx.x; t < kHist; t += kLvT) h[t] = 0;
  __syncthreads();
  const int64_t base = (int64_t)blockIdx.x * kLvT * kLvItems;
  for (int k = 0; k < kLvItems; ++k) {
    const int64_t i = base + threadIdx.x + (int64_t)k * kLvT;
    const bool valid = i < nrows;
    const int L = valid ? lev[i] : 0;
    if (valid && L < kHist) atomicAdd(&h[L], 1);
    int mine;
    wave_aggregate_add(valid && L >= kHist, L, lcount, mine);
  }
  __syncthreads();
  for (int t = threadIdx.x; t < kHist; t += kLvT)
    if (h[t]) atomicAdd(&lcount[t], h[t]);
}

hipError_t launch_level_count(int64_t nrows, const int32_t *lev, int32_t *lcount, hipStream_t s) {
  hipLaunchKernelGGL(k_level_count, dim3(nblk(nrows, kLvT * kLvItems)), dim3(kLvT), 0, s, nrows, lev,
                     lcount);
  return hipGetLastError();
}

__global__ __launch_bounds__(kLvT) void k_level_place(int64_t nrows, const int32_t *__restrict__ lev,
                                                      const int64_t *__restrict__ lptr,
                                                      int32_t *lcursor, int32_t *order) {
  __shared__ int32_t h[kHist];
  __shared__ int32_t bs[kHist];
  for (int t = threadIdx.x; t < kHist; t += kLvT) h[t] = 0;
  __syncthreads();
  const int64_t base = (int64_t)blockIdx.x * kLvT * kLvItems;
  int rank[kLvItems], Ls[kLvItems];
  for (int k = 0; k < kLvItems; ++k) {
    const int64_t i = base + threadIdx.x + (int64_t)k * kLvT;
    const bool valid = i < nrows;
    Ls[k] = valid ? lev[i] : -1;
    rank[k] = (valid && Ls[k] < kHist) ? atomicAdd(&h[Ls[k]], 1) : 0;
  }
  __syncthreads();
  for (int t = threadIdx.x; t < kHist; t += kLvT)
    if (h[t]) bs[t] = atomicAdd(&lcursor[t], h[t]);
  __syncthreads();
  for (int k = 0; k < kLvItems; ++k) {
    const int64_t i = base + threadIdx.x + (int64_t)k * kLvT;
    const int L = Ls[k];
    const bool hi = L >= kHist;
    int mine;
    wave_aggregate_add(hi, hi ? L : 0, lcursor, mine);
    if (L >= 0 && !hi) order[lptr[L] + bs[L] + rank[k]] = (int32_t)i;
    if (hi) order[lptr[L] + mine] = (int32_t)i;
  }
}

hipError_t launch_level_place(int64_t nrows, const int32_t *lev, const int64_t *lptr,
                              int32_t *lcursor, int32_t *order, hipStream_t s) {
  hipLaunchKernelGGL(k_level_place, dim3(nblk(nrows, kLvT * kLvItems)), dim3(kLvT), 0, s, nrows, lev,
                     lptr, lcursor, order);
  return hipGetLastError();
}

__global__ void k_cast32(int64_t n, const double *__restrict__ a, float *b) {
  int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i < n) b[i] = (float)a[i];
}

hipError_t launch_cast32(int64_t n, const double *a, float *b, hipStream_t s) {
  if (n == 0) return hipSuccess;
  hipLaunchKernelGGL(k_cast32, dim3(nblk(n, 256)), dim3(256), 0, s, n, a, b);
  return hipGetLastError();
}

// out: [0] max gather, [1] max d_k, [2] sum max(d_k - 1, 0), [3] max level,
//      [4] zero pivots -- reduced per block in LDS, one atomic per block
__global__ __launch_bounds__(1024) void k_max_stats(int64_t ntot, const int64_t *__restrict__ uptr,
                                                    const int32_t *__restrict__ fill_cnt,
                                                    const int32_t *__restrict__ colcnt,
                                                    const int32_t *__restrict__ lev,
                                                    unsigned long long *out) {
  __shared__ unsigned long long sh[5][16];
  unsigned long long g = 0, d = 0, f = 0, L = 0, z = 0;
  for (int64_t k = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; k < ntot;
       k += (int64_t)gridDim.x * blockDim.x) {
    unsigned long long gk = (unsigned long long)(uptr[k + 1] - uptr[k] + fill_cnt[k]);
    unsigned long long dk = (unsigned long long)colcnt[k];
    unsigned long long Lk = (unsigned long long)lev[k];
    g = gk > g ? gk : g;
    d = dk > d ? dk : d;
    L = Lk > L ? Lk : L;
    f += (unsigned long long)fill_cnt[k];  // fill records addressed to k
    z += colcnt[k] == 0 ? 1 : 0;
  }
  for (int o = 32; o >= 1; o >>= 1) {
    unsigned long long g2 = __shfl_xor(g, o, kWave), d2 = __shfl_xor(d, o, kWave);
    unsigned long long L2 = __shfl_xor(L, o, kWave);
    g = g2 > g ? g2 : g;
    d = d2 > d ? d2 : d;
    L = L2 > L ? L2 : L;
    f += __shfl_xor(f, o, kWave);
    z += __shfl_xor(z, o, kWave);
  }
  const int w = threadIdx.x >> 6;
  if (lane() == 0) {
    sh[0][w] = g;
    sh[1][w] = d;
    sh[2][w] = f;
    sh[3][w] = L;
    sh[4][w] = z;
  }
  __syncthreads();
  if (threadIdx.x == 0) {
    const int nw = blockDim.x >> 6;
    for (int i = 1; i < nw; ++i) {
      g = sh[0][i] > g ? sh[0][i] : g;
      d = sh[1][i] > d ? sh[1][i] : d;
      f += sh[2][i];
      L = sh[3][i] > L ? sh[3][i] : L;
      z += sh[4][i];
    }
    atomicMax(&out[0], g);
    atomicMax(&out[1], d);
    atomicAdd(&out[2], f);
    atomicMax(&out[3], L);
    atomicAdd(&out[4], z);
  }
}

hipError_t launch_max_stats(int64_t ntot, const int64_t *uptr, const int32_t *fill_cnt,
                            const int32_t *colcnt, const int32_t *lev, unsigned long long *out,
                            hipStream_t s) {
  const unsigned blocks = nblk(ntot, 1024) < 512 ? nblk(ntot, 1024) : 512;
  hipLaunchKernelGGL(k_max_stats, dim3(blocks), dim3(1024), 0, s, ntot, uptr, fill_cnt, colcnt, lev,
                     out);
  return hipGetLastError();
}

__global__ void k_fill_u64(uint64_t *p, uint64_t v, int64_t n) {
  int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i < n) p[i] = v;
}
__global__ void k_fill_u32(uint32_t *p, uint32_t v, int64_t n) {
  int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i < n) p[i] = v;
}

hipError_t launch_fill_u64(uint64_t *p, uint64_t v, int64_t n, hipStream_t s) {
  if (n == 0) return hipSuccess;
  hipLaunchKernelGGL(k_fill_u64, dim3(nblk(n, 256)), dim3(256), 0, s, p, v, n);
  return hipGetLastError();
}
hipError_t launch_fill_u32(uint32_t *p, uint32_t v, int64_t n, hipStream_t s) {
  if (n == 0) return hipSuccess;
  hipLaunchKernelGGL(k_fill_u32, dim3(nblk(n, 256)), dim3(256), 0, s, p, v, n);
  return hipGetLastError();
}

}  // namespace parac
