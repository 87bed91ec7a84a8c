// solve.hip -- the preconditioner apply z = P^T F^-T D^+ F^-1 P r and the
// kernels of preconditioned conjugate gradients.
//
// Both triangular solves follow the elimination levels: the rows of one
// level depend only on rows of lower levels (forward) or higher levels
// (backward), so a level is solved in parallel once its predecessors are.
#include <float.h>

#include "device.hpp"
#include "internal.hpp"

namespace parac {

// ---------------------------------------------------------------------------
// Layout of the preconditioner apply.  The factor is stored twice in level
// order: the rows of F for the forward sweep and its columns (without the
// ground row) for the backward sweep; position p of either copy is the row
// order[p].  Rows of one level are independent.  Per direction, the
// positions of each level are listed by row class, and the sweep's units
// (ready.hip) are cut from these lists.
// ---------------------------------------------------------------------------
__global__ void k_class_count(int64_t n, const int32_t *__restrict__ order,
                              const int32_t *__restrict__ lev, const int64_t *__restrict__ ptr,
                              int32_t *ccount) {
  const int64_t p = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  const bool valid = p < n;
  const int key = valid ? lev[order[p]] * kRowClasses + row_class(ptr[p + 1] - ptr[p]) : 0;
  // one atomic per distinct key of the wave
  uint64_t act = __ballot(valid);
  while (act) {
    const int leader = __ffsll((long long)act) - 1;
    const int kl = __shfl(key, leader, kWave);
    const uint64_t peers = __ballot(valid && key == kl) & act;
    if (lane() == leader) atomicAdd(&ccount[kl], __popcll(peers));
    act &= ~peers;
  }
}

__global__ void k_class_place(int64_t n, const int32_t *__restrict__ order,
                              const int32_t *__restrict__ lev, const int64_t *__restrict__ ptr,
                              const int64_t *__restrict__ cbase, int32_t *ccursor, int32_t *list) {
  const int64_t p = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  const bool valid = p < n;
  const int key = valid ? lev[order[p]] * kRowClasses + row_class(ptr[p + 1] - ptr[p]) : 0;
  uint64_t act = __ballot(valid);
  while (act) {
    const int leader = __ffsll((long long)act) - 1;
    const int kl = __shfl(key, leader, kWave);
    const uint64_t peers = __ballot(valid && key == kl) & act;
    int base = 0;
    if (lane() == leader) base = atomicAdd(&ccursor[kl], __popcll(peers));
    base = __shfl(base, leader, kWave);
    if ((peers >> lane()) & 1ull)
      list[cbase[kl] + base + __popcll(peers & lanemask_lt())] = (int32_t)p;
    act &= ~peers;
  }
}

hipError_t launch_class_count(int64_t n, const int32_t *order, const int32_t *lev,
                              const int64_t *ptr, int32_t *ccount, hipStream_t s) {
  if (n == 0) return hipSuccess;
  hipLaunchKernelGGL(k_class_count, dim3((unsigned)((n + 255) / 256)), dim3(256), 0, s, n, order,
                     lev, ptr, ccount);
  return hipGetLastError();
}

hipError_t launch_class_place(int64_t n, const int32_t *order, const int32_t *lev,
                              const int64_t *ptr, const int64_t *cbase, int32_t *ccursor,
                              int32_t *list, hipStream_t s) {
  if (n == 0) return hipSuccess;
  hipLaunchKernelGGL(k_class_place, dim3((unsigned)((n + 255) / 256)), dim3(256), 0, s, n, order,
                     lev, ptr, cbase, ccursor, list);
  return hipGetLastError();
}

// ---------------------------------------------------------------------------
// Units of the dependency-driven sweeps (ready.hip), per direction, from the
// class lists (level-major, each level ordered by row class): a group unit
// per 64 / 4^c rows of class c < 4 of a level, and for a longer row one
// block unit per kBlockChunks chunks followed by its fold unit.  Units come
// out level by level in the order the sweep solves the levels (ascending
// forward, descending backward: rev), in class-list order within a level,
// and a fold follows its blocks.
// ---------------------------------------------------------------------------
__device__ __forceinline__ int64_t level_of(const int64_t *lptr, int64_t depth, int64_t i) {
  int64_t lo = 0, hi = depth;  // lptr[lo] <= i < lptr[hi]
  while (hi - lo > 1) {
    const int64_t mid = (lo + hi) >> 1;
    if (lptr[mid] <= i) lo = mid;
    else hi = mid;
  }
  return lo;
}

struct UnitShape {
  int units;    // units that start at this class-list index
  int kind;     // group units: their kind
  int rows;     // group units: rows
  int64_t nch;  // chunk sums it needs (longer rows)
  int64_t j;    // index of the class-list entry in sweep order
};

__device__ __forceinline__ UnitShape unit_shape(int64_t n, int64_t depth, const int64_t *lptr,
                                                const int64_t *cls, const int32_t *list,
                                                const int64_t *ptr, int64_t i, bool rev) {
  UnitShape u{0, 0, 0, 0, i};
  const int64_t pos = list[i];
  const int64_t m = ptr[pos + 1] - ptr[pos];
  const int64_t L = level_of(lptr, depth, i);
  if (rev) u.j = (n - lptr[L + 1]) + (i - lptr[L]);
  const int c = row_class(m);
  if (c < kRowClasses - 1) {
    const int per = kWave >> (2 * c);  // rows of one group unit
    const int64_t b0 = cls[kRowClasses * L + c], b1 = cls[kRowClasses * L + c + 1];
    const int64_t k = i - b0;
    if (k % per == 0) {
      u.units = 1;
      u.kind = kUnitGroup1 + c;
      u.rows = (int)(b1 - i < per ? b1 - i : per);
    }
  } else {
    u.nch = (m + kChunk - 1) / kChunk;
    u.units = (int)((u.nch + kBlockChunks - 1) / kBlockChunks) + 1;
  }
  return u;
}

__global__ void k_unit_count(int64_t n, int64_t depth, const int64_t *__restrict__ lptr,
                             const int64_t *__restrict__ cls, const int32_t *__restrict__ list,
                             const int64_t *__restrict__ ptr, int32_t *ucnt, int32_t *ccnt,
                             bool rev) {
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= n) return;
  const UnitShape u = unit_shape(n, depth, lptr, cls, list, ptr, i, rev);
  ucnt[u.j] = u.units;
  ccnt[u.j] = (int32_t)u.nch;
}

__global__ void k_unit_write(int64_t n, int64_t depth, const int64_t *__restrict__ lptr,
                             const int64_t *__restrict__ cls, const int32_t *__restrict__ list,
                             const int64_t *__restrict__ ptr, const int64_t *__restrict__ uoff,
                             const int64_t *__restrict__ coff, int4 *units, bool rev) {
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= n) return;
  const UnitShape u = unit_shape(n, depth, lptr, cls, list, ptr, i, rev);
  if (u.units == 0) return;
  const int64_t o = uoff[u.j];
  const int pos = list[i];
  if (u.nch == 0) {
    units[o] = make_int4(u.kind, (int)i, u.rows, 0);
  } else {
    const int c = (int)coff[u.j];
    const int nb = u.units - 1;
    for (int j = 0; j < nb; ++j) units[o + j] = make_int4(kUnitBlock, pos, j * kBlockChunks, c);
    units[o + nb] = make_int4(kUnitFold, pos, (int)u.nch, c);
  }
}

hipError_t launch_unit_count(int64_t n, int64_t depth, const int64_t *lptr, const int64_t *cls,
                             const int32_t *list, const int64_t *ptr, int32_t *ucnt,
                             int32_t *ccnt, bool rev, hipStream_t s) {
  if (n == 0) return hipSuccess;
  hipLaunchKernelGGL(k_unit_count, dim3((unsigned)((n + 255) / 256)), dim3(256), 0, s, n, depth,
                     lptr, cls, list, ptr, ucnt, ccnt, rev);
  return hipGetLastError();
}

hipError_t launch_unit_write(int64_t n, int64_t depth, const int64_t *lptr, const int64_t *cls,
                             const int32_t *list, const int64_t *ptr, const int64_t *uoff,
                             const int64_t *coff, int4 *units, bool rev, hipStream_t s) {
  if (n == 0) return hipSuccess;
  hipLaunchKernelGGL(k_unit_write, dim3((unsigned)((n + 255) / 256)), dim3(256), 0, s, n, depth,
                     lptr, cls, list, ptr, uoff, coff, units, rev);
  return hipGetLastError();
}

// level-ordered copies: position p holds row order[p]'s entries of F (rows
// for the forward solve; columns minus the ground row for the backward one)
__global__ void k_level_lengths(int64_t n, const int32_t *__restrict__ order,
                                const int64_t *__restrict__ rowptr_f,
                                const int64_t *__restrict__ colptr,
                                const int32_t *__restrict__ rowind, int32_t *flen, int32_t *blen) {
  int64_t p = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (p >= n) return;
  const int32_t i = order[p];
  flen[p] = (int32_t)(rowptr_f[i + 1] - rowptr_f[i]);
  int64_t b = colptr[i], e = colptr[i + 1];
  if (e > b && rowind[e - 1] >= n) --e;  // the ground row is dropped
  blen[p] = (int32_t)(e - b);
}

// position maps: posof[label] = position, src[position] = original vertex,
// D^+ by position (zero pivots give zero: one per component)
__global__ void k_position_maps(int64_t n, const int32_t *__restrict__ order,
                                const int32_t *__restrict__ iperm, const double *__restrict__ D,
                                int32_t *posof, int32_t *src, double *pdinv, float *pdinv32) {
  int64_t p = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (p >= n) return;
  const int32_t i = order[p];
  posof[i] = (int32_t)p;
  src[p] = iperm[i];
  const double d = D[i];
  const double v = d > 0.0 ? 1.0 / d : 0.0;
  pdinv[p] = v;
  if (pdinv32) pdinv32[p] = (float)v;
}

// position p holds row order[p]'s entries of F (rows for the forward solve;
// columns minus the ground row for the backward one), indices as positions
// 16 lanes per position, so that a row's (and a column's) reads and writes
// are contiguous
constexpr int kCopyLanes = 16;
__global__ void k_level_copy(int64_t n, const int32_t *__restrict__ order,
                             const int32_t *__restrict__ posof,
                             const int64_t *__restrict__ rowptr_f,
                             const int32_t *__restrict__ colind_f, const double *__restrict__ val_f,
                             const int64_t *__restrict__ colptr, const int32_t *__restrict__ rowind,
                             const double *__restrict__ val, const int64_t *__restrict__ lf_ptr,
                             const int64_t *__restrict__ lb_ptr, int32_t *lf_idx, double *lf_val,
                             int32_t *lb_idx, double *lb_val) {
  const int64_t t = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  const int64_t p = t / kCopyLanes;
  const int q = (int)(t % kCopyLanes);
  if (p >= n) return;
  const int32_t i = order[p];
  const int64_t o = lf_ptr[p], e0 = rowptr_f[i], e1 = rowptr_f[i + 1];
  for (int64_t e = e0 + q; e < e1; e += kCopyLanes) {
    lf_idx[o + (e - e0)] = posof[colind_f[e]];
    lf_val[o + (e - e0)] = val_f[e];
  }
  const int64_t ob = lb_ptr[p], cnt = lb_ptr[p + 1] - ob, c0 = colptr[i];
  for (int64_t k = q; k < cnt; k += kCopyLanes) {
    lb_idx[ob + k] = posof[rowind[c0 + k]];
    lb_val[ob + k] = val[c0 + k];
  }
}

hipError_t launch_level_layout(int64_t n, const int32_t *order, const int64_t *rowptr_f,
                               const int64_t *colptr, const int32_t *rowind, int32_t *flen,
                               int32_t *blen, hipStream_t s) {
  if (n == 0) return hipSuccess;
  hipLaunchKernelGGL(k_level_lengths, dim3((unsigned)((n + 255) / 256)), dim3(256), 0, s, n, order,
                     rowptr_f, colptr, rowind, flen, blen);
  return hipGetLastError();
}

__global__ void k_level_offsets(int64_t depth, const int64_t *__restrict__ lptr,
                                const int64_t *__restrict__ lf_ptr,
                                const int64_t *__restrict__ lb_ptr, int64_t *lqf, int64_t *lqb) {
  const int64_t L = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (L > depth) return;
  lqf[L] = lf_ptr[lptr[L]];
  lqb[L] = lb_ptr[lptr[L]];
}

hipError_t launch_level_offsets(int64_t depth, const int64_t *lptr, const int64_t *lf_ptr,
                                const int64_t *lb_ptr, int64_t *lqf, int64_t *lqb, hipStream_t s) {
  hipLaunchKernelGGL(k_level_offsets, dim3((unsigned)((depth + 256) / 256)), dim3(256), 0, s,
                     depth, lptr, lf_ptr, lb_ptr, lqf, lqb);
  return hipGetLastError();
}

// narrow entry slots: the input position of an entry inside the narrow
// range (position - np0), -1 for an input before it and for padding
__global__ void k_narrow_index(int64_t ns, const int32_t *__restrict__ smap,
                               const int32_t *__restrict__ idx, int32_t np0, int16_t *nidx) {
  const int64_t sl = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (sl >= ns) return;
  const int32_t e = smap[sl];
  const int32_t c = e >= 0 ? idx[e] : -1;
  nidx[sl] = (int16_t)(c >= np0 ? c - np0 : -1);
}

hipError_t launch_narrow_index(int64_t ns, const int32_t *smap, const int32_t *idx, int32_t np0,
                               int16_t *nidx, hipStream_t s) {
  if (ns == 0) return hipSuccess;
  hipLaunchKernelGGL(k_narrow_index, dim3((unsigned)((ns + 255) / 256)), dim3(256), 0, s, ns, smap,
                     idx, np0, nidx);
  return hipGetLastError();
}

hipError_t launch_position_maps(int64_t n, const int32_t *order, const int32_t *iperm,
                                const double *D, int32_t *posof, int32_t *src, double *pdinv,
                                float *pdinv32, hipStream_t s) {
  if (n == 0) return hipSuccess;
  hipLaunchKernelGGL(k_position_maps, dim3((unsigned)((n + 255) / 256)), dim3(256), 0, s, n, order,
                     iperm, D, posof, src, pdinv, pdinv32);
  return hipGetLastError();
}

hipError_t launch_level_copy(int64_t n, const int32_t *order, const int32_t *posof,
                             const int64_t *rowptr_f, const int32_t *colind_f,
                             const double *val_f, const int64_t *colptr, const int32_t *rowind,
                             const double *val, const int64_t *lf_ptr, const int64_t *lb_ptr,
                             int32_t *lf_idx, double *lf_val, int32_t *lb_idx, double *lb_val,
                             hipStream_t s) {
  if (n == 0) return hipSuccess;
  hipLaunchKernelGGL(k_level_copy, dim3((unsigned)((n * kCopyLanes + 255) / 256)), dim3(256), 0, s,
                     n, order, posof, rowptr_f, colind_f, val_f, colptr, rowind, val, lf_ptr,
                     lb_ptr, lf_idx, lf_val, lb_idx, lb_val);
  return hipGetLastError();
}

// ==========================================================================
// Consistency of b with the null space: per connected component of the
// factor (labels joined by their first off-diagonal entry), the sum of b.
// ==========================================================================
constexpr int kRedT = 256;

__device__ __forceinline__ double block_sum(double v, double *sh) {
  const int t = threadIdx.x;
  sh[t] = v;
  __syncthreads();
  for (int o = kRedT / 2; o > 0; o >>= 1) {
    if (t < o) sh[t] = sh[t] + sh[t + o];
    __syncthreads();
  }
  double r = sh[0];
  __syncthreads();
  return r;
}

// consistency of b per component: comp[label] = root label, sums per root
__global__ void k_comp_init(int64_t ntot, const int64_t *__restrict__ colptr,
                            const int32_t *__restrict__ rowind, int32_t *parent) {
  int64_t k = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (k >= ntot) return;
  parent[k] = colptr[k + 1] > colptr[k] ? rowind[colptr[k]] : (int32_t)k;
}

__global__ void k_comp_jump(int64_t ntot, const int32_t *__restrict__ src, int32_t *dst,
                            int *changed) {
  int64_t k = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (k >= ntot) return;
  int32_t p = src[k], pp = src[p];
  dst[k] = pp;
  if (pp != p) *changed = 1;
}

hipError_t launch_comp_init(int64_t ntot, const int64_t *colptr, const int32_t *rowind,
                            int32_t *parent, hipStream_t s) {
  hipLaunchKernelGGL(k_comp_init, dim3((unsigned)((ntot + 255) / 256)), dim3(256), 0, s, ntot,
                     colptr, rowind, parent);
  return hipGetLastError();
}

hipError_t launch_comp_jump(int64_t ntot, const int32_t *src, int32_t *dst, int *changed,
                            hipStream_t s) {
  hipLaunchKernelGGL(k_comp_jump, dim3((unsigned)((ntot + 255) / 256)), dim3(256), 0, s, ntot, src,
                     dst, changed);
  return hipGetLastError();
}

// per-root sum and absolute sum of b (label space through perm); lanes of a
// block that share the block's first root are reduced in LDS first (the
// common single-component case), the rest add atomically
__global__ __launch_bounds__(kRedT) void k_comp_sums(int64_t n, const int32_t *__restrict__ perm,
                                                     const int32_t *__restrict__ root,
                                                     const double *__restrict__ b, double *sum,
                                                     double *sabs) {
  __shared__ double sh[kRedT];
  __shared__ int32_t r0;
  int64_t v = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  const bool valid = v < n;
  const int32_t rt = valid ? root[perm[v]] : -1;
  if (threadIdx.x == 0) r0 = rt;
  __syncthreads();
  const bool same = valid && rt == r0;
  const double bv = valid ? b[v] : 0.0;
  double s1 = block_sum(same ? bv : 0.0, sh);
  double s2 = block_sum(same ? fabs(bv) : 0.0, sh);
  if (threadIdx.x == 0 && r0 >= 0) {
    atomicAdd(&sum[r0], s1);
    atomicAdd(&sabs[r0], s2);
  }
  if (valid && !same) {
    atomicAdd(&sum[rt], bv);
    atomicAdd(&sabs[rt], fabs(bv));
  }
}

// flag: a root (label < n, not joined to the ground) with |sum| > 1e-8 sum|b|
__global__ void k_comp_check(int64_t n, int64_t ground, const int32_t *__restrict__ root,
                             const double *__restrict__ sum, const double *__restrict__ sabs,
                             int *bad) {
  int64_t k = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (k >= n) return;
  if (root[k] != k) return;
  if (ground >= 0 && root[k] == ground) return;
  if (fabs(sum[k]) > 1e-8 * sabs[k]) *bad = 1;
}

hipError_t launch_comp_check(int64_t n, int64_t ground, const int32_t *perm, const int32_t *root,
                             const double *b, double *sum, double *sabs, int *bad, hipStream_t s) {
  hipLaunchKernelGGL(k_comp_sums, dim3((unsigned)((n + kRedT - 1) / kRedT)), dim3(kRedT), 0, s, n,
                     perm, root, b, sum, sabs);
  hipLaunchKernelGGL(k_comp_check, dim3((unsigned)((n + 255) / 256)), dim3(256), 0, s, n, ground,
                     root, sum, sabs, bad);
  return hipGetLastError();
}

}  // namespace parac
