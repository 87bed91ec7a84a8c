// serve.hip -- PCG over a batch of independent systems ("slots") in shared
// launches: one launch per PCG phase covers every slot of the batch.
//
// A slot owns a fixed range of workgroups of the launch ([blk0, blk0+nblk),
// nblk a function of its own size only) and walks its rows with that range
// as the grid; its partial sums land in partial[blk0 .. blk0+nblk) and are
// summed in a fixed order by the slot's own reduction block.  Every number a
// slot computes therefore depends on its own data only: a system gives the
// same bits alone (a batch of one, which is how single-system PCG runs) and
// in any mix.
//
// The apply of a batch is one forward and one backward sweep launch over
// every slot (ready.hip); a single system is a batch of one.
#include <float.h>

#include "device.hpp"
#include "internal.hpp"

namespace parac {

constexpr int kST = 256;   // threads of a PCG workgroup
constexpr int kSG = 8;     // lanes per SpMV row
constexpr int kSRPW = kWave / kSG;
constexpr int kSpmvBatch = 8;  // entries per lane whose loads are issued together

int slot_blocks(int64_t n) {
  const int64_t b = (n + 2047) / 2048;
  return (int)(b < 1 ? 1 : (b > kSlotMaxBlocks ? kSlotMaxBlocks : b));
}

__device__ __forceinline__ double sblock_sum(double v, double *sh) {
  const int t = threadIdx.x;
  sh[t] = v;
  __syncthreads();
  for (int o = kST / 2; o > 0; o >>= 1) {
    if (t < o) sh[t] = sh[t] + sh[t + o];
    __syncthreads();
  }
  double r = sh[0];
  __syncthreads();
  return r;
}

// this workgroup's slot (a copy: the kernels' stores cannot alias it, so its
// fields stay in registers), its local block index and the slot's block count
struct SlotBlock {
  PcgSlot s;
  int64_t lb, nb;
  __device__ SlotBlock(const PcgSlot *S, const int32_t *bslot) {
    s = S[bslot[blockIdx.x]];
    lb = (int64_t)blockIdx.x - s.blk0;
    nb = s.nblk;
  }
  __device__ bool done() const { return s.ist[1] != 0; }
  __device__ void put(double v, double *sh, double *partial) const {
    const double b = sblock_sum(v, sh);
    if (threadIdx.x == 0) partial[blockIdx.x] = b;
  }
};

// x = 0, r = b, p = 0; partial b.b
__global__ __launch_bounds__(kST) void k_sinit(const PcgSlot *S, const int32_t *bslot,
                                               double *partial) {
  __shared__ double sh[kST];
  SlotBlock sb(S, bslot);
  const PcgSlot &s = sb.s;
  double acc = 0.0;
  for (int64_t i = sb.lb * kST + threadIdx.x; i < s.n; i += sb.nb * kST) {
    const double v = s.b[i];
    s.x[i] = 0.0;
    s.r[i] = v;
    s.p[i] = 0.0;
    acc = acc + v * v;
  }
  sb.put(acc, sh, partial);
}

// q = A v (kSG lanes per row); partial v.q  (v = p)   or
// q = b - A x; partial q.q                  (residual)
template <bool RESID>
__global__ __launch_bounds__(kST) void k_sspmv(const PcgSlot *S, const int32_t *bslot,
                                               double *partial) {
  __shared__ double sh[kST];
  SlotBlock sb(S, bslot);
  const PcgSlot &s = sb.s;
  if (!RESID && sb.done()) return;
  const double *v = RESID ? s.x : s.p;
  const int l = lane(), grp = l / kSG, sub = l % kSG;
  const int64_t wid = (sb.lb * kST + threadIdx.x) >> 6;
  const int64_t nw = (sb.nb * kST) >> 6;
  double acc = 0.0;
  for (int64_t r0 = wid * kSRPW; r0 < s.n; r0 += nw * kSRPW) {
    const int64_t i = r0 + grp;
    double t = 0.0;
    if (i < s.n) {
      // eight of the lane's entries at a time: their indices and values,
      // then their gathers, then the additions in entry order
      const int64_t e = s.rowptr[i + 1];
      for (int64_t k0 = s.rowptr[i] + sub; k0 < e; k0 += kSG * kSpmvBatch) {
        int32_t cc[kSpmvBatch];
        double vv[kSpmvBatch], xv[kSpmvBatch];
#pragma unroll
        for (int u = 0; u < kSpmvBatch; ++u) {
          const int64_t k = k0 + (int64_t)u * kSG;
          cc[u] = k < e ? s.col[k] : 0;
          vv[u] = k < e ? s.val[k] : 0.0;
        }
#pragma unroll
        for (int u = 0; u < kSpmvBatch; ++u) xv[u] = k0 + (int64_t)u * kSG < e ? v[cc[u]] : 0.0;
#pragma unroll
        for (int u = 0; u < kSpmvBatch; ++u)
          if (k0 + (int64_t)u * kSG < e) t = t + vv[u] * xv[u];
      }
    }
#pragma unroll
    for (int o = kSG / 2; o >= 1; o >>= 1) t = t + __shfl_xor(t, o, kWave);
    if (i < s.n && sub == 0) {
      if (RESID) {
        const double y = s.b[i] - t;
        s.q[i] = y;
        acc = acc + y * y;
      } else {
        s.q[i] = t;
        acc = acc + v[i] * t;
      }
    }
  }
  sb.put(acc, sh, partial);
}

// partial r.z
__global__ __launch_bounds__(kST) void k_sdot(const PcgSlot *S, const int32_t *bslot,
                                              double *partial) {
  __shared__ double sh[kST];
  SlotBlock sb(S, bslot);
  const PcgSlot &s = sb.s;
  if (sb.done()) return;
  double acc = 0.0;
  for (int64_t i = sb.lb * kST + threadIdx.x; i < s.n; i += sb.nb * kST)
    acc = acc + s.r[i] * s.z[i];
  sb.put(acc, sh, partial);
}

// x += alpha p ; r -= alpha q ; partial r.r
__global__ __launch_bounds__(kST) void k_saxpy2(const PcgSlot *S, const int32_t *bslot,
                                                double *partial) {
  __shared__ double sh[kST];
  SlotBlock sb(S, bslot);
  const PcgSlot &s = sb.s;
  if (sb.done()) return;
  const double alpha = s.st[4];
  double acc = 0.0;
  for (int64_t i = sb.lb * kST + threadIdx.x; i < s.n; i += sb.nb * kST) {
    s.x[i] = s.x[i] + alpha * s.p[i];
    const double ri = s.r[i] - alpha * s.q[i];
    s.r[i] = ri;
    acc = acc + ri * ri;
  }
  sb.put(acc, sh, partial);
}

// p = z + beta p
__global__ __launch_bounds__(kST) void k_sxpby(const PcgSlot *S, const int32_t *bslot) {
  SlotBlock sb(S, bslot);
  const PcgSlot &s = sb.s;
  if (sb.done()) return;
  const double beta = s.st[5];
  for (int64_t i = sb.lb * kST + threadIdx.x; i < s.n; i += sb.nb * kST)
    s.p[i] = s.z[i] + beta * s.p[i];
}

// workgroup j reduces slot j.  st: ||b||^2, r.z, p.q, r.r, alpha, beta, rtol,
// true ||b-Ax||^2; ist: iterations, done.  mode 0: ||b||^2 (zero b: done);
// 1: r.z -> beta (first: 0); 2: p.q -> alpha; 3: r.r -> iteration count,
// stopping test and iteration cap; 4: true residual
__global__ __launch_bounds__(kST) void k_sreduce(const PcgSlot *S, const double *partial, int mode,
                                                 int first) {
  __shared__ double sh[kST];
  const PcgSlot s = S[blockIdx.x];
  if (mode != 0 && mode != 4 && s.ist[1]) return;
  double acc = 0.0;
  for (int i = threadIdx.x; i < s.nblk; i += kST) acc = acc + partial[s.blk0 + i];
  const double v = sblock_sum(acc, sh);
  if (threadIdx.x != 0) return;
  double *st = s.st;
  int *ist = s.ist;
  if (mode == 0) {
    st[0] = v;
    ist[0] = 0;
    ist[1] = v > 0.0 ? 0 : 1;
  } else if (mode == 1) {
    st[5] = first ? 0.0 : v / st[1];
    st[1] = v;
  } else if (mode == 2) {
    st[2] = v;
    st[4] = st[1] / v;
  } else if (mode == 3) {
    st[3] = v;
    ist[0] += 1;
    if (sqrt(v) <= st[6] * sqrt(st[0])) ist[1] = 1;
    else if (ist[0] >= ist[2]) ist[1] = 2;  // iteration cap reached
  } else {
    st[7] = v;
  }
}

hipError_t slots_init(const SlotBatch &B, hipStream_t s) {
  hipLaunchKernelGGL(k_sinit, dim3(B.nblocks), dim3(kST), 0, s, B.slots, B.bslot, B.partial);
  hipLaunchKernelGGL(k_sreduce, dim3(B.nslots), dim3(kST), 0, s, B.slots, B.partial, 0, 0);
  return hipGetLastError();
}

hipError_t slots_rz(const SlotBatch &B, int first, hipStream_t s) {
  hipLaunchKernelGGL(k_sdot, dim3(B.nblocks), dim3(kST), 0, s, B.slots, B.bslot, B.partial);
  hipLaunchKernelGGL(k_sreduce, dim3(B.nslots), dim3(kST), 0, s, B.slots, B.partial, 1, first);
  hipLaunchKernelGGL(k_sxpby, dim3(B.nblocks), dim3(kST), 0, s, B.slots, B.bslot);
  return hipGetLastError();
}

hipError_t slots_step(const SlotBatch &B, hipStream_t s) {
  hipLaunchKernelGGL(k_sspmv<false>, dim3(B.nblocks), dim3(kST), 0, s, B.slots, B.bslot,
                     B.partial);
  hipLaunchKernelGGL(k_sreduce, dim3(B.nslots), dim3(kST), 0, s, B.slots, B.partial, 2, 0);
  hipLaunchKernelGGL(k_saxpy2, dim3(B.nblocks), dim3(kST), 0, s, B.slots, B.bslot, B.partial);
  hipLaunchKernelGGL(k_sreduce, dim3(B.nslots), dim3(kST), 0, s, B.slots, B.partial, 3, 0);
  return hipGetLastError();
}

hipError_t slots_true_res(const SlotBatch &B, hipStream_t s) {
  hipLaunchKernelGGL(k_sspmv<true>, dim3(B.nblocks), dim3(kST), 0, s, B.slots, B.bslot,
                     B.partial);
  hipLaunchKernelGGL(k_sreduce, dim3(B.nslots), dim3(kST), 0, s, B.slots, B.partial, 4, 0);
  return hipGetLastError();
}

hipError_t slots_apply(const SlotBatch &B, int prec, hipStream_t s, hipEvent_t mid) {
  return ready_apply(B, prec, s, mid);
}

}  // namespace parac
