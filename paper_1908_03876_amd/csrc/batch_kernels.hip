// Batched kernels: many independent control problems of uneven size in one
// launch (periodic square lattices, each with its own coefficients).
//
// The forward pass and the adjoint pass are each ONE persistent launch: the
// work-groups stay resident, walk a tile table that covers every instance,
// and meet at a grid barrier between time steps.  The per-node arithmetic is
// the single-lattice code (mrt_device.h), so a batched instance computes the
// same numbers as a single run.
//
// The grid barrier spins with a time limit.  A wait that exceeds it (which
// can only happen if the work-groups are not all resident) sets a sticky
// abort flag; from then on every barrier returns at once and every block
// leaves its loops, so the launch always terminates and the host reports
// the error.
#include <hip/hip_runtime.h>

#include "batch_internal.h"
#include "mrt_device.h"

namespace mrt {
namespace {

using namespace dev;

// Grid barrier of the persistent kernels.  Every wavefront first waits
// until its own stores have completed into its XCD's L2 (a work-group
// barrier alone does not wait for them: it orders memory only within the
// work-group, whose wavefronts share one CU), so that the block's stores
// are all in L2 when thread 0 arrives.  Arrivals are spread over 8 group
// counters on their own cache lines, group = block id mod 8: work-groups
// are dealt to the 8 XCDs round-robin, so a group's blocks share one L2,
// and the last arriver of each group writes that L2 back once
// (agent-scope release) before it arrives at the top.  (A release by
// every block instead measured the same at 512 blocks and 35% slower at
// 2048.)  The waiting blocks poll with plain atomic loads and each block
// acquires once after the generation has moved on.  A wall-clock limit
// turns a barrier that never completes into a sticky abort flag.
__device__ __forceinline__ bool grid_sync(BarrierState* bs, unsigned nblocks,
                                          unsigned long long timeout) {
  __shared__ int ok;
  __builtin_amdgcn_s_waitcnt(0);  // vmcnt(0) expcnt(0) lgkmcnt(0)
  __syncthreads();
  if (threadIdx.x == 0) {
    ok = 1;
    if (__hip_atomic_load(&bs->abort.v, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT)) {
      ok = 0;
    } else {
      const unsigned gen =
          __hip_atomic_load(&bs->gen.v, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
      const unsigned ngroups = nblocks < unsigned(kBarrierGroups) ? nblocks : kBarrierGroups;
      const unsigned grp = blockIdx.x % kBarrierGroups;
      const unsigned gsize = (nblocks - grp + kBarrierGroups - 1) / kBarrierGroups;
      bool last = false;
      const unsigned arrived = __hip_atomic_fetch_add(&bs->group[grp].v, 1u, __ATOMIC_RELAXED,
                                                      __HIP_MEMORY_SCOPE_AGENT);
      if (arrived == gsize - 1) {
        // last of its group: every member's stores are in this L2; publish
        // them, reset the group counter, arrive at the top
        __hip_atomic_store(&bs->group[grp].v, 0u, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
        __builtin_amdgcn_fence(__ATOMIC_RELEASE, "agent");
        const unsigned top = __hip_atomic_fetch_add(&bs->top.v, 1u, __ATOMIC_ACQ_REL,
                                                    __HIP_MEMORY_SCOPE_AGENT);
        if (top == ngroups - 1) {
          __hip_atomic_store(&bs->top.v, 0u, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
          __hip_atomic_store(&bs->gen.v, gen + 1u, __ATOMIC_RELEASE, __HIP_MEMORY_SCOPE_AGENT);
          last = true;
        }
      }
      if (!last) {
        const unsigned long long t0 = wall_clock64();
        unsigned spins = 0;
        while (__hip_atomic_load(&bs->gen.v, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT) == gen) {
          __builtin_amdgcn_s_sleep(2);
          // the clock and the abort flag are checked at the first poll and
          // then every 32 polls
          if ((spins++ & 31u) != 0u) continue;
          if (wall_clock64() - t0 > timeout) {
            __hip_atomic_store(&bs->abort.v, 1u, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
            ok = 0;
            break;
          }
          if (__hip_atomic_load(&bs->abort.v, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT)) {
            ok = 0;
            break;
          }
        }
      }
      __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "agent");  // see the other XCDs' stores
    }
  }
  __syncthreads();
  return ok != 0;
}

// Geometry of instance k (periodic, no mask, pitch = L).
__device__ __forceinline__ Geometry inst_geom(int L) {
  Geometry g;
  g.nx = L;
  g.ny = L;
  g.pitch = L;
  g.periodic = 1;
  g.masked = 0;
  g.plane = size_t(L) * L;
  g.link = nullptr;
  g.wflag = nullptr;
  g.nsx = (L + 63) / 64;
  return g;
}

// Node of this thread in tile t; false if outside its lattice.
__device__ __forceinline__ bool tile_node(const BatchTile& tl, int tile_w,
                                          const Geometry& g, NodeIdx& n) {
  const int x = tl.x0 + int(threadIdx.x) % tile_w;
  const int y = tl.y0 + int(threadIdx.x) / tile_w;
  if (x >= g.nx || y >= g.ny) return false;
  make_node(g, x, y, n);
  return true;
}

// Recording is a run-time pointer here as in the single-lattice kernels:
// no call site is specialised on it, so the recorded forward and the
// recomputation compute identical values.
// Node of tile t for this thread: instance offset, geometry, coefficients.
template <typename T>
struct TileNode {
  bool ok;
  size_t fo;
  Geometry g;
  NodeIdx n;
  int k;
};

// The tile table and the per-instance coefficients are read-only for the
// whole launch and are indexed by wave-uniform values, so they are read
// through the constant address space: scalar loads into SGPRs, instead of
// a dozen vector loads per wavefront and tile that the compiler would issue
// for a pointer held in the by-value argument struct.
template <typename U>
__device__ __forceinline__ U uniform_load(const U* p) {
#if __HIP_DEVICE_COMPILE__
  return *reinterpret_cast<const __attribute__((address_space(4))) U*>(
      reinterpret_cast<uintptr_t>(p));
#else
  return *p;  // the host pass only parses device code
#endif
}

template <typename T>
__device__ __forceinline__ TileNode<T> tile_of(const BatchArgs<T>& a, int t) {
  TileNode<T> r;
  const BatchTile tl = uniform_load(a.tiles + t);
  r.k = __builtin_amdgcn_readfirstlane(tl.k);
  r.g = inst_geom(__builtin_amdgcn_readfirstlane(tl.L));
  r.ok = tile_node(tl, a.tile_w, r.g, r.n);
  r.fo = size_t(tl.fo);
  return r;
}

// Forward and adjoint sweeps over this block's tiles, one tile at a time,
// each tile's descriptor and coefficients in SGPRs.  Holding two tiles'
// loads in registers (paired, or the next tile's gathers issued before the
// current collision) measured slower over a gradient iteration.
template <typename T, bool FIRST>
__device__ __forceinline__ void forward_sweep_tiles(const BatchArgs<T>& a, const T* src, T* dst,
                                    T* rec) {
  for (int t = blockIdx.x; t < a.ntiles; t += gridDim.x) {
    const TileNode<T> A = tile_of(a, t);
    if (!A.ok) continue;
    const ModelCoef<T> m = uniform_load(a.coef + A.k);
    T fa[9], ga[9], ca = T(0);
    forward_gather<T, true, FIRST>(A.g, A.n, m, src ? src + 18 * A.fo : nullptr,
                                   a.u0 + A.fo, a.v0 + A.fo, a.ctrl + A.fo, fa, ga, ca);
    forward_collide_store<T, false>(A.g, A.n, m, fa, ga, ca, dst + 18 * A.fo,
                                    rec ? rec + 3 * A.fo : nullptr, 0u);
  }
}

template <typename T, bool FIRST>
__device__ __forceinline__ void adjoint_sweep_tiles(const BatchArgs<T>& a, const T* src, T* dst,
                                    const T* rec) {
  for (int t = blockIdx.x; t < a.ntiles; t += gridDim.x) {
    const TileNode<T> A = tile_of(a, t);
    if (!A.ok) continue;
    const ModelCoef<T> m = uniform_load(a.coef + A.k);
    adjoint_node<T, true, false, FIRST, false>(
        A.g, A.n, m, src ? src + 18 * A.fo : nullptr,
        dst ? dst + 18 * A.fo : nullptr, a.seed_u + A.fo, nullptr, rec + 3 * A.fo,
        a.gacc + A.fo, nullptr, nullptr);
  }
}

// Output of forward step n (checkpoint slot when it closes a segment).
template <typename T>
__device__ __forceinline__ T* fwd_dst(const BatchArgs<T>& a, int n, bool ckpt) {
  if (ckpt && a.mode == 2 && (n + 1) % a.K == 0 && n + 1 < a.N)
    return a.ckpt + size_t((n + 1) / a.K - 1) * a.state_elems;
  return a.buf[n & 1];
}

// Forward steps [n0, n1): step n reads src (or the initial fields when
// n == 0), writes fwd_dst and, from step rec0 on, the record slot n - rec0.
// A barrier follows every step except the last one of the launch.
template <typename T>
__device__ void forward_steps(const BatchArgs<T>& a, int n0, int n1, int rec0,
                              const T* src, bool ckpt, bool sync_last,
                              unsigned nblocks, bool* alive) {
  for (int n = n0; n < n1 && *alive; ++n) {
    T* dst = fwd_dst(a, n, ckpt);
    T* rec = n >= rec0 ? a.rec + size_t(n - rec0) * a.rec_elems : nullptr;
    if (n == 0)
      forward_sweep_tiles<T, true>(a, nullptr, dst, rec);
    else
      forward_sweep_tiles<T, false>(a, src, dst, rec);
    src = dst;
    if (n + 1 < n1 || sync_last) *alive = grid_sync(a.barrier, nblocks, a.timeout);
  }
}

// The persistent grids are sized from the runtime's occupancy query, and
// every work-group must be resident for the grid barrier to complete.  The
// declared minimum of wavefronts per SIMD (8 for FP32, 4 for FP64) keeps
// the compiler's vector AND scalar register allocation within what that
// occupancy allows; without it the scalar-loaded descriptors and
// coefficients took 106 SGPRs, which leaves room for 7 wavefronts per SIMD
// where the vector registers alone allow 8.
template <typename T>
__global__ __launch_bounds__(256, sizeof(T) == 4 ? 8 : 4) void batch_forward_kernel(BatchArgs<T> a) {
  bool alive = true;
  // record the last segment (it is the first one the adjoint needs)
  const int rec0 = a.mode > 0 ? (a.nseg - 1) * a.K : a.N;
  forward_steps<T>(a, 0, a.N, rec0, nullptr, true, false, gridDim.x, &alive);
}

template <typename T>
__global__ __launch_bounds__(256, sizeof(T) == 4 ? 8 : 4) void batch_adjoint_kernel(BatchArgs<T> a) {
  bool alive = true;
  const unsigned nb = gridDim.x;
  const T* asrc = nullptr;
  for (int seg = a.nseg - 1; seg >= 0 && alive; --seg) {
    const int n0 = seg * a.K, n1 = min(a.N, n0 + a.K);
    if (seg != a.rec_seg) {
      const T* src = seg == 0 ? nullptr : a.ckpt + size_t(seg - 1) * a.state_elems;
      forward_steps<T>(a, n0, n1, n0, src, false, true, nb, &alive);
    }
    for (int n = n1 - 1; n >= n0 && alive; --n) {
      T* dst = n == 0 ? nullptr : a.abuf[n & 1];
      const T* rec = a.rec + size_t(n - n0) * a.rec_elems;
      if (n == a.N - 1)
        adjoint_sweep_tiles<T, true>(a, nullptr, dst, rec);
      else
        adjoint_sweep_tiles<T, false>(a, asrc, dst, rec);
      asrc = dst;
      if (n > 0) alive = grid_sync(a.barrier, nb, a.timeout);
    }
  }
}

template <typename T>
__global__ __launch_bounds__(256) void batch_finalize_kernel(BatchArgs<T> a, const T* src) {
  for (int t = blockIdx.x; t < a.ntiles; t += gridDim.x) {
    const BatchTile tl = a.tiles[t];
    const int k = __builtin_amdgcn_readfirstlane(tl.k);
    const Geometry g = inst_geom(a.L[k]);
    NodeIdx n;
    if (!tile_node(tl, a.tile_w, g, n)) continue;
    const size_t fo = a.foff[k];
    finalize_node<T, true, false>(g, n, src + 18 * fo, nullptr, a.uN + fo, a.vN + fo);
  }
}

// Per-tile partial sums; phase 1 (grad == 0): J terms and the seed;
// phase 2: gradient = g + alpha c and its norms.
template <typename T>
__global__ __launch_bounds__(256) void batch_cost_kernel(BatchArgs<T> a, int phase,
                                                         double* partials) {
  for (int t = blockIdx.x; t < a.ntiles; t += gridDim.x) {
    const BatchTile tl = a.tiles[t];
    const int k = tl.k;
    const int L = a.L[k];
    const int x = tl.x0 + int(threadIdx.x) % a.tile_w;
    const int y = tl.y0 + int(threadIdx.x) / a.tile_w;
    double acc[kRedSlots] = {0.0, 0.0, 0.0, 0.0, 0.0};
    if (x < L && y < L) {
      const size_t i = a.foff[k] + size_t(y) * L + x;
      const double alpha = a.alpha[k];
      const double c = double(a.ctrl[i]);
      if (phase == 1) {
        const double d = double(a.uN[i]) - double(a.ut[i]);
        acc[0] = 0.5 * d * d;
        acc[1] = 0.5 * alpha * c * c;
        if (!isfinite(d) || !isfinite(c)) acc[4] = 1.0;
        a.seed_u[i] = T(d);
      } else {
        const double e = a.gacc[i] + alpha * c;
        acc[2] = e * e;
        acc[3] = fabs(e);
        if (!isfinite(e)) acc[4] = 1.0;
        a.grad[i] = T(e);
      }
    }
    block_reduce_store(acc, partials + size_t(t) * kRedSlots);
    __syncthreads();
  }
}

// One block per instance: reduce its tiles' partials in fixed order.
__global__ __launch_bounds__(256) void batch_finish_kernel(
    const double* __restrict__ partials, const int* __restrict__ tbeg,
    double* __restrict__ result) {
  const int k = blockIdx.x;
  double acc[kRedSlots] = {0.0, 0.0, 0.0, 0.0, 0.0};
  for (int t = tbeg[k] + threadIdx.x; t < tbeg[k + 1]; t += blockDim.x) {
#pragma unroll
    for (int s = 0; s < kRedSlots; ++s) {
      const double v = partials[size_t(t) * kRedSlots + s];
      acc[s] = (s == 3) ? fmax(acc[s], v) : acc[s] + v;
    }
  }
  block_reduce_store(acc, result + size_t(k) * kBatchSlots);
}

// Gradient step per instance; zeta <= 0: min(1, 1/||E_k||_inf) from the
// phase-2 reduction (slot 3); the step used goes to slot 5.
template <typename T>
__global__ __launch_bounds__(256) void batch_gd_kernel(BatchArgs<T> a, double zeta,
                                                       double* result) {
  for (int t = blockIdx.x; t < a.ntiles; t += gridDim.x) {
    const BatchTile tl = a.tiles[t];
    const int k = tl.k;
    const int L = a.L[k];
    double z = zeta;
    if (z <= 0.0) {
      const double emax = result[size_t(k) * kBatchSlots + 3];
      z = emax > 0.0 ? fmin(1.0, 1.0 / emax) : 1.0;
    }
    if (threadIdx.x == 0 && tl.x0 == 0 && tl.y0 == 0) result[size_t(k) * kBatchSlots + 5] = z;
    const int x = tl.x0 + int(threadIdx.x) % a.tile_w;
    const int y = tl.y0 + int(threadIdx.x) / a.tile_w;
    if (x < L && y < L) {
      const size_t i = a.foff[k] + size_t(y) * L + x;
      a.ctrl[i] = T(double(a.ctrl[i]) - z * double(a.grad[i]));
    }
  }
}

__global__ void barrier_reset_kernel(BarrierState* bs) {
  if (threadIdx.x == 0 && blockIdx.x == 0) {
    for (int g = 0; g < kBarrierGroups; ++g) bs->group[g].v = 0u;
    bs->top.v = 0u;
    bs->gen.v = 0u;
    bs->abort.v = 0u;
  }
}

}  // namespace

template <typename T>
int batch_max_blocks_per_cu(int which) {
  int n = 0;
  hipError_t e = which == 0
      ? hipOccupancyMaxActiveBlocksPerMultiprocessor(&n, batch_forward_kernel<T>, 256, 0)
      : hipOccupancyMaxActiveBlocksPerMultiprocessor(&n, batch_adjoint_kernel<T>, 256, 0);
  return e == hipSuccess ? n : 0;
}

template <typename T>
void launch_batch_forward(const BatchArgs<T>& a, int blocks, hipStream_t s) {
  hipLaunchKernelGGL(batch_forward_kernel<T>, dim3(blocks), dim3(256), 0, s, a);
}

template <typename T>
void launch_batch_adjoint(const BatchArgs<T>& a, int blocks, hipStream_t s) {
  hipLaunchKernelGGL(batch_adjoint_kernel<T>, dim3(blocks), dim3(256), 0, s, a);
}

template <typename T>
void launch_batch_finalize(const BatchArgs<T>& a, const T* src, int blocks, hipStream_t s) {
  hipLaunchKernelGGL(batch_finalize_kernel<T>, dim3(blocks), dim3(256), 0, s, a, src);
}

template <typename T>
void launch_batch_cost(const BatchArgs<T>& a, int phase, double* partials,
                       const int* tbeg, double* result, int count, int blocks,
                       hipStream_t s) {
  hipLaunchKernelGGL(batch_cost_kernel<T>, dim3(blocks), dim3(256), 0, s, a, phase, partials);
  hipLaunchKernelGGL(batch_finish_kernel, dim3(count), dim3(256), 0, s, partials, tbeg, result);
}

template <typename T>
void launch_batch_gd(const BatchArgs<T>& a, double zeta, double* result, int blocks,
                     hipStream_t s) {
  hipLaunchKernelGGL(batch_gd_kernel<T>, dim3(blocks), dim3(256), 0, s, a, zeta, result);
}

void launch_barrier_reset(BarrierState* bs, hipStream_t s) {
  hipLaunchKernelGGL(barrier_reset_kernel, dim3(1), dim3(64), 0, s, bs);
}

#define MRT_BATCH_INST(T)                                                           \
  template int batch_max_blocks_per_cu<T>(int);                                     \
  template void launch_batch_forward<T>(const BatchArgs<T>&, int, hipStream_t);     \
  template void launch_batch_adjoint<T>(const BatchArgs<T>&, int, hipStream_t);     \
  template void launch_batch_finalize<T>(const BatchArgs<T>&, const T*, int,        \
                                         hipStream_t);                              \
  template void launch_batch_cost<T>(const BatchArgs<T>&, int, double*, const int*, \
                                     double*, int, int, hipStream_t);               \
  template void launch_batch_gd<T>(const BatchArgs<T>&, double, double*, int,       \
                                   hipStream_t);
MRT_BATCH_INST(float)
MRT_BATCH_INST(double)
#undef MRT_BATCH_INST

}  // namespace mrt
