// Internal interface of the batched persistent kernels (batch_kernels.hip)
// and their runtime (mrt_batch.cpp).  Not part of the public ABI.
#pragma once

#include <hip/hip_runtime.h>

#include <cstddef>
#include <cstdint>

#include "mrt_internal.h"

namespace mrt {

// One work tile: tile_w x (256 / tile_w) nodes of instance k at (x0, y0).
// One tile of the sweep: instance k, its first row and column, and the
// instance's size and field offset (so that a tile needs one table load).
struct BatchTile {
  int k, y0, x0, L;
  unsigned long long fo;
  unsigned long long pad;
};

// Two-level grid barrier, each word on its own 128-byte line: blocks arrive
// at the counter of their group (block id mod 8, the XCD they run on), the
// last arriver of a group at the top counter; the last group flips the
// generation the waiting blocks poll.  `abort` is the sticky time-out flag.
constexpr int kBarrierGroups = 8;
struct BarrierLine {
  unsigned v;
  unsigned pad[31];
};
struct BarrierState {
  BarrierLine group[kBarrierGroups];
  BarrierLine top;
  BarrierLine gen;
  BarrierLine abort;
};

// Per-instance reduction slots: [0] J_track, [1] J_reg, [2] sum E^2,
// [3] max |E|, [4] non-finite count, [5] step used by the update.
constexpr int kBatchSlots = 8;

template <typename T>
struct BatchArgs {
  const BatchTile* tiles;
  int ntiles, tile_w;
  const ModelCoef<T>* coef;  // [count]
  const int* L;              // [count] lattice side
  const size_t* foff;        // [count] offset of instance k's fields
  const double* alpha;       // [count] control penalty
  int N, K, nseg, mode;      // steps, segment length, segments, tape mode
  int rec_seg;               // segment held by the record (adjoint pass)
  size_t state_elems;        // 18 * F: one batched distribution state
  size_t rec_elems;          // 3 * F: one record slot
  T* buf[2];                 // forward ping-pong
  T* abuf[2];                // adjoint ping-pong
  T* ckpt;                   // (nseg - 1) checkpoint states
  T* rec;                    // K record slots
  const T* u0;
  const T* v0;
  T* ctrl;
  const T* ut;
  T* uN;
  T* vN;
  T* seed_u;
  double* gacc;
  T* grad;
  BarrierState* barrier;
  unsigned long long timeout;  // barrier wait limit in wall-clock ticks
};

template <typename T>
int batch_max_blocks_per_cu(int which /*0 forward, 1 adjoint*/);
template <typename T>
void launch_batch_forward(const BatchArgs<T>& a, int blocks, hipStream_t s);
template <typename T>
void launch_batch_adjoint(const BatchArgs<T>& a, int blocks, hipStream_t s);
template <typename T>
void launch_batch_finalize(const BatchArgs<T>& a, const T* src, int blocks,
                           hipStream_t s);
template <typename T>
void launch_batch_cost(const BatchArgs<T>& a, int phase, double* partials,
                       const int* tbeg, double* result, int count, int blocks,
                       hipStream_t s);
template <typename T>
void launch_batch_gd(const BatchArgs<T>& a, double zeta, double* result,
                     int blocks, hipStream_t s);
void launch_barrier_reset(BarrierState* bs, hipStream_t s);

}  // namespace mrt
