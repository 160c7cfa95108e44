// Single and grouped launches of a kernel body OP (device code).
//
// OP::run(args, b) does the work of block b of one grid.  k_one runs it over
// one grid (block b = blockIdx.x).  k_group runs many independent grids in
// one launch: entry bmap[w] = (segment << 20) | b names the grid
// (segs[segment]) and its block, w being the workgroup's position in XCD
// order (xcd_block); a segment whose system is marked finished
// (live[args.sys] == 0) is skipped.
#pragma once
#include <hip/hip_runtime.h>

namespace smg {

template <class OP>
__global__ __launch_bounds__(256) void k_one(const typename OP::Args a) {
  OP::run(a, blockIdx.x);
}

// As k_one, with workgroups spread over the chip's 8 XCDs (workgroup b is
// dispatched to XCD b % 8, each with its own L2) so that every XCD works on
// a contiguous range of blocks: neighbouring blocks, which share halo data,
// then share an L2.  A bijection of [0, nb).
__device__ inline unsigned xcd_block(unsigned b, unsigned nb) {
  const unsigned q = nb / 8u, r = nb % 8u, x = b % 8u;
  return x * q + (x < r ? x : r) + b / 8u;
}
template <class OP>
__global__ __launch_bounds__(256) void k_one_xcd(const typename OP::Args a) {
  OP::run(a, xcd_block(blockIdx.x, gridDim.x));
}

template <class OP>
__global__ __launch_bounds__(256) void k_group(const typename OP::Args* __restrict__ segs,
                                               const unsigned* __restrict__ bmap, const int* __restrict__ live) {
  // consecutive map entries (neighbouring blocks of one grid) stay on one XCD
  const unsigned e = bmap[xcd_block(blockIdx.x, gridDim.x)];
  const typename OP::Args& a = segs[e >> 20];
  if (live != nullptr && live[a.sys] == 0) return;
  OP::run(a, e & 0xFFFFFu);
}

}  // namespace smg
