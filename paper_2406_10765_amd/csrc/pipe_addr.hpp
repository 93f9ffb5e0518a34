// Address arithmetic of the direct global-to-LDS loads of the pipelined split-bf16 GEMMs
// (gemm16.hip), shared by the kernels and the host-side bounds test of every load.
//
// A load of 16 bytes per lane is issued as a wave-uniform base pointer plus a per-lane 32-bit byte
// offset.  All offsets are non-negative, and every address stays inside its operand: columns
// beyond the last one are replaced by the last one, rows beyond the last group of four rows of
// the leading dimension by that group.
#pragma once

namespace pw {

// K-contiguous operand (ncols columns of ld words), K tile starting at word k0, group g of 16
// columns of the tile starting at column c0: the group's base column and the lane's byte offset
// from (base column, k0).  Lane l takes slot s = l / 16 (words 4 s .. 4 s + 3 of the K tile) of
// column (l % 16) ^ s of the group.
__host__ __device__ inline int pipe_kbase_col(int c0, int g, int ncols) {
  const int c = c0 + g * 16;
  return c < ncols - 1 ? c : ncols - 1;
}
__host__ __device__ inline unsigned int pipe_koff_bytes(int c0, int g, int ncols, long ld, int lane) {
  const int slot = lane >> 4, cl = (lane & 15) ^ slot;
  const int first = pipe_kbase_col(c0, g, ncols);
  const int col = first + cl < ncols - 1 ? first + cl : ncols - 1;
  return (unsigned int)(((long)(col - first) * ld + 4 * slot) * 4);
}
// M-contiguous operand (ld words per k column, ld a multiple of 4), tile of 256 rows from r0
// (r0 a multiple of 256 below the row count, so r0 <= ld - 4): lane l copies rows 4 l .. 4 l + 3,
// clamped to the last group of four rows of the leading dimension.
__host__ __device__ inline unsigned int pipe_moff_bytes(long ld, int r0, int lane) {
  long row = r0 + 4L * lane;
  if (row > ld - 4) row = ld - 4;
  return (unsigned int)((row - r0) * 4);
}

}  // namespace pw
