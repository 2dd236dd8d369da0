// Global-memory addressing for the tile kernels (gfx950).
//
// A block's tile is addressed as a wave-uniform base pointer (kernel
// arguments and block index only, so it lives in scalar registers) plus a
// 32-bit per-lane byte offset that is computed once.  Each access then needs
// no 64-bit vector address arithmetic: the compiler emits the scalar-base
// form of the global load/store with the lane offset in one VGPR.
#pragma once
#include <hip/hip_runtime.h>

#include <cstdint>

namespace hvk {

template <typename T>
__device__ inline T ld_off(const T* base, uint32_t byte_off) {
  return *reinterpret_cast<const T*>(reinterpret_cast<const char*>(base) + byte_off);
}

template <typename T>
__device__ inline void st_off(T* base, uint32_t byte_off, T v) {
  *reinterpret_cast<T*>(reinterpret_cast<char*>(base) + byte_off) = v;
}

// Element q = tid + i * NT of a tile with rows of N elements, split over NT
// threads: row = row_thr(tid) + row_i(i), column = col_thr(tid) + col_i(i).
// One of N, NT divides the other (both are powers of two).
template <int N, int NT>
struct TileSplit {
  static constexpr bool WIDE = NT >= N;  // one pass of the threads covers whole rows
  __device__ static int row_thr(int tid) { return WIDE ? tid / N : 0; }
  __device__ static int col_thr(int tid) { return WIDE ? tid % N : tid; }
  __host__ __device__ static constexpr int row_i(int i) { return WIDE ? i * (NT / N) : i / (WIDE ? 1 : N / NT); }
  __host__ __device__ static constexpr int col_i(int i) { return WIDE ? 0 : (i % (WIDE ? 1 : N / NT)) * NT; }
};

}  // namespace hvk
