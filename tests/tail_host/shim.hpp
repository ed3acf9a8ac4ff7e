// Host emulation of the HIP device environment of one workgroup, for running the
// library's device source on the CPU (tests only): one host thread per work-item,
// workgroup barriers and 64-wide wave shuffles emulated, __shared__ variables static.
#pragma once
#include <algorithm>
#include <barrier>
#include <cmath>
#include <cstdint>
#include <cstdio>
#include <cstdlib>
#include <cstring>
#include <thread>
#include <vector>
#define __host__
#define __device__
#define __global__
#define __forceinline__ inline
#define __launch_bounds__(...)
#define __shared__ static
typedef void *hipStream_t;
struct dim3 {
  unsigned x, y, z;
  dim3(unsigned a = 1, unsigned b = 1, unsigned c = 1) : x(a), y(b), z(c) {}
};
struct Dim3 {
  unsigned x, y, z;
};
inline thread_local Dim3 threadIdx{0, 0, 0};
inline Dim3 blockIdx{0, 0, 0};
inline Dim3 blockDim{1024, 1, 1};
inline Dim3 gridDim{1, 1, 1};
inline std::barrier<> *g_block_bar = nullptr;
inline std::barrier<> *g_wave_bar[16] = {};
inline double g_wave_buf[16][64];
inline void __syncthreads() { g_block_bar->arrive_and_wait(); }
template <typename V>
inline V __shfl_down(V v, int o, int) {
  const int lane = threadIdx.x & 63, wid = threadIdx.x >> 6;
  g_wave_buf[wid][lane] = (double)v;
  g_wave_bar[wid]->arrive_and_wait();
  const V r = lane + o < 64 ? (V)g_wave_buf[wid][lane + o] : v;
  g_wave_bar[wid]->arrive_and_wait();
  return r;
}
#define hipLaunchKernelGGL(...) ((void)0)
using std::fma;
using std::sqrt;
template <typename A, typename B>
inline auto min(A a, B b) { return a < b ? a : b; }
template <typename A, typename B>
inline auto max(A a, B b) { return a > b ? a : b; }
