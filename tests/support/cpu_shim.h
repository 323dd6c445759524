// cpu_shim.h -- lets a generated gfx950 kernel source compile as plain C++ on
// the host, so that its per-lane function perm_lane() can be run on the CPU in
// tests of the code generator.  Only the per-lane arithmetic is exercised; the
// cross-lane reduction of the kernel is compiled but never called.
#include <cmath>
#include <cstdint>
#define __global__
#define __device__
#define __forceinline__ inline
#define __launch_bounds__(...)
#define __restrict__
#define __shared__ static
#define __constant__ static const
struct cpu_dim3 { unsigned x, y, z; };
static cpu_dim3 threadIdx, blockIdx;
static inline void __syncthreads() {}
static inline double __shfl_xor(double v, int, int) { return v; }
static inline unsigned long long __shfl_xor(unsigned long long v, int, int) { return v; }
// one-lane wave: the ballot is the lane's own bit, and no lane is below it
static inline unsigned long long __ballot(int p) { return p ? 1ull : 0ull; }
static inline int __popcll(unsigned long long v) { return __builtin_popcountll(v); }
static inline unsigned __builtin_amdgcn_mbcnt_lo(unsigned, unsigned acc) { return acc; }
static inline unsigned __builtin_amdgcn_mbcnt_hi(unsigned, unsigned acc) { return acc; }
// one emulated lane is the whole "wave"
static inline int __all(int p) { return p; }
static inline int __any(int p) { return p; }
using std::fma;
using std::rint;
using std::fabs;
// a one-lane wave: the first lane's value is the value
static inline int __builtin_amdgcn_readfirstlane(int v) { return v; }  // int, as the device builtin
