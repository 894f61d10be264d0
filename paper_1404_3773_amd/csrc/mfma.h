// MFMA 16x16x4 wrappers for gfx950 (FP32 and FP64), one wave per tile.
// Operand layout (wave64): lane q supplies A[q % 16][q / 16] and
// B[q / 16][q % 16]; the FP32 result of lane q, register v is
// D[4 (q / 16) + v][q % 16], the FP64 result D[q / 16 + 4 v][q % 16].
#pragma once
#include <hip/hip_runtime.h>

namespace ces {

typedef float f4 __attribute__((ext_vector_type(4)));
typedef double d4 __attribute__((ext_vector_type(4)));

template <typename T>
struct MF;
template <>
struct MF<float> {
  typedef f4 acc;
  __device__ static acc mma(float a, float b, acc c) {
    return __builtin_amdgcn_mfma_f32_16x16x4f32(a, b, c, 0, 0, 0);
  }
  __device__ static int row(int lane, int v) { return 4 * (lane >> 4) + v; }
};
template <>
struct MF<double> {
  typedef d4 acc;
  __device__ static acc mma(double a, double b, acc c) {
    return __builtin_amdgcn_mfma_f64_16x16x4f64(a, b, c, 0, 0, 0);
  }
  __device__ static int row(int lane, int v) { return (lane >> 4) + 4 * v; }
};

// N consecutive values as one vector access (dwordx2 / dwordx4 and the
// like); the address must be aligned to N * sizeof(T).
template <typename T, int N>
struct alignas(sizeof(T) * N) VecN {
  T v[N];
};
template <typename T, int N>
__device__ __forceinline__ void load_vec(const T* p, T (&out)[N]) {
  const VecN<T, N> x = *reinterpret_cast<const VecN<T, N>*>(p);
#pragma unroll
  for (int i = 0; i < N; ++i) out[i] = x.v[i];
}
// Stores of the transform stages' outputs (global memory).  With NTS (an
// output larger than the last-level cache, so the next stage reads it back
// from HBM anyway) they go out as non-temporal (streaming) stores (309
// atoms, FP32 Legendre synthesis: 10.3 -> 9.3 ms); a smaller output is
// stored normally and stays cached for its reader (13 atoms: the synthesis
// read G 30 % slower after streaming stores).  The choice is a template
// parameter of the kernels: as a runtime branch the compiler merged the two
// stores into one plain store.  Measured slower, so not used:
// non-temporal loads of the stages' inputs, and non-temporal scalar stores
// of the radial forward and projector outputs.
constexpr size_t kStreamStoreBytes = size_t(256) << 20;   // MI355X last-level cache
template <typename T, int N, bool NTS>
__device__ __forceinline__ void store_vec(T* p, const T (&in)[N]) {
  typedef T vt __attribute__((ext_vector_type(N)));
  vt x;
#pragma unroll
  for (int i = 0; i < N; ++i) x[i] = in[i];
  if constexpr (NTS)
    __builtin_nontemporal_store(x, reinterpret_cast<vt*>(p));
  else
    *reinterpret_cast<vt*>(p) = x;
}

template <typename A>
__device__ __forceinline__ A zero_acc() {
  A z;
  z[0] = 0;
  z[1] = 0;
  z[2] = 0;
  z[3] = 0;
  return z;
}

}  // namespace ces
