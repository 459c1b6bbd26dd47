// Internal declarations shared by the kernel launchers and the C-ABI layer.
#pragma once
#include <hip/hip_runtime.h>
#include <stddef.h>
#include <stdint.h>

#include <algorithm>

#include "pinv_device.h"

namespace pinv {

struct ApplyItemDev {
  const void* D;   // [F][M]
  const void* R;   // [N][M]
  void* X;         // [F][N]
  int F, N, M;
  int tile0;       // first tile of this item in the grouped launch
};

constexpr int kMaxGroup = 32;
struct ApplyBatch {     // passed by value as a kernel argument
  int n;
  ApplyItemDev it[kMaxGroup];
};

template <typename T> hipError_t launch_gram(const EncDev<T>& e, double* G, int flush, hipStream_t s);
template <typename T> hipError_t launch_gram_shared(const EncDev<T>& e, double* G, hipStream_t s);
hipError_t launch_cholinv(double* A, double* Li, int N, double lam, int* info, hipStream_t s);
template <typename T> hipError_t launch_trmm_w(const EncDev<T>& e, const T* Li, T* W, hipStream_t s);
template <typename T>
hipError_t launch_trmm_r(const T* Li, const T* W, T* R, int N, int M, hipStream_t s);
template <typename T> int apply_tiles(int F, int N);
template <typename T> hipError_t launch_apply(const ApplyBatch& b, int total_tiles, hipStream_t s);
template <typename T, typename SX, typename SD>
hipError_t launch_forward(const EncDev<T>& e, const SX* X, int F, const SD* Din, T* Dout,
                          hipStream_t s);
template <typename T, typename SD, typename SX, typename SO>
hipError_t launch_adjoint(const EncDev<T>& e, const SD* D, int F, const SX* X, double lam, SO* Z,
                          hipStream_t s);
template <typename SX, typename SO>
hipError_t launch_resid(const double* G, const double* b, const SX* X, int F, int N, double lam,
                        SO* Out, hipStream_t s);
hipError_t launch_herm_fill(double* G, int N, hipStream_t s);
template <typename T, int MODE, typename SO>
hipError_t launch_tri_frames(const T* Li, const T* In, int F, int N, SO* Out, hipStream_t s);
hipError_t launch_trmm_w_b3(const EncDev<float>& e, const float* Li, float* W, hipStream_t s);
hipError_t launch_trmm_r_b3(const float* Li, const float* W, float* R, int N, int M, hipStream_t s);
int apply_tiles_b3(int F, int N);
hipError_t launch_apply_b3(const ApplyBatch& b, int total_tiles, hipStream_t s);
hipError_t launch_to_f32(const double* in, float* out, size_t n_complex, hipStream_t s);

}  // namespace pinv
