// Device helpers shared by the kernel translation units (included inside
// namespace mgrit::{anonymous}).
#pragma once

__device__ __forceinline__ int padix(int i) { return i + (i >> 4); }

// i + 1 on the periodic mesh, for 0 <= i < nx
__device__ __forceinline__ int next_periodic(int i, int nx) { return i + 1 == nx ? 0 : i + 1; }

__device__ __forceinline__ int wrap_hi(int i, int nx) {
  while (i >= nx) i -= nx;
  return i;
}

__device__ __forceinline__ int wrap_lo(int i, int nx) {
  while (i < 0) i += nx;
  return i;
}

// Rows of the level arrays live in device memory: they are read and written
// through global-address-space pointers (a flat access would also count
// against the LDS wait counter and hold up the next LDS wait).
template <class T>
using GlobalPtr = __attribute__((address_space(1))) T *;

template <int L, class T>
__device__ __forceinline__ void load_chunk(const T *__restrict__ row_, int base, int cnt, T (&x)[L]) {
  const GlobalPtr<const T> row = (GlobalPtr<const T>)row_;
  if (cnt == L) {
#pragma unroll
    for (int j = 0; j < L; ++j) x[j] = row[base + j];
  } else {
#pragma unroll
    for (int j = 0; j < L; ++j) x[j] = (j < cnt) ? row[base + j] : T(0);
  }
}

template <int L, class T>
__device__ __forceinline__ void store_chunk(T *__restrict__ row_, int base, int cnt, const T (&x)[L]) {
  const GlobalPtr<T> row = (GlobalPtr<T>)row_;
  if (cnt == L) {
#pragma unroll
    for (int j = 0; j < L; ++j) row[base + j] = x[j];
  } else {
#pragma unroll
    for (int j = 0; j < L; ++j)
      if (j < cnt) row[base + j] = x[j];
  }
}

template <int L, class T>
__device__ __forceinline__ void chunk_to_lds(T *vec, int base, int cnt, const T (&x)[L]) {
  if (cnt == L) {
#pragma unroll
    for (int j = 0; j < L; ++j) vec[padix(base + j)] = x[j];
  } else {
#pragma unroll
    for (int j = 0; j < L; ++j)
      if (j < cnt) vec[padix(base + j)] = x[j];
  }
}

// Sum over the workgroup, deterministic order; result valid in thread 0.
__device__ __forceinline__ double block_sum(double v, double *red) {
#pragma unroll
  for (int d = WAVE / 2; d > 0; d >>= 1) v += __shfl_down(v, d, WAVE);
  __syncthreads();
  if ((threadIdx.x & (WAVE - 1)) == 0) red[threadIdx.x >> 6] = v;
  __syncthreads();
  double tot = 0.0;
  if (threadIdx.x == 0) {
    const int nw = blockDim.x >> 6;
    for (int w = 0; w < nw; ++w) tot += red[w];
  }
  return tot;
}
