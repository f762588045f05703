// Fused linear-combination epilogue shared by the product kernels.
//
// After the k loop, one band of WTM rows at a time, the waves of that band
// write their MFMA accumulators to LDS (the 16 x 16 block layout of lane
// (lg, lr), register r is column lr and row M::row_in_block(lg, r)), then all
// threads read the band back in row-major order, VEC consecutive columns per
// thread, and write every output
//   O_o = e_o D + sum_q c_oq M_q + d_o [i == j < nvalid]
// with coalesced 16-byte reads of the inputs M_q and 16-byte writes.
#pragma once

#include "common.hpp"

namespace sc {

template <typename T>
struct VecOf;
template <>
struct VecOf<double> {
  typedef double __attribute__((ext_vector_type(2))) t;
  static constexpr int N = 2;
};
template <>
struct VecOf<float> {
  typedef float __attribute__((ext_vector_type(4))) t;
  static constexpr int N = 4;
};

// smem must hold at least (BM / WGM) * (BN + VEC) elements of T. The waves
// 0 .. WGM WGN - 1 own the accumulators; NTHR threads (a multiple of 64, at
// least the owners') share the reading and writing, and all of them call this.
template <typename T, int BM, int BN, int WGM, int WGN, typename M, typename AccT, int FM, int FN,
          int NTHR = WGM * WGN * 64>
__device__ inline void epilogue_bands(const Problem& P, int np, int tile_m, int tile_n, AccT (&acc)[FM][FN],
                                      T* smem) {
  using vec_t = typename VecOf<T>::t;
  constexpr int VEC = VecOf<T>::N;
  constexpr int NT = NTHR;
  static_assert(NT % 64 == 0 && NT >= WGM * WGN * 64, "epilogue threads");
  constexpr int WTM = BM / WGM, WTN = BN / WGN;
  constexpr int LDE = BN + VEC;
  const int tid = threadIdx.x;
  const int lane = tid & 63, wave = tid >> 6;
  const int wm = wave / WGN, wn = wave % WGN;
  const int lr = lane & 15, lg = lane >> 4;
  const int nin = P.nin, nout = P.nout, nvalid = P.nvalid;
  T* const E = smem;
  for (int band = 0; band < WGM; ++band) {
    if (wm == band) {
#pragma unroll
      for (int i = 0; i < FM; ++i)
#pragma unroll
        for (int j = 0; j < FN; ++j)
#pragma unroll
          for (int r = 0; r < 4; ++r)
            E[(i * 16 + M::row_in_block(lg, r)) * LDE + wn * WTN + j * 16 + lr] = acc[i][j][r];
    }
    __syncthreads();
    for (int e = tid * VEC; e < WTM * BN; e += NT * VEC) {
      const int br = e / BN, bc = e - br * BN;
      const int row = tile_m * BM + band * WTM + br;
      const int col = tile_n * BN + bc;
      const vec_t v = *(const vec_t*)(E + br * LDE + bc);
      vec_t x[MAX_IN];
#pragma unroll
      for (int q = 0; q < MAX_IN; ++q)
        if (q < nin) x[q] = *(const vec_t*)((const T*)P.in[q].p + (int64_t)row * np + col);
#pragma unroll
      for (int o = 0; o < MAX_OUT; ++o) {
        if (o >= nout) break;
        const EpiOut& O = P.out[o];
        vec_t val;
#pragma unroll
        for (int t = 0; t < VEC; ++t) {
          T y = (row == col + t && row < nvalid) ? (T)O.d : (T)0;
          y = __builtin_fma((T)O.e, v[t], y);
#pragma unroll
          for (int q = 0; q < MAX_IN; ++q)
            if (q < nin) y = __builtin_fma((T)O.c[q], x[q][t], y);
          val[t] = y;
        }
        const int64_t off = (int64_t)row * O.ld + col;
        const bool internal = O.lim == np && O.ld == np && (O.f64 != 0) == (sizeof(T) == 8);
        if (internal) {
          *(vec_t*)((T*)O.p + off) = val;
        } else if (row < O.lim) {
#pragma unroll
          for (int t = 0; t < VEC; ++t) {
            if (col + t < O.lim) {
              if (O.f64) ((double*)O.p)[off + t] = (double)val[t];
              else ((T*)O.p)[off + t] = val[t];
            }
          }
        }
      }
    }
    __syncthreads();
  }
}


}  // namespace sc
