// Split-BF16 x3 products with float32 accumulation (precision tier).
//
// Each float32 operand value x is split while it is staged into LDS as
//   hi = bf16(x)  (round to nearest even),   lo = bf16(x - hi)
// (x - hi is exact in float32), and a product is accumulated as
//   A B ~ Ahi Bhi + Ahi Blo + Alo Bhi
// on the gfx950 16x16x32 bf16 MFMA with float32 accumulators; the dropped
// Alo Blo term and the rounding of lo leave a relative error of order 2^-16
// per product. (Splitting float32 into bfloat16 pieces to use low-precision
// matrix units is the method of Henry, Tang and Heinecke, "Leveraging the
// bfloat16 artificial intelligence datatype for higher-precision
// computations", ARITH 2019.)
//
// Layout: BK = 32 (one MFMA k-depth). LDS holds hi and lo planes of the A tile
// as [m][k] and of the B tile as [n][k] (k contiguous, pitch 40 bf16 = 80
// bytes, so 16 lanes reading 16 rows hit distinct banks); each lane feeds its
// MFMA with one 16-byte read of 8 consecutive k per plane. The B tile is read
// from global memory column-wise (each thread one column, BN/8 rows, the
// wavefront's loads contiguous along the row) so that its LDS writes are
// contiguous too. The epilogue is the shared fused linear combination.
#include "common.hpp"
#include "epilogue.hpp"

namespace sc {

typedef __bf16 v8bf __attribute__((ext_vector_type(8)));
typedef __bf16 v4bf __attribute__((ext_vector_type(4)));
typedef float v4f_b __attribute__((ext_vector_type(4)));

struct MmaBf16 {
  typedef v4f_b acc_t;
  __device__ static inline int row_in_block(int lg, int r) { return 4 * lg + r; }
};

// hi = bf16(x), lo = bf16(x - hi) for four values, both rounded to nearest
// even: gfx950 converts two float32 values to a bfloat16 pair in one
// instruction; the pair widens back with a shift and a mask of its 32 bits,
// and x - hi is exact.
typedef __bf16 v2bf __attribute__((ext_vector_type(2)));
typedef float v2f_b __attribute__((ext_vector_type(2)));
__device__ inline void split2(float x0, float x1, unsigned& hi, unsigned& lo) {
  const v2f_b x = {x0, x1};
  const v2bf h = __builtin_convertvector(x, v2bf);
  hi = __builtin_bit_cast(unsigned, h);
  const v2f_b hf = {__uint_as_float(hi << 16), __uint_as_float(hi & 0xffff0000u)};
  lo = __builtin_bit_cast(unsigned, __builtin_convertvector(x - hf, v2bf));
}
__device__ inline void split4(v4f_b x, v4bf& hi, v4bf& lo) {
  unsigned h[2], l[2];
  split2(x[0], x[1], h[0], l[0]);
  split2(x[2], x[3], h[1], l[1]);
  hi = __builtin_bit_cast(v4bf, h);
  lo = __builtin_bit_cast(v4bf, l);
}

__device__ inline void tile_coords_b(int np, int BM, int BN, int nprob, int& p, int& tm, int& tn) {
  const int tmc = np / BM, tnc = np / BN, tiles = tmc * tnc;
  const int total = tiles * nprob;
  int b = blockIdx.x;
  if ((total & 7) == 0) b = (b & 7) * (total >> 3) + (b >> 3);
  p = b / tiles;
  const int t = b - p * tiles;
  constexpr int GROUP = 8;
  const int group = t / (GROUP * tnc);
  const int first = group * GROUP;
  const int rows = (tmc - first) < GROUP ? (tmc - first) : GROUP;
  const int in_group = t - group * GROUP * tnc;
  tm = first + in_group % rows;
  tn = in_group / rows;
}

// SCALED: some k-segment carries an operand scale other than 1 (otherwise
// the split skips the multiplications).
// COND: the launch is decided on the device (DevCond), as in the FP64/FP32
// product kernel; COND = false kernels carry none of it.
template <int BM, int BN, int WGM, int WGN, int WPE, bool SCALED, bool COND>
__global__ __launch_bounds__(WGM * WGN * 64) __attribute__((amdgpu_waves_per_eu(WPE, WPE)))
void gemm_bf16x3_kernel(const GemmLaunch g) {
  constexpr int NT = WGM * WGN * 64;
  constexpr int BK = 32;
  constexpr int WTM = BM / WGM, WTN = BN / WGN;
  constexpr int FM = WTM / 16, FN = WTN / 16;
  constexpr int LDK = BK + 8;                  // bf16 elements per LDS row
  constexpr int A_LOADS = BM * BK / 4 / NT;    // float4 loads per thread
  constexpr int B_ROWS = BK * BN / NT;         // rows (k) per thread, one column
  constexpr int PLANE_A = BM * LDK, PLANE_B = BN * LDK;
  constexpr int BUF = 2 * PLANE_A + 2 * PLANE_B;   // hi, lo of A and B (ushort)
  constexpr int STAGE_BYTES = 2 * BUF * 2;
  constexpr int EPI_BYTES = WTM * (BN + 4) * 4;
  constexpr int SMEM_BYTES = STAGE_BYTES > EPI_BYTES ? STAGE_BYTES : EPI_BYTES;
  static_assert(A_LOADS >= 1 && A_LOADS * 4 * NT == BM * BK, "A staging");
  static_assert(B_ROWS >= 4 && B_ROWS * NT == BK * BN && NT % BN == 0, "B staging");
  static_assert(FM >= 1 && FN >= 1, "wave tile");

  __shared__ __attribute__((aligned(16))) unsigned char smem_raw[SMEM_BYTES];
  unsigned short* const sm = (unsigned short*)smem_raw;

  int dyn_s = 0, dyn_level = 0;
  if constexpr (COND) {
    if (!cond_applies(g.cond, dyn_s, dyn_level)) return;   // uniform: the whole workgroup leaves
  }

  const int np = g.np;
  int p, tile_m, tile_n;
  if (COND && g.cond.select) {
    tile_coords_b(np, BM, BN, 1, p, tile_m, tile_n);
    p = cond_problem(g.cond, g.nprob, dyn_level);
    if (p < 0) return;
  } else {
    tile_coords_b(np, BM, BN, g.nprob, p, tile_m, tile_n);
  }
  const Problem& P = g.prob[p];

  const int tid = threadIdx.x;
  const int lane = tid & 63, wave = tid >> 6;
  const int wm = wave / WGN, wn = wave % WGN;
  const int lr = lane & 15, lg = lane >> 4;

  v4f_b acc[FM][FN];
#pragma unroll
  for (int i = 0; i < FM; ++i)
#pragma unroll
    for (int j = 0; j < FN; ++j)
#pragma unroll
      for (int r = 0; r < 4; ++r) acc[i][j][r] = 0.f;

  int offA[A_LOADS], ldsA[A_LOADS];
#pragma unroll
  for (int i = 0; i < A_LOADS; ++i) {
    const int e = (i * NT + tid) * 4;
    const int r = e / BK, c = e - r * BK;
    offA[i] = r * np + c;
    ldsA[i] = r * LDK + c;
  }
  const int bcol = tid % BN, bgrp = tid / BN;   // B: one column, rows bgrp*B_ROWS ..
  const unsigned boffB = (unsigned)(bgrp * B_ROWS * np + bcol) * 4u;
  const int ldsB = bcol * LDK + bgrp * B_ROWS;

  const int nk = np / BK;
  const int nkt = P.nseg * nk;
  const int64_t a_tile = (int64_t)tile_m * BM * np;
  const int64_t b_tile = (int64_t)tile_n * BN;
  v4f_b ra[A_LOADS];
  float rb[B_ROWS];

  auto gload = [&](int kt) {
    const int sidx = kt / nk;
    const int k0 = (kt - sidx * nk) * BK;
    const float* L = (const float*)P.seg[sidx].L + a_tile + k0;
    const float* R = (const float*)P.seg[sidx].R + b_tile + (int64_t)k0 * np;
#pragma unroll
    for (int i = 0; i < A_LOADS; ++i) ra[i] = *(const v4f_b*)(L + offA[i]);
    // row j of this thread's column: a uniform row pointer plus the thread's
    // 32-bit byte offset (one scalar base per load, no 64-bit vector adds)
#pragma unroll
    for (int j = 0; j < B_ROWS; ++j)
      rb[j] = *(const float*)((const char*)(R + (int64_t)j * np) + boffB);
  };

  auto lstore = [&](int buf, int kt) {
    const Seg& S = P.seg[kt / nk];
    const float ls = SCALED ? (float)(COND ? resolve_scale(S.lscale, dyn_s) : S.lscale) : 1.f;
    const float rs = SCALED ? (float)(COND ? resolve_scale(S.rscale, dyn_s) : S.rscale) : 1.f;
    unsigned short* ahi = sm + buf * BUF;
    unsigned short* alo = ahi + PLANE_A;
    unsigned short* bhi = alo + PLANE_A;
    unsigned short* blo = bhi + PLANE_B;
#pragma unroll
    for (int i = 0; i < A_LOADS; ++i) {
      v4bf h, l;
      split4(ra[i] * ls, h, l);
      *(v4bf*)(ahi + ldsA[i]) = h;
      *(v4bf*)(alo + ldsA[i]) = l;
    }
#pragma unroll
    for (int j0 = 0; j0 < B_ROWS; j0 += 4) {
      const v4f_b x = {rb[j0] * rs, rb[j0 + 1] * rs, rb[j0 + 2] * rs, rb[j0 + 3] * rs};
      v4bf h, l;
      split4(x, h, l);
      *(v4bf*)(bhi + ldsB + j0) = h;
      *(v4bf*)(blo + ldsB + j0) = l;
    }
  };

  if (nkt > 0) {
    gload(0);
    lstore(0, 0);
  }
  __syncthreads();

  for (int kt = 0; kt < nkt; ++kt) {
    const int cur = kt & 1;
    if (kt + 1 < nkt) gload(kt + 1);
    const unsigned short* ahi = sm + cur * BUF;
    const unsigned short* alo = ahi + PLANE_A;
    const unsigned short* bhi = alo + PLANE_A;
    const unsigned short* blo = bhi + PLANE_B;
    v8bf ah[FM], al[FM], bh[FN], bl[FN];
#pragma unroll
    for (int i = 0; i < FM; ++i) {
      const int o = (wm * WTM + i * 16 + lr) * LDK + lg * 8;
      ah[i] = *(const v8bf*)(ahi + o);
      al[i] = *(const v8bf*)(alo + o);
    }
#pragma unroll
    for (int j = 0; j < FN; ++j) {
      const int o = (wn * WTN + j * 16 + lr) * LDK + lg * 8;
      bh[j] = *(const v8bf*)(bhi + o);
      bl[j] = *(const v8bf*)(blo + o);
    }
#pragma unroll
    for (int i = 0; i < FM; ++i)
#pragma unroll
      for (int j = 0; j < FN; ++j) {
        acc[i][j] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(al[i], bh[j], acc[i][j], 0, 0, 0);
        acc[i][j] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(ah[i], bl[j], acc[i][j], 0, 0, 0);
        acc[i][j] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(ah[i], bh[j], acc[i][j], 0, 0, 0);
      }
    if (kt + 1 < nkt) lstore(cur ^ 1, kt + 1);
    __syncthreads();
  }

  epilogue_bands<float, BM, BN, WGM, WGN, MmaBf16>(P, np, tile_m, tile_n, acc, (float*)smem_raw);
}

template <int BM, int BN, int WGM, int WGN, int WPE>
static sincosm_status launch_b(const GemmLaunch& g, hipStream_t stream) {
  const int tiles = (g.np / BM) * (g.np / BN) * (g.cond.plan && g.cond.select ? 1 : g.nprob);
  if (tiles <= 0) return SINCOSM_OK;
  bool scaled = false;
  for (int p = 0; p < g.nprob; ++p)
    for (int s = 0; s < g.prob[p].nseg; ++s)
      scaled |= g.prob[p].seg[s].lscale != 1.0 || g.prob[p].seg[s].rscale != 1.0;
  const bool cond = g.cond.plan != nullptr;
  if (scaled && cond)
    gemm_bf16x3_kernel<BM, BN, WGM, WGN, WPE, true, true><<<tiles, WGM * WGN * 64, 0, stream>>>(g);
  else if (scaled)
    gemm_bf16x3_kernel<BM, BN, WGM, WGN, WPE, true, false><<<tiles, WGM * WGN * 64, 0, stream>>>(g);
  else if (cond)
    gemm_bf16x3_kernel<BM, BN, WGM, WGN, WPE, false, true><<<tiles, WGM * WGN * 64, 0, stream>>>(g);
  else
    gemm_bf16x3_kernel<BM, BN, WGM, WGN, WPE, false, false><<<tiles, WGM * WGN * 64, 0, stream>>>(g);
  SC_HIP(hipGetLastError());
  return SINCOSM_OK;
}

sincosm_status launch_gemm_bf16x3(int tile, const GemmLaunch& g, hipStream_t stream) {
  switch (tile) {
    case 0: return launch_b<128, 128, 2, 2, 2>(g, stream);
    case 1: return launch_b<64, 64, 2, 2, 2>(g, stream);
    default: return launch_b<32, 32, 2, 2, 2>(g, stream);
  }
}

bool bf16x3_available() { return true; }

}  // namespace sc
