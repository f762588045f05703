// Product X Y of float64 matrices on the int8 matrix cores by error-free
// splitting into slices (the scheme of Ozaki, Ogita, Oishi and Rump, 2012, as
// used for emulated float64 products on integer matrix units by Ootomo,
// Ozaki and Yokota, 2024).
//
// Every row i of X is scaled by 2^-e_i (e_i from the row's largest magnitude,
// so the scaled entries lie in (-1, 1)) and written as five signed 7-bit
// digits, x = 2^e_i sum_{k=1..5} d_k 2^-7k, exactly up to a remainder below
// 2^(e_i - 35); every column j of Y likewise with 2^f_j. Then
//   (X Y)_ij = 2^(e_i + f_j) sum_{k, l} 2^-7(k + l) (D_k E_l)_ij,
// each D_k E_l an int8 product with exact int32 accumulation. The 15 pairs
// with k + l <= 6 are kept, summed per k + l in int32 (exact up to order
// 26000) and combined in float64. Error, elementwise: the digits cut off give
// at most 2^-34 (rowmax|X| colsum|Y| + rowsum|X| colmax|Y|); the 10 pairs
// left out (weights 2^-49 and below, digits up to 127) at most
// 2^-33 n 2^(e_i + f_j) < 2^-31 n rowmax|X| colmax|Y|, a bound reached only
// when the digits agree in sign along the inner dimension; for uncorrelated
// digits their sums grow like n^(1/2) and the first term dominates. Four
// digits (28 bits) were measured too few: the schemes' intermediates cancel,
// and the double-angle steps double what is left, so at s = 6 the
// single-accuracy bar was exceeded; five leave a margin of about two orders
// of magnitude.
//
// Three preparation kernels write the slices (left operand by rows, right
// operand by columns, transposed so that both read 64 consecutive k bytes per
// row of the tile), then the product kernel: 64 x 64 output tiles of four
// waves (2 x 2 blocks of 16 x 16 each), k steps of 64 on
// v_mfma_i32_16x16x64_i8, the slices loaded straight into two LDS buffers
// (64-byte rows whose 16-byte slots are permuted against bank conflicts), and
// the fused linear-combination epilogue of the other product kernels.
#include <math.h>

#include "epilogue.hpp"

namespace sc {
namespace {

typedef int v4i __attribute__((ext_vector_type(4)));
typedef double v4d __attribute__((ext_vector_type(4)));

constexpr int NS = 5;            // slices per operand (7 bits each)
constexpr int QT = 64;           // output tile and k step
constexpr int QTHR = 256;        // threads of the product kernel (4 waves)
constexpr int QROW = 64;         // LDS bytes per staged row (16-byte slots permuted, no padding)
constexpr int QPLANE = QT * QROW;             // bytes per staged plane
constexpr int QSTAGE = 2 * NS * QPLANE;       // A and B planes of one k step
constexpr int QLDS = 2 * QSTAGE;              // two buffers: 160 KiB for 2 workgroups per CU

// result layout of the int8 16 x 16 MFMA: lane (lr, lg), register r -> row 4 lg + r, column lr
struct MI8 {
  __device__ static inline int row_in_block(int lg, int r) { return 4 * lg + r; }
};

// Exponent of a row or column holding Inf or NaN (outside every float64
// exponent): its digits are written as zeros and its results as NaN.
constexpr int I8_NONFINITE = 1 << 16;

// The exponent e with |x| < 2^e for every x of a row or column whose largest
// magnitude is m (0 for m = 0). m is the maximum of the |x| bit patterns, so
// it is Inf or NaN exactly when one of the entries is.
__device__ inline int slice_exponent(double m) {
  if (!isfinite(m)) return I8_NONFINITE;
  if (!(m > 0.0)) return 0;
  int e = 0;
  frexp(m, &e);
  return e;
}

// NS digits of y = x 2^-e in (-1, 1): d_k = trunc(128 y_k), y_{k+1} = 128 y_k - d_k
// (exact in float64).
__device__ inline void slice_digits(double y, int8_t (&d)[NS]) {
  if (!isfinite(y)) y = 0.0;   // a row or column with Inf or NaN (its results are NaN)
#pragma unroll
  for (int k = 0; k < NS; ++k) {
    const double t = y * 128.0;
    const double q = trunc(t);
    d[k] = (int8_t)(int)q;
    y = t - q;
  }
}

// The operands of a launch's problems and its device-side condition, for the
// preparation kernels.
struct I8Operands {
  DevCond cond;
  int nprob;
  const double* L[MAX_PROB];
  const double* R[MAX_PROB];
  int64_t ldl[MAX_PROB], ldr[MAX_PROB];
};

// The problem a launch computes: 0 for a launch without a device plan, else
// the one the plan record selects; -1 when the record rules the launch out
// (every workgroup of every kernel of the product then returns at once).
__device__ inline int i8_problem(const DevCond& c, int nprob, int& s) {
  s = 0;
  if (!c.plan) return 0;
  int level;
  if (!cond_applies(c, s, level)) return -1;
  return c.select ? cond_problem(c, nprob, level) : 0;
}

// Left operand: one workgroup per row; planes P[k][i][c] (np x np each).
__global__ __launch_bounds__(256) void slice_rows_kernel(const I8Operands op, int np, int8_t* __restrict__ P,
                                                         int* __restrict__ ex) {
  __shared__ unsigned long long red[256];
  int s;
  const int q = i8_problem(op.cond, op.nprob, s);
  if (q < 0) return;
  const double* __restrict__ X = op.L[q];
  const int64_t ld = op.ldl[q];
  const int i = blockIdx.x, tid = threadIdx.x;
  const double* row = X + (int64_t)i * ld;
  unsigned long long m = 0ull;
  for (int c = tid; c < np; c += 256) {
    const unsigned long long b = (unsigned long long)__double_as_longlong(fabs(row[c]));
    m = b > m ? b : m;
  }
  red[tid] = m;
  __syncthreads();
  for (int w = 128; w > 0; w >>= 1) {
    if (tid < w && red[tid + w] > red[tid]) red[tid] = red[tid + w];
    __syncthreads();
  }
  const int e = slice_exponent(__longlong_as_double((long long)red[0]));
  if (tid == 0) ex[i] = e;
  const int64_t plane = (int64_t)np * np;
  for (int c = tid; c < np; c += 256) {
    int8_t d[NS];
    slice_digits(ldexp(row[c], -e), d);
#pragma unroll
    for (int k = 0; k < NS; ++k) P[k * plane + (int64_t)i * np + c] = d[k];
  }
}

// Right operand, pass 1: column maxima (bit patterns of |x|, compared as
// integers) over 64 x 64 blocks into cmax (zeroed by the caller).
__global__ __launch_bounds__(256) void col_max_kernel(const I8Operands op, unsigned long long* __restrict__ cmax) {
  __shared__ unsigned long long red[4][64];
  int s;
  const int q = i8_problem(op.cond, op.nprob, s);
  if (q < 0) return;
  const double* __restrict__ X = op.R[q];
  const int64_t ld = op.ldr[q];
  const int c0 = blockIdx.x * 64, r0 = blockIdx.y * 64;
  const int tid = threadIdx.x, c = tid & 63, g = tid >> 6;
  unsigned long long m = 0ull;
  for (int r = g; r < 64; r += 4) {
    const unsigned long long b =
        (unsigned long long)__double_as_longlong(fabs(X[(int64_t)(r0 + r) * ld + c0 + c]));
    m = b > m ? b : m;
  }
  red[g][c] = m;
  __syncthreads();
  if (g == 0) {
    for (int q = 1; q < 4; ++q) m = red[q][c] > m ? red[q][c] : m;
    atomicMax(cmax + c0 + c, m);
  }
}

// Right operand, pass 2: planes of the transpose, P[l][j][r] = digit l of
// X[r][j] 2^-f_j, one 64 x 64 block per workgroup through LDS.
__global__ __launch_bounds__(256) void slice_cols_kernel(const I8Operands op, int np,
                                                         const unsigned long long* __restrict__ cmax,
                                                         int8_t* __restrict__ P, int* __restrict__ ex) {
  __shared__ double tile[64][65];
  int s;
  const int q = i8_problem(op.cond, op.nprob, s);
  if (q < 0) return;
  const double* __restrict__ X = op.R[q];
  const int64_t ld = op.ldr[q];
  const int c0 = blockIdx.x * 64, r0 = blockIdx.y * 64;
  const int tid = threadIdx.x;
  for (int e = tid; e < 64 * 64; e += 256) {
    const int r = e >> 6, c = e & 63;
    tile[r][c] = X[(int64_t)(r0 + r) * ld + c0 + c];
  }
  __syncthreads();
  // thread -> output row j = c0 + (tid >> 2), 16 consecutive r
  const int jc = tid >> 2, rq = (tid & 3) * 16;
  const int f = slice_exponent(__longlong_as_double((long long)cmax[c0 + jc]));
  if (blockIdx.y == 0 && (tid & 3) == 0) ex[c0 + jc] = f;
  int8_t d[NS][16];
#pragma unroll
  for (int t = 0; t < 16; ++t) {
    int8_t dd[NS];
    slice_digits(ldexp(tile[rq + t][jc], -f), dd);
#pragma unroll
    for (int k = 0; k < NS; ++k) d[k][t] = dd[k];
  }
  const int64_t plane = (int64_t)np * np;
#pragma unroll
  for (int k = 0; k < NS; ++k) {
    v4i v;
#pragma unroll
    for (int w = 0; w < 4; ++w)
      v[w] = (int)((uint32_t)(uint8_t)d[k][4 * w] | ((uint32_t)(uint8_t)d[k][4 * w + 1] << 8) |
                   ((uint32_t)(uint8_t)d[k][4 * w + 2] << 16) | ((uint32_t)(uint8_t)d[k][4 * w + 3] << 24));
    *(v4i*)(P + k * plane + (int64_t)(c0 + jc) * np + r0 + rq) = v;
  }
}

__global__ void zero_u64_kernel(unsigned long long* p, int n) {
  const int i = blockIdx.x * 256 + threadIdx.x;
  if (i < n) p[i] = 0ull;
}

// Output tile of this workgroup: consecutive workgroups go to different XCDs
// (round robin), so when the tile count allows, each XCD takes a contiguous
// range of tiles; within it, groups of 8 tile rows are walked column by
// column, so that the panels a group shares stay in that XCD's L2.
__device__ inline void i8_tile_coords(int tpd, int& tm, int& tn) {
  const int tiles = tpd * tpd, b = blockIdx.x;
  const int t = (tiles & 7) == 0 ? (b & 7) * (tiles >> 3) + (b >> 3) : b;
  const int group = t / (8 * tpd), first = group * 8;
  const int rows = tpd - first < 8 ? tpd - first : 8;
  const int in_group = t - group * 8 * tpd;
  tm = first + in_group % rows;
  tn = in_group / rows;
}

// The product kernel. A: planes of the left operand by rows, B: planes of
// the right operand's transpose; both [NS][np][np] int8.
__global__ __launch_bounds__(QTHR) void gemm_i8x5_kernel(const int8_t* __restrict__ A,
                                                           const int8_t* __restrict__ B,
                                                           const int* __restrict__ ea,
                                                           const int* __restrict__ eb, GemmLaunch g) {
  __shared__ __attribute__((aligned(16))) unsigned char smem[QLDS];
  int dyn_s;
  const int pq = i8_problem(g.cond, g.nprob, dyn_s);
  if (pq < 0) return;   // uniform: the whole workgroup leaves
  const Problem& P = g.prob[pq];
  const double scale = resolve_scale(P.seg[0].lscale, dyn_s) * resolve_scale(P.seg[0].rscale, dyn_s);
  const int np = g.np;
  int tile_m, tile_n;
  i8_tile_coords(np / QT, tile_m, tile_n);
  const int tid = threadIdx.x, lane = tid & 63, wave = __builtin_amdgcn_readfirstlane(tid >> 6);
  const int wm = wave >> 1, wn = wave & 1;
  const int lr = lane & 15, lg = lane >> 4;
  const int64_t plane = (int64_t)np * np;
  const int nk = np / QT;

  // Direct loads (global_load_lds, 16 bytes per lane): one wave instruction
  // fills 1 KiB of LDS, 16 rows of one plane, lane l writing row l >> 2 at
  // slot l & 3. Slot s of row r holds k chunk s ^ ((r >> 2) & 3) of that row,
  // so the lane loads chunk (l & 3) ^ ((l >> 4) & 3). Wave w fills rows
  // 16 w .. 16 w + 15 of every plane of both operands. With 64-byte rows,
  // rows r, r + 4, r + 8, r + 12 fall on the same banks; the permutation puts
  // their k chunks on distinct slots, so the 16 rows of a fragment read (and
  // the 4 rows x 4 slots of a load) cover the 64 banks once.
  typedef __attribute__((address_space(3))) void lds_void;
  typedef __attribute__((address_space(1))) void glb_void;
  const int lrow = wave * 16 + (lane >> 2);
  const int lchunk = 16 * ((lane & 3) ^ ((lane >> 4) & 3));
  const int8_t* const arow = A + (int64_t)(tile_m * QT + lrow) * np + lchunk;
  const int8_t* const brow = B + (int64_t)(tile_n * QT + lrow) * np + lchunk;
  auto dload = [&](int buf, int kt) {
    const int k0 = kt * QT;
    unsigned char* dst = smem + buf * QSTAGE + wave * 1024;
#pragma unroll
    for (int u = 0; u < 2 * NS; ++u) {
      const int8_t* src = (u < NS ? arow + u * plane : brow + (u - NS) * plane) + k0;
      __builtin_amdgcn_global_load_lds((glb_void*)src, (lds_void*)(dst + u * QPLANE), 16, 0, 0);
    }
  };
  // fragment rows: wm 32 + 16 i + lr (A), wn 32 + 16 i + lr (B); k chunk lg
  const int rslot = 16 * (lg ^ ((lr >> 2) & 3));
  const int ra0 = (wm * 32 + lr) * QROW + rslot, rb0 = NS * QPLANE + (wn * 32 + lr) * QROW + rslot;

  constexpr int NG = NS;   // groups k + l = 0 .. NS - 1 (slice indices from 0)
  v4i acc[NG][2][2];
#pragma unroll
  for (int gq = 0; gq < NG; ++gq)
#pragma unroll
    for (int i = 0; i < 2; ++i)
#pragma unroll
      for (int j = 0; j < 2; ++j) acc[gq][i][j] = (v4i){0, 0, 0, 0};

  // Two buffers, one barrier per k step. The buffer a step loads was last
  // read in the step before: every wave finished those reads before the
  // barrier that ended that step. Each wave waits for its own direct loads
  // (vmcnt) before the barrier that publishes them; the last barrier also
  // frees the LDS for the epilogue.
  // Step kt first issues the loads of step kt + 1 into the other buffer (the
  // last step loads its own k block again, so that the loop body has no
  // branch: the copy is never read, and it has landed before the final
  // barrier), then reads its fragments from buffer kt & 1 and runs its MFMAs.
  // The scheduling barriers keep the loads at the start of the step and every
  // MFMA ahead of the wait for them, so that the loads overlap the products.
  dload(0, 0);
  asm volatile("s_waitcnt vmcnt(0)" ::: "memory");
  __syncthreads();
  for (int kt = 0; kt < nk; ++kt) {
    const int buf = kt & 1;
    const unsigned char* sb = smem + buf * QSTAGE;
    dload(buf ^ 1, kt + 1 < nk ? kt + 1 : kt);
    __builtin_amdgcn_sched_barrier(0);
    v4i fa[NS][2], fb[NS][2];
#pragma unroll
    for (int p = 0; p < NS; ++p)
#pragma unroll
      for (int i = 0; i < 2; ++i) {
        fa[p][i] = *(const v4i*)(sb + p * QPLANE + ra0 + i * 16 * QROW);
        fb[p][i] = *(const v4i*)(sb + p * QPLANE + rb0 + i * 16 * QROW);
      }
#pragma unroll
    for (int k = 0; k < NS; ++k)
#pragma unroll
      for (int l = 0; l < NS; ++l) {
        if (k + l > NS - 1) continue;   // weights 2^-7(k + l + 2) down to 2^-42 kept
#pragma unroll
        for (int i = 0; i < 2; ++i)
#pragma unroll
          for (int j = 0; j < 2; ++j)
            acc[k + l][i][j] = __builtin_amdgcn_mfma_i32_16x16x64_i8(fa[k][i], fb[l][j], acc[k + l][i][j], 0, 0, 0);
      }
    __builtin_amdgcn_sched_barrier(0);
    asm volatile("s_waitcnt vmcnt(0)" ::: "memory");
    __syncthreads();
  }

  // float64 values of the block results: sum over k + l, then the row and
  // column scales 2^(e_i + f_j) and the launch's operand scale
  v4d dd[2][2];
#pragma unroll
  for (int i = 0; i < 2; ++i)
#pragma unroll
    for (int j = 0; j < 2; ++j)
#pragma unroll
      for (int r = 0; r < 4; ++r) {
        double v = 0.0;
#pragma unroll
        for (int gq = NG - 1; gq >= 0; --gq) v += ldexp((double)acc[gq][i][j][r], -7 * (gq + 2));
        const int row = tile_m * QT + wm * 32 + i * 16 + MI8::row_in_block(lg, r);
        const int col = tile_n * QT + wn * 32 + j * 16 + lr;
        const int e = ea[row], f = eb[col];
        dd[i][j][r] = (e == I8_NONFINITE || f == I8_NONFINITE) ? __builtin_nan("") : ldexp(v, e + f) * scale;
      }
  epilogue_bands<double, QT, QT, 2, 2, MI8, v4d, 2, 2>(P, np, tile_m, tile_n, dd, (double*)smem);
}

}  // namespace

size_t i8x5_scratch_bytes(int64_t np) {
  const size_t planes = (size_t)NS * (size_t)np * (size_t)np;
  return 2 * align_up(planes, 256) + 2 * align_up((size_t)np * 4, 256) + align_up((size_t)np * 8, 256);
}

sincosm_status launch_gemm_i8x5(const GemmLaunch& g, void* scratch, hipStream_t stream) {
  const int np = g.np;
  if (!scratch || np <= 0 || np % QT != 0 || np > 16384) return SINCOSM_E_UNSUPPORTED;
  // one problem, or (device-planned, select) alternatives of which the plan
  // record picks one; each a single k segment
  if (g.nprob < 1 || g.nprob > MAX_PROB || (g.nprob > 1 && !(g.cond.plan && g.cond.select)))
    return SINCOSM_E_UNSUPPORTED;
  I8Operands op;
  op.cond = g.cond;
  op.nprob = g.nprob;
  for (int q = 0; q < g.nprob; ++q) {
    if (g.prob[q].nseg != 1) return SINCOSM_E_UNSUPPORTED;
    const Seg& sg = g.prob[q].seg[0];
    op.L[q] = (const double*)sg.L;
    op.R[q] = (const double*)sg.R;
    op.ldl[q] = sg.ldl;
    op.ldr[q] = sg.ldr;
  }
  const size_t planes = (size_t)NS * (size_t)np * (size_t)np;
  char* base = (char*)scratch;
  int8_t* Ap = (int8_t*)base;
  int8_t* Bp = (int8_t*)(base + align_up(planes, 256));
  int* ea = (int*)(base + 2 * align_up(planes, 256));
  int* eb = (int*)((char*)ea + align_up((size_t)np * 4, 256));
  unsigned long long* cmax = (unsigned long long*)((char*)eb + align_up((size_t)np * 4, 256));
  slice_rows_kernel<<<np, 256, 0, stream>>>(op, np, Ap, ea);
  zero_u64_kernel<<<(np + 255) / 256, 256, 0, stream>>>(cmax, np);
  dim3 gb(np / 64, np / 64);
  col_max_kernel<<<gb, 256, 0, stream>>>(op, cmax);
  slice_cols_kernel<<<gb, 256, 0, stream>>>(op, np, cmax, Bp, eb);
  const int tiles = np / QT;
  gemm_i8x5_kernel<<<tiles * tiles, QTHR, 0, stream>>>(Ap, Bp, ea, eb, g);
  SC_HIP(hipGetLastError());
  return SINCOSM_OK;
}

}  // namespace sc
