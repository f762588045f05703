// 1-norm, padded copy, plan and small elementwise kernels.
//
// The 1-norm (maximum absolute column sum) drives the choice of scheme and
// scaling (Section 3 bounds in terms of theta = ||A||, Tables 1-2, and the
// 1-norm named in Section 4). It is computed in float64 with a fixed
// summation order, so the plan is reproducible bit for bit:
//   stage 1: each block sums |a_ij| down a chunk of NORM_ROWS rows for 256
//            columns, writing one partial per (chunk, column), and writes the
//            zero-padded copy of the same elements;
//   stage 2: each column adds its partials in chunk order, and the maximum
//            over columns is taken with an integer atomicMax on the float64
//            bit pattern (order-independent, so still deterministic; NaN and
//            Inf patterns compare above every finite value);
//   stage 3: the block of stage 2 that finishes last applies the plan rule.
#include "common.hpp"

namespace sc {

constexpr int NORM_ROWS = 64;
constexpr int NORM_COLS = 256;

size_t norm_scratch_bytes(int64_t np) {
  const int64_t nchunks = (np + NORM_ROWS - 1) / NORM_ROWS;
  return align_up(sizeof(sincosm_plan), 256) + 256 + align_up((size_t)nchunks * np * sizeof(double), 256);
}

NormScratch norm_scratch(void* base, int64_t np) {
  NormScratch s;
  char* p = (char*)base;
  s.plan = (sincosm_plan*)p;
  p += align_up(sizeof(sincosm_plan), 256);
  s.maxbits = (unsigned long long*)p;
  p += 256;
  s.partial = (double*)p;
  s.nchunks = (int)((np + NORM_ROWS - 1) / NORM_ROWS);
  return s;
}

// counter (nullable): the block count of the fused stage 2 + 3 kernel, reset here.
template <typename TS, typename TD>
__global__ __launch_bounds__(NORM_COLS) void norm_copy_kernel(int64_t n, int64_t np, const TS* __restrict__ A,
                                                             int64_t lda, double pre, TD* __restrict__ Ap,
                                                             double* __restrict__ partial,
                                                             unsigned long long* maxbits,
                                                             unsigned int* counter = nullptr) {
  const int64_t j = (int64_t)blockIdx.x * NORM_COLS + threadIdx.x;
  const int64_t i0 = (int64_t)blockIdx.y * NORM_ROWS;
  if (blockIdx.x == 0 && blockIdx.y == 0 && threadIdx.x == 0) {
    *maxbits = 0ull;
    if (counter) *counter = 0u;
  }
  if (j >= np) return;
  double sum = 0.0;
  const int64_t i1 = i0 + NORM_ROWS < np ? i0 + NORM_ROWS : np;
  // rows in groups of U: the group's loads are issued together (two memory
  // round trips per chunk), then added in row order (the same sum as one row
  // at a time)
  constexpr int U = NORM_ROWS / 2;
  for (int64_t ib = i0; ib < i1; ib += U) {
    double v[U];
#pragma unroll
    for (int u = 0; u < U; ++u) {
      const int64_t i = ib + u;
      v[u] = (i < i1 && i < n && j < n) ? (double)A[i * lda + j] * pre : 0.0;
    }
#pragma unroll
    for (int u = 0; u < U; ++u) {
      const int64_t i = ib + u;
      if (i < i1) {
        if (Ap) Ap[i * np + j] = (TD)v[u];
        sum += fabs(v[u]);
      }
    }
  }
  partial[(int64_t)blockIdx.y * np + j] = sum;
}

__global__ __launch_bounds__(NORM_COLS) void norm_reduce_kernel(int64_t np, int nchunks,
                                                               const double* __restrict__ partial,
                                                               unsigned long long* maxbits) {
  __shared__ unsigned long long red[NORM_COLS];
  const int64_t j = (int64_t)blockIdx.x * NORM_COLS + threadIdx.x;
  unsigned long long bits = 0ull;
  if (j < np) {
    // chunk partials in chunk order, loads issued in groups of 8
    double s = 0.0;
    for (int c0 = 0; c0 < nchunks; c0 += 8) {
      double v[8];
#pragma unroll
      for (int u = 0; u < 8; ++u) v[u] = c0 + u < nchunks ? partial[(int64_t)(c0 + u) * np + j] : 0.0;
#pragma unroll
      for (int u = 0; u < 8; ++u)
        if (c0 + u < nchunks) s += v[u];
    }
    bits = (unsigned long long)__double_as_longlong(s);
  }
  red[threadIdx.x] = bits;
  __syncthreads();
  for (int w = NORM_COLS / 2; w > 0; w >>= 1) {
    if ((int)threadIdx.x < w) {
      const unsigned long long o = red[threadIdx.x + w];
      if (o > red[threadIdx.x]) red[threadIdx.x] = o;
    }
    __syncthreads();
  }
  if (threadIdx.x == 0) atomicMax(maxbits, red[0]);
}

// Stages 2 and 3 in one launch: the column sums and their maximum as in
// norm_reduce_kernel; the block that finishes last (a device-scope counter,
// reset by norm_copy_kernel) reads the maximum and applies the plan rule as
// plan_kernel does.
__global__ __launch_bounds__(NORM_COLS) void norm_reduce_plan_kernel(int64_t np, int nchunks,
                                                                    const double* __restrict__ partial,
                                                                    unsigned long long* maxbits,
                                                                    unsigned int* counter, int acc, int mode,
                                                                    sincosm_plan* plan, int s_max,
                                                                    sincosm_plan* plan_dev) {
  __shared__ unsigned long long red[NORM_COLS];
  __shared__ int last;
  const int64_t j = (int64_t)blockIdx.x * NORM_COLS + threadIdx.x;
  unsigned long long bits = 0ull;
  if (j < np) {
    // chunk partials in chunk order, loads issued in groups of 8
    double s = 0.0;
    for (int c0 = 0; c0 < nchunks; c0 += 8) {
      double v[8];
#pragma unroll
      for (int u = 0; u < 8; ++u) v[u] = c0 + u < nchunks ? partial[(int64_t)(c0 + u) * np + j] : 0.0;
#pragma unroll
      for (int u = 0; u < 8; ++u)
        if (c0 + u < nchunks) s += v[u];
    }
    bits = (unsigned long long)__double_as_longlong(s);
  }
  red[threadIdx.x] = bits;
  __syncthreads();
  for (int w = NORM_COLS / 2; w > 0; w >>= 1) {
    if ((int)threadIdx.x < w) {
      const unsigned long long o = red[threadIdx.x + w];
      if (o > red[threadIdx.x]) red[threadIdx.x] = o;
    }
    __syncthreads();
  }
  if (threadIdx.x == 0) {
    atomicMax(maxbits, red[0]);
    __threadfence();
    last = atomicAdd(counter, 1u) == gridDim.x - 1;
  }
  __syncthreads();
  if (!last || threadIdx.x != 0) return;
  __threadfence();
  const double nrm = __longlong_as_double((long long)atomicMax(maxbits, 0ull));   // the final maximum
  sincosm_plan p;
  if (mode == 1) plan_rule_wave(nrm, acc, &p);
  else plan_rule(nrm, acc, &p);
  if (s_max >= 0 && p.status == SINCOSM_OK && p.s > s_max) p.status = SINCOSM_E_SCALING;
  *plan = p;
  if (plan_dev) *plan_dev = p;
}

__global__ void plan_sq_kernel(const unsigned long long* maxbits, int acc, sincosm_plan* plan) {
  if (threadIdx.x != 0 || blockIdx.x != 0) return;
  const double t1 = __longlong_as_double((long long)maxbits[0]);
  const double t2 = __longlong_as_double((long long)maxbits[1]);
  const double big = 1.7976931348623157e308;
  double t = t1;
  int y_ok = 0;
  if (t1 >= 0.0 && t1 <= big && t2 >= 0.0 && t2 <= big) {
    const double r = sqrt(t2);
    t = r < t1 ? r : t1;
    y_ok = 1;
  }
  sincosm_plan p;
  plan_rule(t, acc, &p);
  plan[0] = p;
  sincosm_plan q;
  q.level = y_ok; q.s = 0; q.products = 0; q.status = 0; q.norm1 = t2;
  plan[1] = q;
}

sincosm_status launch_norm_sq_plan(int64_t n, int64_t np, const void* Y, bool y_f64, int acc,
                                   const NormScratch& ns, hipStream_t stream) {
  dim3 g1((unsigned)((np + NORM_COLS - 1) / NORM_COLS), (unsigned)ns.nchunks);
  if (y_f64)
    norm_copy_kernel<double, double><<<g1, NORM_COLS, 0, stream>>>(n, np, (const double*)Y, np, 1.0, nullptr,
                                                                   ns.partial, ns.maxbits + 1);
  else
    norm_copy_kernel<float, double><<<g1, NORM_COLS, 0, stream>>>(n, np, (const float*)Y, np, 1.0, nullptr,
                                                                  ns.partial, ns.maxbits + 1);
  dim3 g2((unsigned)((np + NORM_COLS - 1) / NORM_COLS));
  norm_reduce_kernel<<<g2, NORM_COLS, 0, stream>>>(np, ns.nchunks, ns.partial, ns.maxbits + 1);
  plan_sq_kernel<<<1, 64, 0, stream>>>(ns.maxbits, acc, ns.plan);
  SC_HIP(hipGetLastError());
  return SINCOSM_OK;
}

template <typename TS, typename TD>
static void launch_norm_t(int64_t n, int64_t np, const void* A, int64_t lda, void* Ap, const NormScratch& ns,
                          int acc, int mode, double pre, int s_max, sincosm_plan* plan_dev, hipStream_t stream) {
  unsigned int* counter = (unsigned int*)(ns.maxbits + 2);
  dim3 g1((unsigned)((np + NORM_COLS - 1) / NORM_COLS), (unsigned)ns.nchunks);
  norm_copy_kernel<TS, TD><<<g1, NORM_COLS, 0, stream>>>(n, np, (const TS*)A, lda, pre, (TD*)Ap,
                                                         ns.partial, ns.maxbits, counter);
  dim3 g2((unsigned)((np + NORM_COLS - 1) / NORM_COLS));
  norm_reduce_plan_kernel<<<g2, NORM_COLS, 0, stream>>>(np, ns.nchunks, ns.partial, ns.maxbits, counter, acc,
                                                        mode, ns.plan, s_max, plan_dev);
}

sincosm_status launch_norm_copy_plan(int64_t n, int64_t np, const void* A, int64_t lda, bool src_f64, void* Ap,
                                     bool dst_f64, int acc, const NormScratch& ns, hipStream_t stream, int mode,
                                     double pre, int s_max, sincosm_plan* plan_dev) {
  if (src_f64 && dst_f64)
    launch_norm_t<double, double>(n, np, A, lda, Ap, ns, acc, mode, pre, s_max, plan_dev, stream);
  else if (src_f64 && !dst_f64)
    launch_norm_t<double, float>(n, np, A, lda, Ap, ns, acc, mode, pre, s_max, plan_dev, stream);
  else if (!src_f64 && dst_f64)
    launch_norm_t<float, double>(n, np, A, lda, Ap, ns, acc, mode, pre, s_max, plan_dev, stream);
  else
    launch_norm_t<float, float>(n, np, A, lda, Ap, ns, acc, mode, pre, s_max, plan_dev, stream);
  SC_HIP(hipGetLastError());
  return SINCOSM_OK;
}

// Tiled transpose with zero padding: dst[j][i] = src[i][j] for i, j < n.
template <typename TS, typename TD>
__global__ __launch_bounds__(256) void transpose_pad_kernel(int64_t n, int64_t np, const TS* __restrict__ src,
                                                           int64_t lds, TD* __restrict__ dst) {
  __shared__ double tile[32][33];
  const int64_t bi = (int64_t)blockIdx.y * 32, bj = (int64_t)blockIdx.x * 32;
  const int tx = threadIdx.x & 31, ty = threadIdx.x >> 5;  // 32 x 8
  for (int r = ty; r < 32; r += 8) {
    const int64_t i = bi + r, j = bj + tx;
    tile[r][tx] = (i < n && j < n) ? (double)src[i * lds + j] : 0.0;
  }
  __syncthreads();
  for (int r = ty; r < 32; r += 8) {
    const int64_t i = bj + r, j = bi + tx;  // dst row i = src column
    if (i < np && j < np) dst[i * np + j] = (TD)tile[tx][r];
  }
}

sincosm_status launch_transpose_pad(int64_t n, int64_t np, const void* src, int64_t lds, bool src_f64, void* dst,
                                    bool dst_f64, hipStream_t stream) {
  dim3 g((unsigned)((np + 31) / 32), (unsigned)((np + 31) / 32));
  if (src_f64 && dst_f64)
    transpose_pad_kernel<double, double><<<g, 256, 0, stream>>>(n, np, (const double*)src, lds, (double*)dst);
  else if (src_f64)
    transpose_pad_kernel<double, float><<<g, 256, 0, stream>>>(n, np, (const double*)src, lds, (float*)dst);
  else if (dst_f64)
    transpose_pad_kernel<float, double><<<g, 256, 0, stream>>>(n, np, (const float*)src, lds, (double*)dst);
  else
    transpose_pad_kernel<float, float><<<g, 256, 0, stream>>>(n, np, (const float*)src, lds, (float*)dst);
  SC_HIP(hipGetLastError());
  return SINCOSM_OK;
}

template <typename TS, typename TD>
__global__ __launch_bounds__(256) void convert_pad_kernel(int64_t n, int64_t np, const TS* __restrict__ src,
                                                         int64_t lds, TD* __restrict__ dst) {
  const int64_t j = (int64_t)blockIdx.x * 256 + threadIdx.x;
  const int64_t i = blockIdx.y;
  if (j >= np) return;
  dst[i * np + j] = (TD)((i < n && j < n) ? (double)src[i * lds + j] : 0.0);
}

sincosm_status launch_convert_pad(int64_t n, int64_t np, const void* src, int64_t lds, bool src_f64, void* dst,
                                  bool dst_f64, hipStream_t stream) {
  dim3 g((unsigned)((np + 255) / 256), (unsigned)np);
  if (src_f64 && dst_f64)
    convert_pad_kernel<double, double><<<g, 256, 0, stream>>>(n, np, (const double*)src, lds, (double*)dst);
  else if (src_f64)
    convert_pad_kernel<double, float><<<g, 256, 0, stream>>>(n, np, (const double*)src, lds, (float*)dst);
  else if (dst_f64)
    convert_pad_kernel<float, double><<<g, 256, 0, stream>>>(n, np, (const float*)src, lds, (double*)dst);
  else
    convert_pad_kernel<float, float><<<g, 256, 0, stream>>>(n, np, (const float*)src, lds, (float*)dst);
  SC_HIP(hipGetLastError());
  return SINCOSM_OK;
}

sincosm_status launch_fill_zero(int64_t np, void* X, bool f64, hipStream_t stream) {
  // convert_pad with an empty source writes zeros over the whole np x np buffer
  return launch_convert_pad(0, np, X, np, f64, X, f64, stream);
}

template <typename T>
__global__ __launch_bounds__(256) void fill_nan_kernel(int64_t cols, T* X, int64_t ld) {
  const int64_t j = (int64_t)blockIdx.x * 256 + threadIdx.x;
  const int64_t i = blockIdx.y;
  if (j < cols) X[i * ld + j] = (T)__longlong_as_double(0x7ff8000000000000ll);
}

sincosm_status launch_fill_nan_rect(int64_t rows, int64_t cols, void* X, int64_t ld, bool f64,
                                    hipStream_t stream) {
  if (rows <= 0 || cols <= 0) return SINCOSM_OK;
  dim3 g((unsigned)((cols + 255) / 256), (unsigned)rows);
  if (f64) fill_nan_kernel<double><<<g, 256, 0, stream>>>(cols, (double*)X, ld);
  else fill_nan_kernel<float><<<g, 256, 0, stream>>>(cols, (float*)X, ld);
  SC_HIP(hipGetLastError());
  return SINCOSM_OK;
}

sincosm_status launch_fill_nan(int64_t n, void* X, int64_t ld, bool f64, hipStream_t stream) {
  return launch_fill_nan_rect(n, n, X, ld, f64, stream);
}

// A caller's plan covers A when ||A||_1 2^-s <= theta of its level (the
// bounds of Tables 1-2 the plan rule uses).
__global__ void check_plan_kernel(const unsigned long long* maxbits, int acc, int level, int s,
                                  sincosm_plan* plan, sincosm_plan* plan_dev) {
  if (threadIdx.x != 0 || blockIdx.x != 0) return;
  const double nrm = __longlong_as_double((long long)*maxbits);
  sincosm_plan p;
  p.level = level;
  p.s = s;
  p.products = level + 2 * s;
  p.norm1 = nrm;
  const int base = acc & 1;
  const double th = level == 5 ? plan_theta_level5(base)
                               : plan_theta(base, level == 3 ? 0 : level == 4 ? 1 : level == 6 ? 2 : 3);
  if (!(nrm >= 0.0 && nrm <= 1.7976931348623157e308)) p.status = SINCOSM_E_NONFINITE;
  else p.status = ldexp(nrm, -s) <= th ? SINCOSM_OK : SINCOSM_E_PLAN;
  *plan = p;
  if (plan_dev) *plan_dev = p;
}

sincosm_status launch_check_plan(int acc, int level, int s, const NormScratch& ns, sincosm_plan* plan_dev,
                                 hipStream_t stream) {
  check_plan_kernel<<<1, 64, 0, stream>>>(ns.maxbits, acc, level, s, ns.plan, plan_dev);
  SC_HIP(hipGetLastError());
  return SINCOSM_OK;
}

// After s double-angle steps the pair (C, S) sits in (q1, q0) for even s and
// in (q3, q2) for odd s (the scheme writes (q1, q0), step i writes the other
// pair of the two). Copies rows of both into the caller's matrices, S
// multiplied by ss (1 copies exactly), or fills them with NaN when the plan
// record's status is not SINCOSM_OK. CPLX: one interleaved complex matrix
// U = C + i ss S at C (leading dimension ldc in complex elements).
template <typename T, bool CPLX>
__global__ __launch_bounds__(256) void copy_result_kernel(const sincosm_plan* plan, int64_t n, int64_t np,
                                                          const T* q0, const T* q1, const T* q2, const T* q3,
                                                          T* C, int64_t ldc, T* S, int64_t lds, T ss) {
  typedef T v2 __attribute__((ext_vector_type(2)));
  const bool ok = plan->status == SINCOSM_OK;
  const bool odd = (plan->s & 1) != 0;
  const T* srcC = odd ? q3 : q1;
  const T* srcS = odd ? q2 : q0;
  const int64_t j = (int64_t)blockIdx.x * 256 + threadIdx.x;
  const int64_t i = blockIdx.y;
  if (j < n) {
    const T nan = (T)__longlong_as_double(0x7ff8000000000000ll);
    const T c = ok ? srcC[i * np + j] : nan;
    const T sv = ok ? ss * srcS[i * np + j] : nan;
    if (CPLX) {
      v2 v;
      v.x = c;
      v.y = sv;
      *(v2*)(C + 2 * (i * ldc + j)) = v;
    } else {
      C[i * ldc + j] = c;
      S[i * lds + j] = sv;
    }
  }
}

sincosm_status launch_copy_result(const sincosm_plan* plan, int64_t n, int64_t np, void* const q[4], void* C,
                                  int64_t ldc, void* S, int64_t lds, bool f64, hipStream_t stream, double ss) {
  if (n <= 0) return SINCOSM_OK;
  dim3 g((unsigned)((n + 255) / 256), (unsigned)n);
  if (f64)
    copy_result_kernel<double, false><<<g, 256, 0, stream>>>(plan, n, np, (const double*)q[0],
                                                             (const double*)q[1], (const double*)q[2],
                                                             (const double*)q[3], (double*)C, ldc, (double*)S,
                                                             lds, ss);
  else
    copy_result_kernel<float, false><<<g, 256, 0, stream>>>(plan, n, np, (const float*)q[0], (const float*)q[1],
                                                            (const float*)q[2], (const float*)q[3], (float*)C,
                                                            ldc, (float*)S, lds, (float)ss);
  SC_HIP(hipGetLastError());
  return SINCOSM_OK;
}

sincosm_status launch_copy_result_complex(const sincosm_plan* plan, int64_t n, int64_t np, void* const q[4],
                                          void* U, int64_t ldu, double ss, bool f64, hipStream_t stream) {
  if (n <= 0) return SINCOSM_OK;
  dim3 g((unsigned)((n + 255) / 256), (unsigned)n);
  if (f64)
    copy_result_kernel<double, true><<<g, 256, 0, stream>>>(plan, n, np, (const double*)q[0],
                                                            (const double*)q[1], (const double*)q[2],
                                                            (const double*)q[3], (double*)U, ldu, nullptr, 0,
                                                            ss);
  else
    copy_result_kernel<float, true><<<g, 256, 0, stream>>>(plan, n, np, (const float*)q[0], (const float*)q[1],
                                                           (const float*)q[2], (const float*)q[3], (float*)U,
                                                           ldu, nullptr, 0, (float)ss);
  SC_HIP(hipGetLastError());
  return SINCOSM_OK;
}

// Device-planned reverse pass and block propagator: copy the pair (x0, x1) of
// np x np matrices (count 8-byte words each) into (y0, y1) when the plan
// record's s is odd and its status is SINCOSM_OK, so that the pair a
// ping-pong sequence ends on is found at (y0, y1) whatever the parity of s.
__global__ __launch_bounds__(256) void copy_pair_if_odd_kernel(const sincosm_plan* plan, int64_t count,
                                                               const double* x0, const double* x1, double* y0,
                                                               double* y1) {
  if (plan->status != SINCOSM_OK || (plan->s & 1) == 0) return;
  const int64_t e = (int64_t)blockIdx.x * 256 + threadIdx.x;
  if (e < count) {
    y0[e] = x0[e];
    y1[e] = x1[e];
  }
}

sincosm_status launch_copy_pair_if_odd(const sincosm_plan* plan, int64_t np, const void* x0, const void* x1,
                                       void* y0, void* y1, hipStream_t stream, size_t es) {
  const int64_t bytes = np * np * (int64_t)es;
  if (bytes <= 0) return SINCOSM_OK;
  if (bytes % 8) return SINCOSM_E_ARG;
  const int64_t count = bytes / 8;
  copy_pair_if_odd_kernel<<<(unsigned)((count + 255) / 256), 256, 0, stream>>>(
      plan, count, (const double*)x0, (const double*)x1, (double*)y0, (double*)y1);
  SC_HIP(hipGetLastError());
  return SINCOSM_OK;
}

// X *= 2^(-k s) for the plan record's s, in place over count elements, when
// the record's status is SINCOSM_OK (an exact scaling for normal results).
template <typename T>
__global__ __launch_bounds__(256) void scale_by_plan_kernel(const sincosm_plan* plan, int k, int64_t count,
                                                            T* X) {
  if (plan->status != SINCOSM_OK || plan->s == 0) return;
  const int e2 = -k * plan->s;
  const int64_t e = (int64_t)blockIdx.x * 256 + threadIdx.x;
  if (e < count) X[e] = ldexp(X[e], e2);
}

sincosm_status launch_scale_by_plan(const sincosm_plan* plan, int k, void* X, int64_t count, bool f64,
                                    hipStream_t stream) {
  if (count <= 0) return SINCOSM_OK;
  const unsigned g = (unsigned)((count + 255) / 256);
  if (f64) scale_by_plan_kernel<double><<<g, 256, 0, stream>>>(plan, k, count, (double*)X);
  else scale_by_plan_kernel<float><<<g, 256, 0, stream>>>(plan, k, count, (float*)X);
  SC_HIP(hipGetLastError());
  return SINCOSM_OK;
}

template <typename T>
__global__ __launch_bounds__(256) void fill_nan_if_kernel(const sincosm_plan* plan, int64_t cols, T* X,
                                                          int64_t ld) {
  if (plan->status == SINCOSM_OK) return;
  const int64_t j = (int64_t)blockIdx.x * 256 + threadIdx.x;
  const int64_t i = blockIdx.y;
  if (j < cols) X[i * ld + j] = (T)__longlong_as_double(0x7ff8000000000000ll);
}

sincosm_status launch_fill_nan_if_rect(const sincosm_plan* plan, int64_t rows, int64_t cols, void* X, int64_t ld,
                                       bool f64, hipStream_t stream) {
  if (rows <= 0 || cols <= 0) return SINCOSM_OK;
  dim3 g((unsigned)((cols + 255) / 256), (unsigned)rows);
  if (f64) fill_nan_if_kernel<double><<<g, 256, 0, stream>>>(plan, cols, (double*)X, ld);
  else fill_nan_if_kernel<float><<<g, 256, 0, stream>>>(plan, cols, (float*)X, ld);
  SC_HIP(hipGetLastError());
  return SINCOSM_OK;
}

sincosm_status launch_fill_nan_if(const sincosm_plan* plan, int64_t n, void* X, int64_t ld, bool f64,
                                  hipStream_t stream) {
  return launch_fill_nan_if_rect(plan, n, n, X, ld, f64, stream);
}

// dst[i][j] = (re[i][j], sgn * im[i][j]) for i, j < n: interleaved complex
// (real, imaginary) pairs from two zero-padded planes of the same type.
template <typename T>
__global__ __launch_bounds__(256) void interleave_kernel(int64_t n, int64_t np, const T* __restrict__ re,
                                                        const T* __restrict__ im, T sgn, T* __restrict__ dst,
                                                        int64_t ldd) {
  typedef T v2 __attribute__((ext_vector_type(2)));
  const int64_t j = (int64_t)blockIdx.x * 256 + threadIdx.x;
  const int64_t i = blockIdx.y;
  if (j < n) {
    v2 v;
    v.x = re[i * np + j];
    v.y = sgn * im[i * np + j];
    *(v2*)(dst + 2 * (i * ldd + j)) = v;
  }
}

sincosm_status launch_interleave(int64_t n, int64_t np, const void* re, const void* im, bool negate_im,
                                 void* dst, int64_t ldd, bool f64, hipStream_t stream) {
  if (n <= 0) return SINCOSM_OK;
  dim3 g((unsigned)((n + 255) / 256), (unsigned)n);
  if (f64)
    interleave_kernel<double><<<g, 256, 0, stream>>>(n, np, (const double*)re, (const double*)im,
                                                     negate_im ? -1.0 : 1.0, (double*)dst, ldd);
  else
    interleave_kernel<float><<<g, 256, 0, stream>>>(n, np, (const float*)re, (const float*)im,
                                                    negate_im ? -1.0f : 1.0f, (float*)dst, ldd);
  SC_HIP(hipGetLastError());
  return SINCOSM_OK;
}

}  // namespace sc
