// Internal declarations shared by the library's translation units.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>
#include <stddef.h>

#include "sincosm.h"

namespace sc {

// ----------------------------------------------------------------------------
// Status helpers
// ----------------------------------------------------------------------------
#define SC_HIP(expr)                                   \
  do {                                                 \
    hipError_t e_ = (expr);                            \
    if (e_ != hipSuccess) return SINCOSM_E_HIP;        \
  } while (0)

#define SC_TRY(expr)                                   \
  do {                                                 \
    sincosm_status st_ = (expr);                       \
    if (st_ != SINCOSM_OK) return st_;                 \
  } while (0)

inline size_t align_up(size_t x, size_t a) { return (x + a - 1) / a * a; }

// ----------------------------------------------------------------------------
// Plan rule (host and device share the constants through this header only
// within the library; the oracle keeps its own copy).
// ----------------------------------------------------------------------------
// min(theta^c, theta^s) per scheme with 3, 4, 6, 7 products: Table 1 (u = 2^-53)
// and Table 2 (u = 2^-24). The 7-product double bound is 1.8548: the sine's
// printed 1.97 is not reproduced by the printed coefficients.
__host__ __device__ inline double plan_theta(int acc, int idx) {
  const double dbl[4] = {6.5633e-3, 8.0438e-2, 9.8108e-1, 1.8548};
  const double sgl[4] = {1.8709e-1, 7.492e-1, 2.9935, 4.3819};
  return acc == SINCOSM_ACC_SINGLE ? sgl[idx] : dbl[idx];
}

// Combined bound of the 5-product scheme (Algorithm4cA cosine, Algorithm5sA
// sine): its sine bound is the larger, so it is the printed T^c_8 bound of
// Tables 1-2. Used only when the caller asks for the extended plan.
__host__ __device__ inline double plan_theta_level5(int acc) {
  return (acc & 1) == SINCOSM_ACC_SINGLE ? 8.5756e-1 : 1.1495e-1;
}

// Accuracy argument check: DOUBLE or SINGLE, optionally with the plan flags in `allowed`.
inline bool acc_valid(int acc, int allowed) {
  const int base = acc & ~allowed;
  return base == SINCOSM_ACC_DOUBLE || base == SINCOSM_ACC_SINGLE;
}

// Fills level, s, products, status; norm1 is stored as given. `acc` may carry
// SINCOSM_PLAN_EXTENDED (the 5-product scheme joins the candidates).
__host__ __device__ inline void plan_rule(double norm1, int acc, sincosm_plan* p) {
  const int levels[5] = {3, 4, 6, 7, 5};
  const int base = acc & 1;
  const int nlev = (acc & SINCOSM_PLAN_EXTENDED) ? 5 : 4;
  p->norm1 = norm1;
  if (!(norm1 >= 0.0 && norm1 <= 1.7976931348623157e308)) {  // NaN, negative or +Inf
    p->level = 0; p->s = 0; p->products = 0; p->status = SINCOSM_E_NONFINITE;
    return;
  }
  int best_cost = 0x7fffffff, best_s = 0, best_level = 3;
  for (int i = 0; i < nlev; ++i) {
    const double th = i < 4 ? plan_theta(base, i) : plan_theta_level5(base);
    int s = 0;
    double t = norm1;
    while (t > th) { t *= 0.5; ++s; }     // exact halving: no log2 rounding
    const int cost = levels[i] + 2 * s;
    if (cost < best_cost || (cost == best_cost && s < best_s)) {
      best_cost = cost; best_s = s; best_level = levels[i];
    }
  }
  p->level = best_level; p->s = best_s; p->products = best_cost; p->status = SINCOSM_OK;
}

// Wave-equation functions c(t^2 A), s(t, A) (Section 2.2): schemes with 2, 3,
// 4, 5 products in B = t^2 A; bounds on ||B||_1 derived from the scheme
// polynomials as for Tables 1-2 (the cosine bound is the square of the cos
// table's), rounded down to 5 digits. Halving t quarters B.
__host__ __device__ inline double wave_theta(int acc, int idx) {
  const double dbl[4] = {3.4458e-3, 1.3213e-2, 9.6251e-1, 3.6404};
  const double sgl[4] = {5.2237e-1, 7.354e-1, 8.9612, 2.1848e1};
  return acc == SINCOSM_ACC_SINGLE ? sgl[idx] : dbl[idx];
}

__host__ __device__ inline void plan_rule_wave(double normB, int acc, sincosm_plan* p) {
  p->norm1 = normB;
  if (!(normB >= 0.0 && normB <= 1.7976931348623157e308)) {
    p->level = 0; p->s = 0; p->products = 0; p->status = SINCOSM_E_NONFINITE;
    return;
  }
  int best_cost = 0x7fffffff, best_s = 0, best_level = 2;
  for (int i = 0; i < 4; ++i) {
    const double th = wave_theta(acc, i);
    int s = 0;
    double t = normB;
    while (t > th) { t *= 0.25; ++s; }
    const int cost = (2 + i) + 2 * s;
    if (cost < best_cost || (cost == best_cost && s < best_s)) {
      best_cost = cost; best_s = s; best_level = 2 + i;
    }
  }
  p->level = best_level; p->s = best_s; p->products = best_cost; p->status = SINCOSM_OK;
}

// ----------------------------------------------------------------------------
// GEMM-with-epilogue descriptors.
//
// One launch computes, for each problem p in [0, nprob) and each output tile,
//   D = sum_seg scale_seg * L_seg R_seg          (K = kdim per segment)
// and writes every output o of the problem as
//   O_o = e_o D + sum_q c_oq M_q + d_o [i == j < nvalid]
// where M_q are same-position tiles of the problem's inputs. Outputs are
// stored only where row < lim_o and col < lim_o; internal (padded) buffers
// use lim = padded size so their padding stays exactly zero.
// ----------------------------------------------------------------------------
constexpr int MAX_SEG = 3;
constexpr int MAX_IN = 6;
constexpr int MAX_OUT = 6;
constexpr int MAX_PROB = 3;

struct Seg {
  const void* L;
  const void* R;
  int64_t ldl, ldr;
  double lscale;     // multiplies the left operand values as they are staged
  double rscale;     // multiplies the right operand values (powers of two or -1 keep it exact)
};

struct EpiIn {
  const void* p;
  int64_t ld;
};

struct EpiOut {
  void* p;
  int64_t ld;
  int32_t lim;
  int32_t f64;       // 1: store float64, 0: store the kernel's compute type
  double e, d;
  double c[MAX_IN];
};

struct Problem {
  int32_t nseg, nin, nout, nvalid;
  Seg seg[MAX_SEG];
  EpiIn in[MAX_IN];
  EpiOut out[MAX_OUT];
};

// Operand scale resolved on the device to 2^-s of the launch's plan record
// (a value no launch uses as a scale: scales are signed powers of two).
constexpr double SCALE_2_POW_MINUS_S = 3.0;

// A launch decided on the device by a plan record that an earlier kernel of
// the stream wrote (plan == nullptr: the launch always runs). Every workgroup
// returns at once when the record's status is not SINCOSM_OK, when level > 0
// and the record's level differs, or when step >= 0 and step >= the record's
// s. With select = 1 the launch's problems are alternatives for different
// levels: the grid covers the tiles of one problem, and it computes the
// problem q whose prob_level[q] is the record's level (none: nothing).
// Operand scales equal to SCALE_2_POW_MINUS_S become 2^-s.
struct DevCond {
  const sincosm_plan* plan;
  int32_t level;
  int32_t step;
  int32_t select;
  int32_t prob_level[MAX_PROB];
};

struct GemmLaunch {
  int32_t np;        // padded order (multiple of the tile); M = N = K = np per segment
  int32_t nprob;
  Problem prob[MAX_PROB];
  DevCond cond;
};

// Decision of a device-planned launch, taken by every workgroup at its start
// (uniform scalar loads of the plan record). Returns false when the launch
// does not apply; s and level receive the record's s and level.
__device__ inline bool cond_applies(const DevCond& c, int& s, int& level) {
  const int status = c.plan->status, ps = c.plan->s;
  level = c.plan->level;
  s = ps;
  if (status != SINCOSM_OK) return false;
  if (c.level > 0 && level != c.level) return false;
  if (c.step >= 0 && c.step >= ps) return false;
  return true;
}

// The launch's problem index and tile of this workgroup. A select launch
// (see DevCond) has the tiles of one problem and takes the problem of the
// plan's level (-1: none applies).
__device__ inline int cond_problem(const DevCond& c, int nprob, int level) {
  for (int q = 0; q < nprob; ++q)
    if (c.prob_level[q] == level) return q;
  return -1;
}

// An operand scale of a launch, with the device-resolved 2^-s substituted.
__host__ __device__ inline double resolve_scale(double v, int s) {
  return v == SCALE_2_POW_MINUS_S ? ldexp(1.0, -s) : v;
}

// Product arithmetic of one GEMM launch.
enum class Arith { F64, F32, BF16X3, I8X5 };

// Launch one GEMM-with-epilogue over all problems. `tile` selects the tile
// configuration (see gemm.hip); np must be a multiple of tile_size(tile).
// I8X5 (float64 storage, products on the int8 matrix cores) needs `scratch` of
// i8x5_scratch_bytes(np) bytes for its operand slices; launches without a
// product (epilogue only) run on the float64 kernel.
sincosm_status launch_gemm(Arith ar, int tile, const GemmLaunch& g, hipStream_t stream, void* scratch = nullptr);
size_t i8x5_scratch_bytes(int64_t np);
sincosm_status launch_gemm_i8x5(const GemmLaunch& g, void* scratch, hipStream_t stream);
// Output tile (64 or 32) of the batched kernel's products for padded order np,
// from the tuning table (64 where it has no entry).
int batched_tile(Arith ar, int64_t np);

// Product-kernel configurations the autotuner chooses among: tile rows and
// columns, k depth, wave grid, waves per SIMD, direct loads into LDS, k groups,
// and the launcher. Entries 0, 1, 2 are the defaults for the padding
// granularities 128, 64 and 32. cfg_table returns nullptr (count 0) for an
// arithmetic without a table.
typedef sincosm_status (*LaunchFn)(const GemmLaunch&, hipStream_t);
struct KernelCfg {
  int bm, bn, bk, wgm, wgn, wpe, dl, ks;
  LaunchFn fn;
};
const KernelCfg* cfg_table(Arith ar, int& count);
// Tuned configuration index for (arithmetic, launch class, padded order), or -1.
// Classes 1 and 2 fall back to class 0 entries; class 3 (the batched tile) does not.
int tuned_cfg(Arith ar, int cls, int64_t np);
int tile_size(int tile);
int choose_tile(Arith ar, int64_t n);
bool bf16x3_available();
sincosm_status launch_gemm_bf16x3(int tile, const GemmLaunch& g, hipStream_t stream);

// ----------------------------------------------------------------------------
// Norm / copy / plan / fill kernels (norm_plan.hip)
// ----------------------------------------------------------------------------
struct NormScratch {
  double* partial;        // [nchunks][np]
  unsigned long long* maxbits;
  sincosm_plan* plan;
  int nchunks;
};
size_t norm_scratch_bytes(int64_t np);
NormScratch norm_scratch(void* base, int64_t np);

// Column abs-sum partials of pre * A (A n x n, lda, type src_f64 ? double : float,
// each element multiplied by `pre` in float64) and the zero-padded copy
// Ap = pre * A (np x np, type dst_f64 ? double : float); then the plan:
// mode 0 the cos/sin rule, mode 1 the wave rule (pre = t^2, so the norm is ||B||_1).
// s_max >= 0 (device-planned calls): the plan's status becomes SINCOSM_E_SCALING
// when s > s_max; plan_dev (nullable) receives a copy of the plan record.
sincosm_status launch_norm_copy_plan(int64_t n, int64_t np, const void* A, int64_t lda, bool src_f64,
                                     void* Ap, bool dst_f64, int acc,
                                     const NormScratch& ns, hipStream_t stream, int mode = 0,
                                     double pre = 1.0, int s_max = -1, sincosm_plan* plan_dev = nullptr);
// dst (np x np, zero padded) = src^T for an n x n src.
// 1-norm of the np x np padded Y (its n x n part) into the second max slot, then
// the refined plan: theta' = min(||A||_1, ||Y||_1^(1/2)) when both are finite
// (else ||A||_1). plan[0] receives the plan, plan[1].level = 1 when Y is finite
// and may be reused as the scheme's first product.
sincosm_status launch_norm_sq_plan(int64_t n, int64_t np, const void* Y, bool y_f64, int acc,
                                   const NormScratch& ns, hipStream_t stream);
sincosm_status launch_transpose_pad(int64_t n, int64_t np, const void* src, int64_t lds, bool src_f64,
                                    void* dst, bool dst_f64, hipStream_t stream);
sincosm_status launch_fill_nan(int64_t n, void* X, int64_t ld, bool f64, hipStream_t stream);
// Check a caller's plan (level, s) against the 1-norm in ns (after
// launch_norm_copy_plan): writes the call's plan record to ns.plan and, when
// given, to plan_dev; status SINCOSM_E_PLAN when ||A||_1 2^-s > theta_level.
sincosm_status launch_check_plan(int acc, int level, int s, const NormScratch& ns, sincosm_plan* plan_dev,
                                 hipStream_t stream);
// Device-planned calls: copy the n x n result pair from the ping-pong buffers
// (np x np, the storage type) that hold it for the record's s into C and S
// (S multiplied by ss), or fill C and S with NaN when the record's status is
// not SINCOSM_OK.
sincosm_status launch_copy_result(const sincosm_plan* plan, int64_t n, int64_t np, void* const q[4], void* C,
                                  int64_t ldc, void* S, int64_t lds, bool f64, hipStream_t stream,
                                  double ss = 1.0);
// The same into one interleaved complex matrix U = C + i ss S (leading
// dimension ldu in complex elements), or NaN.
sincosm_status launch_copy_result_complex(const sincosm_plan* plan, int64_t n, int64_t np, void* const q[4],
                                          void* U, int64_t ldu, double ss, bool f64, hipStream_t stream);
// Copy the np x np pair (x0, x1) of es-byte elements into (y0, y1) when the
// plan record's s is odd and its status is SINCOSM_OK.
sincosm_status launch_copy_pair_if_odd(const sincosm_plan* plan, int64_t np, const void* x0, const void* x1,
                                       void* y0, void* y1, hipStream_t stream, size_t es = 8);
// X *= 2^(-k s) over count elements, s from the plan record (nothing when its
// status is not SINCOSM_OK or s = 0).
sincosm_status launch_scale_by_plan(const sincosm_plan* plan, int k, void* X, int64_t count, bool f64,
                                    hipStream_t stream);
// Fill the n x n (rows x cols) matrix X with NaN if the plan record at `plan`
// has a status other than SINCOSM_OK (decided on the device).
sincosm_status launch_fill_nan_if(const sincosm_plan* plan, int64_t n, void* X, int64_t ld, bool f64,
                                  hipStream_t stream);
sincosm_status launch_fill_nan_if_rect(const sincosm_plan* plan, int64_t rows, int64_t cols, void* X, int64_t ld,
                                       bool f64, hipStream_t stream);
sincosm_status launch_fill_nan_rect(int64_t rows, int64_t cols, void* X, int64_t ld, bool f64,
                                    hipStream_t stream);
// dst (n x n complex, leading dimension ldd in complex elements, pairs of the
// real type) = re + i (negate_im ? -im : im), from np x np zero-padded planes.
sincosm_status launch_interleave(int64_t n, int64_t np, const void* re, const void* im, bool negate_im,
                                 void* dst, int64_t ldd, bool f64, hipStream_t stream);
sincosm_status launch_fill_zero(int64_t np, void* X, bool f64, hipStream_t stream);
sincosm_status launch_convert_pad(int64_t n, int64_t np, const void* src, int64_t lds, bool src_f64,
                                  void* dst, bool dst_f64, hipStream_t stream);

// ----------------------------------------------------------------------------
// Launch timing (timing.cpp); kinds match SINCOSM_TIMING_* in the header.
// ----------------------------------------------------------------------------
struct TimingMark { int kind; void* a; };
bool timing_on();
TimingMark timing_begin(int kind, hipStream_t stream);
void timing_end(const TimingMark& m, hipStream_t stream);

}  // namespace sc
