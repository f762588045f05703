// Batched path: cos and sin of many independent matrices of uneven order
// (n <= 256) in one persistent launch.
//
// The orders and element offsets are device arrays of the caller. A first
// one-workgroup launch checks every entry (order within 1..256 and within the
// workspace's slot size, n x n elements inside the packed arrays), reports
// rejected entries in their plan record, and sorts the accepted ones by
// padded order into the work queue (largest first; a counting sort, so no
// host work and nothing read back). Each workgroup of the persistent launch
// then repeatedly takes the next matrix from the queue, and runs that
// matrix's whole method alone: zero-padded
// copy and 1-norm, plan (Tables 1-2), the scheme's products (Section 2.1) and
// the s double-angle steps (Section 1), each product as a loop over 64 x 64
// or 32 x 32 output tiles of the workgroup (per padded order, from the
// tuning table). Matrices never share a workgroup, so there
// is no synchronisation between workgroups; each resident workgroup owns one
// arena slot of 10 padded matrices, so the workspace does not grow with the
// batch. The stage descriptors of the four schemes are recorded once from the
// same builders the single-matrix path launches (schemes.cpp), with symbolic
// buffer ids resolved per matrix on the device.
//
// Padded orders up to 32 (float64) or 64 (float32) can instead run in kernels
// that keep the whole per-matrix workspace in LDS (batched_small_kernel,
// chosen per order by the tuning table); the queue kernel routes them there
// only when few larger matrices are queued, and they run before the
// persistent one. All product modes give bitwise the same results.
#include <math.h>
#include <string.h>

#include <algorithm>
#include <map>
#include <mutex>

#include "schemes.hpp"

namespace sc {
namespace {

constexpr int BT = 64;        // largest output tile of the per-workgroup product loop
constexpr int BBK = 16;       // k step
constexpr int BNT = 256;      // threads (4 waves in a 2 x 2 grid)
// Resident workgroups per CU the grid and the arena are sized for: the
// persistent kernel's registers allow three waves per SIMD, so three
// workgroups of four waves are resident per CU; a fourth per CU would start
// only once a resident one leaves, with the queue already empty.
constexpr int WG_PER_CU = 3;
constexpr int NMAX = 256;     // largest order of the batched path
// Per padded order: how its products run. TILE_64 / TILE_32: the arena in
// global memory, output tiles of 64 x 64 or 32 x 32 (batched_kernel);
// LDS_RESIDENT: the whole per-matrix workspace in LDS (batched_small_kernel:
// padded orders up to 32 in float64, up to 64 in float32).
constexpr int TILE_64 = 0, TILE_32 = 1, LDS_RESIDENT = 2;
constexpr int SNP = 64;       // largest padded order of any LDS-resident kernel

// symbolic buffer ids of the recorded templates
constexpr int ID_AP = 0;      // 1..9: W0..W8
constexpr int ID_COUT = 10;
constexpr int ID_SOUT = 11;
constexpr double SX_SENTINEL = 3.0;   // marks operand scales equal to 2^-s

__device__ Problem g_tmpl[4][8];
__device__ int g_tmpl_count[4];

// Per-level (C0, S0) slots when s > 0, and the second ping-pong pair.
// level index: 0 -> 3 products, 1 -> 4, 2 -> 6, 3 -> 7.
__host__ __device__ inline void squaring_slots(int li, int& c0, int& s0, int& c1, int& s1) {
  switch (li) {
    case 0: c0 = 1 + 2; s0 = 1 + 0; c1 = 1 + 4; s1 = 1 + 3; break;   // C W2, S W0 | W4, W3
    case 1: c0 = 1 + 5; s0 = 1 + 0; c1 = 1 + 2; s1 = 1 + 1; break;   // C W5, S W0 | W2, W1
    case 2: c0 = 1 + 1; s0 = 1 + 0; c1 = 1 + 3; s1 = 1 + 2; break;   // C W1, S W0 | W3, W2
    default: c0 = 1 + 8; s0 = 1 + 0; c1 = 1 + 2; s1 = 1 + 1; break;  // C W8, S W0 | W2, W1
  }
}

__host__ __device__ inline int level_index(int level) { return level == 3 ? 0 : level == 4 ? 1 : level == 6 ? 2 : 3; }

struct BatchArgs {
  int batch;
  int acc;
  int8_t mode[NMAX / 16 + 1];   // per padded order / 16: product mode (TILE_64, TILE_32 or LDS_RESIDENT)
  const int32_t* nmat;            // caller's orders (device)
  const int64_t* off;             // caller's element offsets (device)
  const int32_t* order;           // work queue: accepted entries, largest padded order first
  const unsigned int* nqueue;     // its length
  const unsigned int* nlarge;     // queue entries [0, nlarge) go to batched_kernel, the rest to the LDS kernels
  const unsigned int* nmid;       // [nlarge, nmid): LDS-resident, padded order 48 or 64; [nmid, nsmall): 32
  const unsigned int* nsmall;     // [nsmall, nqueue): LDS-resident, padded order 16
  const void* A;
  void* C;
  void* S;
  sincosm_plan* plans;
  char* arena;
  int64_t slot_bytes;
  unsigned int* counter;
};

// Check every entry and build the work queue (one workgroup). An entry is
// accepted when 1 <= n <= 256, its padded order fits the workspace's slots
// (npm) and its n x n elements lie inside the packed arrays (0 <= off,
// off + n^2 <= total); a rejected entry gets status SINCOSM_E_ARG (or
// SINCOSM_E_WORKSPACE for an order beyond npm) in its plan record and is not
// computed. Accepted entries are bucketed by padded order, largest first.
// The padded orders whose bit is set in lds_mask (bit k: order 16 k, k <=
// SNP / 16) go to the LDS-resident kernels, after all others in the queue, when
// the other entries number fewer than `fill` (the persistent kernel's
// workgroups): with more, those small matrices are worth more to the
// persistent kernel as the short work that fills the end of its run, and the
// whole queue stays its own. The queue's first *nlarge entries are
// batched_kernel's; of the rest, those of padded orders 48 and 64 (float32
// only) come first, up to *nmid, for the 64-order LDS-resident kernel, then
// those of order 32, up to *nsmall, for the 32-order one, then those of
// order 16 for the 16-order one. The order within a
// bucket does not matter (each matrix is computed by one workgroup the same
// way wherever it sits in the queue, and both kernels give the same bits).
constexpr int ORDER_THREADS = 1024;
constexpr int NBUCKET = NMAX / 16;
constexpr int NSB = SNP / 16;             // padded orders the LDS-resident kernel can take
constexpr int NB2 = NBUCKET + NSB;        // buckets of the queue

__device__ inline int entry_status(int n, int64_t o, int64_t total, int npm) {
  if (n < 1 || n > NMAX) return SINCOSM_E_ARG;
  if (o < 0 || o > total || (int64_t)n * n > total - o) return SINCOSM_E_ARG;
  if (((n + 15) & ~15) > npm) return SINCOSM_E_WORKSPACE;
  return SINCOSM_OK;
}

// Queue bucket of an accepted order: padded order 256 first ... 16 last, then
// the LDS-resident orders (64, 48, 32, 16).
__device__ inline int queue_bucket(int n, unsigned int lds_mask) {
  const int k = (n + 15) >> 4;
  if (k <= NSB && ((lds_mask >> k) & 1u)) return NBUCKET + NSB - k;
  return NBUCKET - k;
}

__global__ __launch_bounds__(ORDER_THREADS) void batched_order_kernel(int batch, const int32_t* nmat,
                                                                     const int64_t* off, int64_t total, int npm,
                                                                     unsigned int lds_mask, int fill,
                                                                     int32_t* order, unsigned int* counter,
                                                                     sincosm_plan* plans) {
  __shared__ unsigned int hist[NBUCKET];
  __shared__ unsigned int next[NB2];
  __shared__ unsigned int mask;
  const int tid = threadIdx.x;
  for (int b = tid; b < NBUCKET; b += ORDER_THREADS) hist[b] = 0u;
  __syncthreads();
  for (int i = tid; i < batch; i += ORDER_THREADS) {
    const int n = nmat[i];
    const int st = entry_status(n, off[i], total, npm);
    if (st != SINCOSM_OK) {
      if (plans) {
        sincosm_plan p;
        p.level = 0; p.s = 0; p.products = 0; p.status = st; p.norm1 = 0.0;
        plans[i] = p;
      }
      continue;
    }
    atomicAdd(&hist[queue_bucket(n, 0u)], 1u);   // by padded order: bucket 0 is order 256
  }
  __syncthreads();
  if (tid == 0) {
    unsigned int others = 0u;
    for (int k = 1; k <= NBUCKET; ++k)
      if (!(k <= NSB && ((lds_mask >> k) & 1u))) others += hist[NBUCKET - k];
    const unsigned int m = others < (unsigned int)fill ? lds_mask : 0u;
    mask = m;
    for (int b = 0; b < NB2; ++b) next[b] = 0u;
    for (int b = 0; b < NBUCKET; ++b) {
      const int k = NBUCKET - b;
      next[queue_bucket(16 * k, m)] = hist[b];
    }
    unsigned int run = 0u;
    for (int b = 0; b < NB2; ++b) {
      const unsigned int h = next[b];
      next[b] = run;
      run += h;
    }
    counter[0] = 0u;            // next entry of batched_kernel
    counter[1] = run;           // queue length
    counter[2] = next[NBUCKET]; // first entry of the LDS-resident kernels
    counter[3] = next[NBUCKET + NSB - 2];   // first LDS-resident entry of padded order 32
    counter[4] = next[NBUCKET + NSB - 1];   // first LDS-resident entry of padded order 16
  }
  __syncthreads();
  const unsigned int m = mask;
  for (int i = tid; i < batch; i += ORDER_THREADS) {
    const int n = nmat[i];
    if (entry_status(n, off[i], total, npm) != SINCOSM_OK) continue;
    order[atomicAdd(&next[queue_bucket(n, m)], 1u)] = i;
  }
}

template <typename T>
struct Vec;
template <>
struct Vec<double> {
  typedef double __attribute__((ext_vector_type(2))) t;
  static constexpr int N = 2;
};
template <>
struct Vec<float> {
  typedef float __attribute__((ext_vector_type(4))) t;
  static constexpr int N = 4;
};

template <typename T>
__device__ inline typename Vec<T>::t mma_step(T a, T b, typename Vec<T>::t c);

typedef double v4d __attribute__((ext_vector_type(4)));
typedef float v4f __attribute__((ext_vector_type(4)));

template <typename T>
struct BMma;
template <>
struct BMma<double> {
  typedef v4d acc_t;
  __device__ static inline acc_t mma(double a, double b, acc_t c) {
    return __builtin_amdgcn_mfma_f64_16x16x4f64(a, b, c, 0, 0, 0);
  }
  __device__ static inline int row_in_block(int lg, int r) { return lg + 4 * r; }
};
template <>
struct BMma<float> {
  typedef v4f acc_t;
  __device__ static inline acc_t mma(float a, float b, acc_t c) {
    return __builtin_amdgcn_mfma_f32_16x16x4f32(a, b, c, 0, 0, 0);
  }
  __device__ static inline int row_in_block(int lg, int r) { return 4 * lg + r; }
};

template <typename T>
struct Smem {
  static constexpr int VEC = Vec<T>::N;
  static constexpr int LDA = BBK + 1, LDB = BT + 16, LDE = BT + VEC;
  static constexpr int STAGE = 2 * (BT * LDA + BBK * LDB);
  static constexpr int EPI = (BT / 2) * LDE;
  static constexpr int ELEMS = STAGE > EPI ? STAGE : EPI;
};

// Output stage of one VEC-wide piece of a product at (row, col) of the padded
// np x np matrix, D = v: every output o of P receives e_o D + d_o I + the sum
// over q of c_oq In_q (I only within the matrix's true order), coalesced
// vector stores where the output is the padded matrix itself.
template <typename T>
__device__ inline void epi_piece(const Problem& P, int np, typename Vec<T>::t v, int row, int col, int nin,
                                 int nout, int nvalid) {
  using vec_t = typename Vec<T>::t;
  constexpr int VEC = Vec<T>::N;
  vec_t x[MAX_IN];
#pragma unroll
  for (int q = 0; q < MAX_IN; ++q)
    if (q < nin) x[q] = *(const vec_t*)((const T*)P.in[q].p + (int64_t)row * np + col);
  // outputs one at a time (coefficients re-read from LDS): keeps the
  // register footprint small, the inputs stay in registers
#pragma unroll 1
  for (int o = 0; o < nout; ++o) {
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
    if (O.lim == np && O.ld == np && (((uintptr_t)O.p) & 15u) == 0) {
      *(vec_t*)((T*)O.p + off) = val;
    } else if (row < O.lim) {
#pragma unroll
      for (int t = 0; t < VEC; ++t)
        if (col + t < O.lim) ((T*)O.p)[off + t] = val[t];
    }
  }
}

// One product of the current problem P (in LDS) over the whole np x np matrix,
// by this workgroup alone: output tiles of tb x tb (tb = 2^lt, 64 or 32; the
// four waves take tb/2 x tb/2 each), operands staged through LDS with
// rows/columns beyond np read as zero, MFMA blocks beyond np skipped. The
// smaller tile keeps all four waves busy on small orders. The tile is a
// run-time value so that one copy of the loop serves both (a second inlined
// copy pushes the kernel past its register budget).
template <typename T>
__device__ void wg_gemm(const Problem& P, int np, T* smem, int lt) {
  using M = BMma<T>;
  using acc_t = typename M::acc_t;
  using vec_t = typename Vec<T>::t;
  constexpr int VEC = Vec<T>::N;
  constexpr int LDA = Smem<T>::LDA, LDB = Smem<T>::LDB, LDE = Smem<T>::LDE;
  constexpr int F = BT / 32;                    // MFMA blocks per wave side at the largest tile
  constexpr int A_LOADS = (BT * BBK / VEC + BNT - 1) / BNT;
  constexpr int B_LOADS = (BBK * BT / VEC + BNT - 1) / BNT;
  const int TB = 1 << lt, WT = TB >> 1;         // tile, wave tile
  const bool two = WT > 16;                     // a wave holds 2 x 2 MFMA blocks
  T* const As0 = smem;
  T* const Bs0 = smem + 2 * BT * LDA;

  // the wave index is uniform across a wave: readfirstlane keeps it (and the
  // per-block validity tests built on it) in scalar registers, so they branch
  // on scalar conditions rather than through the exec mask
  const int tid = threadIdx.x, lane = tid & 63, wave = __builtin_amdgcn_readfirstlane(tid >> 6);
  const int wm = wave >> 1, wn = wave & 1;
  const int lr = lane & 15, lg = lane >> 4;
  const int nseg = P.nseg, nin = P.nin, nout = P.nout, nvalid = P.nvalid;
  const int nk = np / BBK, nkt = nseg * nk;
  const int tiles = (np + TB - 1) >> lt;

  for (int tm = 0; tm < tiles; ++tm) {
    for (int tn = 0; tn < tiles; ++tn) {
      acc_t acc[F][F];
#pragma unroll
      for (int i = 0; i < F; ++i)
#pragma unroll
        for (int j = 0; j < F; ++j)
#pragma unroll
          for (int r = 0; r < 4; ++r) acc[i][j][r] = (T)0;
      vec_t ra[A_LOADS], rb[B_LOADS];
      auto gload = [&](int kt) {
        const int sidx = kt / nk;
        const int k0 = (kt - sidx * nk) * BBK;
        const T* L = (const T*)P.seg[sidx].L;
        const T* R = (const T*)P.seg[sidx].R;
#pragma unroll
        for (int i = 0; i < A_LOADS; ++i) {
          const int e = (i * BNT + tid) * VEC;
          const int r = e / BBK, c = e - r * BBK;
          const int gr = tm * TB + r;
          if (e < TB * BBK && gr < np) ra[i] = *(const vec_t*)(L + (int64_t)gr * np + k0 + c);
          else ra[i] = (vec_t)0;
        }
#pragma unroll
        for (int i = 0; i < B_LOADS; ++i) {
          const int e = (i * BNT + tid) * VEC;
          const int r = e >> lt, c = e - (r << lt);
          const int gc = tn * TB + c;
          if (e < BBK * TB && gc < np) rb[i] = *(const vec_t*)(R + (int64_t)(k0 + r) * np + gc);
          else rb[i] = (vec_t)0;
        }
      };
      auto lstore = [&](int buf, int kt) {
        const Seg& S = P.seg[kt / nk];
        const T ls = (T)S.lscale, rs = (T)S.rscale;
        T* as = As0 + buf * (BT * LDA);
        T* bs = Bs0 + buf * (BBK * LDB);
#pragma unroll
        for (int i = 0; i < A_LOADS; ++i) {
          const int e = (i * BNT + tid) * VEC;
          const int r = e / BBK, c = e - r * BBK;
          if (e < TB * BBK) {
#pragma unroll
            for (int q = 0; q < VEC; ++q) as[r * LDA + c + q] = ra[i][q] * ls;
          }
        }
#pragma unroll
        for (int i = 0; i < B_LOADS; ++i) {
          const int e = (i * BNT + tid) * VEC;
          const int r = e >> lt, c = e - (r << lt);
          if (e < BBK * TB) *(vec_t*)(bs + r * LDB + c) = rb[i] * rs;
        }
      };
      const bool rowok0 = tm * TB + wm * WT < np, rowok1 = two && tm * TB + wm * WT + 16 < np;
      const bool colok0 = tn * TB + wn * WT < np, colok1 = two && tn * TB + wn * WT + 16 < np;
      if (nkt > 0) {
        gload(0);
        lstore(0, 0);
      }
      __syncthreads();
      for (int kt = 0; kt < nkt; ++kt) {
        const int cur = kt & 1;
        if (kt + 1 < nkt) gload(kt + 1);
        if (rowok0 && colok0) {  // wave-uniform: this wave has at least one live block
          const T* as = As0 + cur * (BT * LDA) + (wm * WT + lr) * LDA + lg;
          const T* bs = Bs0 + cur * (BBK * LDB) + lg * LDB + wn * WT + lr;
#pragma unroll
          for (int kk = 0; kk < BBK / 4; ++kk) {
            // the second row/column of blocks lies inside the LDS tile also
            // when tb = 32 (reads of unused staging), its products are skipped
            const T a0 = as[kk * 4], a1 = as[16 * LDA + kk * 4];
            const T b0 = bs[kk * 4 * LDB], b1 = bs[kk * 4 * LDB + 16];
            acc[0][0] = M::mma(a0, b0, acc[0][0]);
            if (colok1) acc[0][1] = M::mma(a0, b1, acc[0][1]);
            if (rowok1) acc[1][0] = M::mma(a1, b0, acc[1][0]);
            if (rowok1 && colok1) acc[1][1] = M::mma(a1, b1, acc[1][1]);
          }
        }
        if (kt + 1 < nkt) lstore(cur ^ 1, kt + 1);
        __syncthreads();
      }
      // epilogue: two bands of WT rows staged through LDS, then coalesced
      T* const E = smem;
      for (int band = 0; band < 2; ++band) {
        if (wm == band) {
#pragma unroll
          for (int i = 0; i < F; ++i)
#pragma unroll
            for (int j = 0; j < F; ++j)
              if ((i == 0 && j == 0) || two) {
#pragma unroll
                for (int r = 0; r < 4; ++r)
                  E[(i * 16 + M::row_in_block(lg, r)) * LDE + wn * WT + j * 16 + lr] = acc[i][j][r];
              }
        }
        __syncthreads();
#pragma unroll 1
        for (int e = tid * VEC; e < WT * TB; e += BNT * VEC) {
          const int br = e >> lt, bc = e - (br << lt);
          const int row = tm * TB + band * WT + br;
          const int col = tn * TB + bc;
          if (row >= np || col >= np) continue;
          epi_piece<T>(P, np, *(const vec_t*)(E + br * LDE + bc), row, col, nin, nout, nvalid);
        }
        __syncthreads();
      }
    }
  }
}

template <typename T>
__device__ inline void* resolve(const void* sym, T* slot, int np) {
  const intptr_t id = (intptr_t)sym - 1;
  return slot + (int64_t)id * np * np;
}

template <typename T>
__global__ __launch_bounds__(BNT) __attribute__((amdgpu_waves_per_eu(3))) void batched_kernel(BatchArgs a) {
  __shared__ __attribute__((aligned(16))) T smem[Smem<T>::ELEMS];
  __shared__ Problem prob;
  __shared__ unsigned long long red[BNT];
  __shared__ int s_item;
  __shared__ sincosm_plan s_plan;
  const int tid = threadIdx.x;
  T* const slot = (T*)(a.arena + (int64_t)blockIdx.x * a.slot_bytes);
  const int nq = (int)*a.nlarge;   // the queue's entries for this kernel

  for (;;) {
    if (tid == 0) s_item = (int)atomicAdd(a.counter, 1u);
    __syncthreads();
    const int item = s_item;
    __syncthreads();
    if (item >= nq) break;
    const int i = a.order[item];
    if (i < 0 || i >= a.batch) continue;     // the queue holds checked entries only
    const int n = a.nmat[i];
    if (n < 1 || n > NMAX) continue;
    const int64_t off = a.off[i];
    const int np = (n + 15) & ~15;
    // log2 of the product tile (orders routed to an LDS-resident kernel that
    // this kernel takes instead, see batched_order_kernel: 32 x 32 up to order
    // 32, 64 x 64 above)
    const int md = a.mode[np >> 4];
    const int lt = (md == TILE_64 || (md == LDS_RESIDENT && np > 32)) ? 6 : 5;
    const T* Ai = (const T*)a.A + off;
    T* Ci = (T*)a.C + off;
    T* Si = (T*)a.S + off;
    T* Ap = slot;

    // zero-padded copy and column sums (each thread one column, rows in order;
    // the loads of 16 rows are issued together, then added in row order)
    for (int c = tid; c < np; c += BNT) {
      double sum = 0.0;
      for (int r0 = 0; r0 < np; r0 += 16) {
        double v[16];
#pragma unroll
        for (int u = 0; u < 16; ++u) {
          const int r = r0 + u;
          v[u] = (r < n && c < n) ? (double)Ai[(int64_t)r * n + c] : 0.0;
        }
#pragma unroll
        for (int u = 0; u < 16; ++u) {
          Ap[(int64_t)(r0 + u) * np + c] = (T)v[u];
          sum += fabs(v[u]);
        }
      }
      red[c] = (unsigned long long)__double_as_longlong(sum);
    }
    for (int c = np + tid; c < BNT; c += BNT) red[c] = 0ull;
    __syncthreads();
    // maximum over the columns (integer compare of the float64 bit patterns:
    // order-independent, so the same result as a sequential scan)
    for (int w = BNT / 2; w > 0; w >>= 1) {
      if (tid < w && red[tid + w] > red[tid]) red[tid] = red[tid + w];
      __syncthreads();
    }
    if (tid == 0) {
      sincosm_plan p;
      plan_rule(__longlong_as_double((long long)red[0]), a.acc, &p);
      s_plan = p;
      if (a.plans) a.plans[i] = p;
    }
    __syncthreads();
    const sincosm_plan plan = s_plan;
    if (plan.status != SINCOSM_OK) {
      const T nanv = (T)__longlong_as_double(0x7ff8000000000000ll);
      for (int e = tid; e < n * n; e += BNT) { Ci[e] = nanv; Si[e] = nanv; }
      __syncthreads();
      continue;
    }
    const int li = level_index(plan.level);
    const int s = plan.s;
    const double sx = ldexp(1.0, -s);
    int c0, s0, c1, s1;
    squaring_slots(li, c0, s0, c1, s1);

    // the scheme's products, then s double-angle steps of two products from
    // (S, C) to (S', C'), ping-pong between the two slot pairs (the last step
    // writes the caller's matrices); one product call site for all of them
    const int nst = g_tmpl_count[li];
    for (int t = 0; t < nst + 2 * s; ++t) {
      if (t < nst) {
        {  // cooperative word copy of the template into LDS
          const unsigned long long* src = (const unsigned long long*)&g_tmpl[li][t];
          unsigned long long* dst = (unsigned long long*)&prob;
          for (int w = tid; w < (int)(sizeof(Problem) / 8); w += BNT) dst[w] = src[w];
        }
        __syncthreads();
        if (tid == 0) {
          prob.nvalid = n;
          for (int q = 0; q < prob.nseg; ++q) {
            Seg& g = prob.seg[q];
            g.L = resolve<T>(g.L, slot, np);
            g.R = resolve<T>(g.R, slot, np);
            g.ldl = g.ldr = np;
            if (g.lscale == SX_SENTINEL) g.lscale = sx;
            if (g.rscale == SX_SENTINEL) g.rscale = sx;
          }
          for (int q = 0; q < prob.nin; ++q) {
            prob.in[q].p = resolve<T>(prob.in[q].p, slot, np);
            prob.in[q].ld = np;
          }
          for (int q = 0; q < prob.nout; ++q) {
            EpiOut& o = prob.out[q];
            const intptr_t id = (intptr_t)o.p - 1;
            if (id == ID_COUT || id == ID_SOUT) {
              if (s == 0) {
                o.p = id == ID_COUT ? (void*)Ci : (void*)Si;
                o.ld = n;
                o.lim = n;
              } else {
                o.p = slot + (int64_t)(id == ID_COUT ? c0 : s0) * np * np;
                o.ld = np;
                o.lim = np;
              }
            } else {
              o.p = resolve<T>(o.p, slot, np);
              o.ld = np;
              o.lim = np;
            }
            o.f64 = sizeof(T) == 8;
          }
        }
      } else {
        const int j = (t - nst) >> 1, half = (t - nst) & 1;
        const bool last = j == s - 1;
        T* Sc = slot + (int64_t)((j & 1) ? s1 : s0) * np * np;
        T* Cc = slot + (int64_t)((j & 1) ? c1 : c0) * np * np;
        T* Sn = last ? Si : slot + (int64_t)((j & 1) ? s0 : s1) * np * np;
        T* Cn = last ? Ci : slot + (int64_t)((j & 1) ? c0 : c1) * np * np;
        {
          unsigned long long* dst = (unsigned long long*)&prob;
          for (int w = tid; w < (int)(sizeof(Problem) / 8); w += BNT) dst[w] = 0ull;
        }
        __syncthreads();
        if (tid == 0) {
          prob.nvalid = n;
          prob.nseg = 1;
          prob.seg[0].L = Sc;
          prob.seg[0].R = half == 0 ? Sc : Cc;
          prob.seg[0].ldl = prob.seg[0].ldr = np;
          prob.seg[0].lscale = prob.seg[0].rscale = 1.0;
          prob.nout = 1;
          EpiOut& o = prob.out[0];
          o.p = half == 0 ? Cn : Sn;
          o.ld = last ? n : np;
          o.lim = last ? n : np;
          o.f64 = sizeof(T) == 8;
          o.e = half == 0 ? -2.0 : 2.0;
          o.d = half == 0 ? 1.0 : 0.0;
        }
      }
      __syncthreads();
      wg_gemm<T>(prob, np, smem, lt);
    }
  }
}

// ----------------------------------------------------------------------------
// LDS-resident kernels for padded orders up to SN, each taking the orders
// above the next smaller instance (16: order 16; 32: order 32; 64: float32
// orders 48 and 64). A matrix's whole workspace
// stays on chip: W0 .. W8 in LDS (row stride SN + 1, so the rows an MFMA
// operand read touches start in different banks; 23 KB for float64 at
// SN = 16, six workgroups per CU; 76 KB at SN = 32, two; 150 KB for float32
// at SN = 64, one), and the padded
// copy of A, which the schemes use only as a product operand, as the MFMA
// operand fragments of each wave in registers. Only A is read from memory and
// only C and S are written. The workgroup has one wave per 16 x 16 output
// block at order SN (1, 4 or 16 waves); at a smaller padded order the waves
// whose block lies outside it sit out the products. Each wave applies the
// epilogue straight from its accumulators. The k order of every product, the operand scaling and the
// epilogue's fused multiply-adds are those of batched_kernel, so the results
// are bitwise the same; the two products of a double-angle step run in one
// pass (they share no output).
//
// At these orders a matrix's arithmetic takes a few microseconds, so the
// kernel is laid out against memory latency: the workgroups take the queue's
// entries round robin (entry w + k G for workgroup w of G: no queue atomic),
// the entry's index, then its order and offset, then its elements are loaded
// three, two and one matrices ahead, and the scheme's products read a compact
// copy of the level's recorded stages that the workgroup stages in LDS per
// matrix (one round trip instead of a chain of dependent loads per product).
// ----------------------------------------------------------------------------
template <int SN>
struct SmallGeom {
  static constexpr int NT = (SN / 16) * (SN / 16) * 64;   // threads: one wave per 16 x 16 block
  static constexpr int LD = SN + 1;                       // LDS row stride
  static constexpr int SLOT = SN * LD;                    // elements per LDS slot
  static constexpr int PF = SN * SN / NT;                 // prefetched input elements per thread
  static constexpr int KK = SN / 4;                       // MFMA k steps at order SN
  static_assert(PF * NT == SN * SN, "prefetch covers the matrix");
};

// One recorded product in the form the LDS-resident kernel reads: operand and
// output ids as in the templates (0: padded copy of A, k + 1: W_k, ID_COUT,
// ID_SOUT), epilogue inputs as W slots, scales with SX_SENTINEL for 2^-s.
struct SmallOp {
  int8_t nseg, nin, nout, pad;
  int8_t L[MAX_SEG], R[MAX_SEG];
  int8_t in[MAX_IN];
  int8_t out[MAX_OUT];
  int8_t pad2[2];
  double lsc[MAX_SEG], rsc[MAX_SEG];
  double e[MAX_OUT], d[MAX_OUT];
  double c[MAX_OUT][MAX_IN];
};
static_assert(sizeof(SmallOp) % 8 == 0, "SmallOp copies as 8-byte words");
__device__ SmallOp g_small[4][8];

template <typename T, int SN>
__device__ inline void small_load_a(const BatchArgs& a, int n, int64_t off, int tid,
                                    T (&v)[SmallGeom<SN>::PF]) {
  using G = SmallGeom<SN>;
  const int np = (n + 15) & ~15;
  const T* Ai = (const T*)a.A + off;
#pragma unroll
  for (int u = 0; u < G::PF; ++u) {
    const int e = tid + u * G::NT;
    const int r = np > 0 ? e / np : 0, c = np > 0 ? e - r * np : 0;
    v[u] = (n > 0 && e < np * np && r < n && c < n) ? Ai[r * n + c] : (T)0;
  }
}

template <typename T, int SN>
__global__ __launch_bounds__(SmallGeom<SN>::NT) void batched_small_kernel(BatchArgs a) {
  using M = BMma<T>;
  using acc_t = typename M::acc_t;
  using Gm = SmallGeom<SN>;
  constexpr int NT = Gm::NT, SLD = Gm::LD, SSLOT = Gm::SLOT, SPF = Gm::PF, SKK = Gm::KK;
  constexpr int NB = SN / 16;                 // blocks per side at order SN
  __shared__ __attribute__((aligned(16))) T W[9 * SSLOT];
  __shared__ SmallOp ops[8];
  __shared__ sincosm_plan s_plan;
  const int tid = threadIdx.x, lane = tid & 63, wave = __builtin_amdgcn_readfirstlane(tid >> 6);
  const int lr = lane & 15, lg = lane >> 4;
  const int bm = wave / NB, bn = wave % NB;   // this wave's output block
  // this kernel's part of the queue (see batched_order_kernel)
  const int nl = (int)(SN > 32 ? *a.nlarge : SN > 16 ? *a.nmid : *a.nsmall);
  const int nq = (int)(SN > 32 ? *a.nmid : SN > 16 ? *a.nsmall : *a.nqueue);
  const int G = (int)gridDim.x;
  T* const TMP = W + 8 * SSLOT;               // the padded copy of A passes through W8's slot

  // entry q of this workgroup's share: queue position nl + blockIdx.x + q G.
  // Loaded values are checked only when the next iteration uses them, so no
  // load issued for the entries ahead is waited for before this matrix's work.
  auto pos_of = [&](int q) { return nl + (int)blockIdx.x + q * G; };
  auto valid_i = [&](int i) { return i >= 0 && i < a.batch ? i : -1; };
  auto valid_n = [&](int n) { return n >= 1 && n <= SN ? n : 0; };
  int i0 = pos_of(0) < nq ? valid_i(a.order[pos_of(0)]) : -1;
  int n0 = i0 >= 0 ? valid_n(a.nmat[i0]) : 0;
  int64_t off0 = n0 > 0 ? a.off[i0] : 0;
  int i1 = pos_of(1) < nq ? valid_i(a.order[pos_of(1)]) : -1;
  int n1 = i1 >= 0 ? valid_n(a.nmat[i1]) : 0;
  int64_t off1 = n1 > 0 ? a.off[i1] : 0;
  int i2 = pos_of(2) < nq ? valid_i(a.order[pos_of(2)]) : -1;
  T cur[SPF], nxt[SPF];
  small_load_a<T, SN>(a, n0, off0, tid, cur);
  for (int q = 0; pos_of(q) < nq; ++q) {
    small_load_a<T, SN>(a, n1, off1, tid, nxt);                  // elements of entry q + 1
    const int i3raw = pos_of(q + 3) < nq ? a.order[pos_of(q + 3)] : -1;   // index of entry q + 3
    const int n2raw = i2 >= 0 ? a.nmat[i2] : 0;                  // order and offset of entry q + 2
    const int64_t off2raw = i2 >= 0 ? a.off[i2] : 0;

    const int n = __builtin_amdgcn_readfirstlane(n0), i = __builtin_amdgcn_readfirstlane(i0);
    if (n > 0) {
      const int np = (n + 15) & ~15;
      const int nkk = np >> 2;
      const bool mine = bm * 16 < np && bn * 16 < np;   // wave-uniform
      T* Ci = (T*)a.C + off0;
      T* Si = (T*)a.S + off0;
      // padded copy through LDS: the column sums (rows in order, in float64)
      // and each wave's operand fragments of A
#pragma unroll
      for (int u = 0; u < SPF; ++u) {
        const int e = tid + u * NT;
        if (e < np * np) {
          const int r = e / np, c = e - r * np;
          TMP[r * SLD + c] = cur[u];
        }
      }
      __syncthreads();
      T La[SKK], Rb[SKK];
#pragma unroll
      for (int kk = 0; kk < SKK; ++kk) {
        La[kk] = (T)0;
        Rb[kk] = (T)0;
        if (mine && kk < nkk) {
          La[kk] = TMP[(bm * 16 + lr) * SLD + kk * 4 + lg];
          Rb[kk] = TMP[(kk * 4 + lg) * SLD + bn * 16 + lr];
        }
      }
      if (tid < 64) {
        // column sums on lanes 0 .. np - 1 of wave 0, then their maximum (an
        // integer compare of the float64 bit patterns, as batched_kernel's tree)
        unsigned long long bits = 0ull;
        if (tid < np) {
          double sum = 0.0;
          for (int r = 0; r < np; ++r) sum += fabs((double)TMP[r * SLD + tid]);
          bits = (unsigned long long)__double_as_longlong(sum);
        }
#pragma unroll
        for (int w = 32; w > 0; w >>= 1) {
          const unsigned long long o = __shfl_xor(bits, w);
          bits = o > bits ? o : bits;
        }
        if (tid == 0) {
          sincosm_plan p;
          plan_rule(__longlong_as_double((long long)bits), a.acc, &p);
          s_plan = p;
          if (a.plans) a.plans[i] = p;
        }
      }
      __syncthreads();
      const sincosm_plan plan = s_plan;
      if (plan.status != SINCOSM_OK) {
        const T nanv = (T)__longlong_as_double(0x7ff8000000000000ll);
        for (int e = tid; e < n * n; e += NT) { Ci[e] = nanv; Si[e] = nanv; }
      } else {
        const int li = __builtin_amdgcn_readfirstlane(level_index(plan.level));
        const int s = __builtin_amdgcn_readfirstlane(plan.s);
        const double sx = ldexp(1.0, -s);
        int c0, s0, c1, s1;
        squaring_slots(li, c0, s0, c1, s1);
        c0 -= 1; s0 -= 1; c1 -= 1; s1 -= 1;    // ids -> LDS slots
        const int nst = g_tmpl_count[li];
        {  // the level's stages into LDS, one 8-byte word per thread
          const unsigned long long* src = (const unsigned long long*)&g_small[li][0];
          unsigned long long* dst = (unsigned long long*)&ops[0];
          const int words = nst * (int)(sizeof(SmallOp) / 8);
          for (int w = tid; w < words; w += NT) dst[w] = src[w];
        }
        __syncthreads();
        for (int t = 0; t < nst; ++t) {
          const SmallOp& P = ops[t];
          if (mine) {
            acc_t acc;
#pragma unroll
            for (int r = 0; r < 4; ++r) acc[r] = (T)0;
            const int nseg = P.nseg;
            for (int g = 0; g < nseg; ++g) {
              const int idl = P.L[g], idr = P.R[g];
              const T ls = (T)(P.lsc[g] == SX_SENTINEL ? sx : P.lsc[g]);
              const T rs = (T)(P.rsc[g] == SX_SENTINEL ? sx : P.rsc[g]);
              // (the padded copy of A comes from the fragments; its slot is never read)
              const T* L = W + (idl == ID_AP ? 0 : idl - 1) * SSLOT + (bm * 16 + lr) * SLD + lg;
              const T* R = W + (idr == ID_AP ? 0 : idr - 1) * SSLOT + lg * SLD + bn * 16 + lr;
#pragma unroll
              for (int kk = 0; kk < SKK; ++kk) {
                if (kk < nkk) {
                  const T av = idl == ID_AP ? La[kk] : L[kk * 4];
                  const T bv = idr == ID_AP ? Rb[kk] : R[kk * 4 * SLD];
                  acc = M::mma(av * ls, bv * rs, acc);
                }
              }
            }
            const int nin = P.nin, nout = P.nout;
#pragma unroll
            for (int r = 0; r < 4; ++r) {
              const int row = bm * 16 + M::row_in_block(lg, r), col = bn * 16 + lr;
              T x[MAX_IN];
#pragma unroll
              for (int qi = 0; qi < MAX_IN; ++qi)
                if (qi < nin) x[qi] = W[P.in[qi] * SSLOT + row * SLD + col];
              for (int o = 0; o < nout; ++o) {
                T y = (row == col && row < n) ? (T)P.d[o] : (T)0;
                y = __builtin_fma((T)P.e[o], acc[r], y);
#pragma unroll
                for (int qi = 0; qi < MAX_IN; ++qi)
                  if (qi < nin) y = __builtin_fma((T)P.c[o][qi], x[qi], y);
                const int id = P.out[o];
                if (id == ID_COUT || id == ID_SOUT) {
                  if (s == 0) {
                    if (row < n && col < n) (id == ID_COUT ? Ci : Si)[row * n + col] = y;
                  } else {
                    W[(id == ID_COUT ? c0 : s0) * SSLOT + row * SLD + col] = y;
                  }
                } else {
                  W[(id - 1) * SSLOT + row * SLD + col] = y;
                }
              }
            }
          }
          __syncthreads();
        }
        // double-angle steps: P = S S -> C' = I - 2 P, Q = S C -> S' = 2 Q
        for (int j = 0; j < s; ++j) {
          const bool last = j == s - 1;
          const int sc = (j & 1) ? s1 : s0, cc = (j & 1) ? c1 : c0;
          const int sn = (j & 1) ? s0 : s1, cn = (j & 1) ? c0 : c1;
          if (mine) {
            acc_t pa, qa;
#pragma unroll
            for (int r = 0; r < 4; ++r) { pa[r] = (T)0; qa[r] = (T)0; }
            const T* L = W + sc * SSLOT + (bm * 16 + lr) * SLD + lg;
            const T* RS = W + sc * SSLOT + lg * SLD + bn * 16 + lr;
            const T* RC = W + cc * SSLOT + lg * SLD + bn * 16 + lr;
#pragma unroll
            for (int kk = 0; kk < SKK; ++kk) {
              if (kk < nkk) {
                const T av = L[kk * 4];
                pa = M::mma(av, RS[kk * 4 * SLD], pa);
                qa = M::mma(av, RC[kk * 4 * SLD], qa);
              }
            }
#pragma unroll
            for (int r = 0; r < 4; ++r) {
              const int row = bm * 16 + M::row_in_block(lg, r), col = bn * 16 + lr;
              T yc = (row == col && row < n) ? (T)1.0 : (T)0;
              yc = __builtin_fma((T)-2.0, pa[r], yc);
              const T ys = __builtin_fma((T)2.0, qa[r], (T)0);
              if (last) {
                if (row < n && col < n) {
                  Ci[row * n + col] = yc;
                  Si[row * n + col] = ys;
                }
              } else {
                W[cn * SSLOT + row * SLD + col] = yc;
                W[sn * SSLOT + row * SLD + col] = ys;
              }
            }
          }
          __syncthreads();
        }
      }
    }
    // advance the pipeline
    i0 = i1; n0 = n1; off0 = off1;
    i1 = i2; n1 = i2 >= 0 ? valid_n(n2raw) : 0; off1 = n1 > 0 ? off2raw : 0;
    i2 = valid_i(i3raw);
#pragma unroll
    for (int u = 0; u < SPF; ++u) cur[u] = nxt[u];
  }
}

// Templates are recorded once per process and copied to each device on first use.
std::mutex tmpl_mu;
bool tmpl_built = false;
Problem tmpl_host[4][8];
SmallOp small_host[4][8];
int tmpl_count_host[4];
std::map<int, bool> tmpl_uploaded;

sincosm_status build_templates() {
  if (tmpl_built) return SINCOSM_OK;
  memset(tmpl_host, 0, sizeof(tmpl_host));
  const int levels[4] = {3, 4, 6, 7};
  for (int li = 0; li < 4; ++li) {
    Modes m;
    memset(&m, 0, sizeof(m));
    m.poly = Arith::F64;
    m.sq = Arith::F64;
    m.poly_f64 = m.sq_f64 = m.user_f64 = true;
    m.np = 16;   // placeholder, resolved per matrix
    Recorder rec;
    Run r;
    r.m = &m;
    r.n = 16;
    r.Ap = (void*)(intptr_t)(ID_AP + 1);
    for (int k = 0; k < 9; ++k) r.W[k] = (void*)(intptr_t)(k + 2);
    r.Cout = Target{(void*)(intptr_t)(ID_COUT + 1), 16, 16, true};
    r.Sout = Target{(void*)(intptr_t)(ID_SOUT + 1), 16, 16, true};
    r.stream = nullptr;
    r.rec = &rec;
    SC_TRY(run_scheme(r, levels[li], SX_SENTINEL));
    for (int t = 0; t < rec.count; ++t) {
      if (rec.launches[t].nprob != 1) return SINCOSM_E_ARG;
      tmpl_host[li][t] = rec.launches[t].prob[0];
    }
    tmpl_count_host[li] = rec.count;
  }
  // the same stages in the LDS-resident kernel's compact form
  memset(small_host, 0, sizeof(small_host));
  for (int li = 0; li < 4; ++li)
    for (int t = 0; t < tmpl_count_host[li]; ++t) {
      const Problem& P = tmpl_host[li][t];
      SmallOp& o = small_host[li][t];
      if (P.nseg > MAX_SEG || P.nin > MAX_IN || P.nout > MAX_OUT) return SINCOSM_E_ARG;
      o.nseg = (int8_t)P.nseg;
      o.nin = (int8_t)P.nin;
      o.nout = (int8_t)P.nout;
      for (int q = 0; q < P.nseg; ++q) {
        o.L[q] = (int8_t)((intptr_t)P.seg[q].L - 1);
        o.R[q] = (int8_t)((intptr_t)P.seg[q].R - 1);
        o.lsc[q] = P.seg[q].lscale;
        o.rsc[q] = P.seg[q].rscale;
      }
      for (int q = 0; q < P.nin; ++q) {
        const intptr_t id = (intptr_t)P.in[q].p - 1;
        if (id < 1 || id > 9) return SINCOSM_E_ARG;   // epilogue inputs are W slots
        o.in[q] = (int8_t)(id - 1);
      }
      for (int q = 0; q < P.nout; ++q) {
        const intptr_t id = (intptr_t)P.out[q].p - 1;
        if (id < 1 || id > ID_SOUT) return SINCOSM_E_ARG;
        o.out[q] = (int8_t)id;
        o.e[q] = P.out[q].e;
        o.d[q] = P.out[q].d;
        for (int k = 0; k < MAX_IN; ++k) o.c[q][k] = P.out[q].c[k];
      }
    }
  tmpl_built = true;
  return SINCOSM_OK;
}

sincosm_status ensure_templates(hipStream_t stream) {
  std::lock_guard<std::mutex> g(tmpl_mu);
  SC_TRY(build_templates());
  int dev = 0;
  SC_HIP(hipGetDevice(&dev));
  if (tmpl_uploaded[dev]) return SINCOSM_OK;
  SC_HIP(hipMemcpyToSymbolAsync(HIP_SYMBOL(g_tmpl), tmpl_host, sizeof(tmpl_host), 0, hipMemcpyHostToDevice,
                                stream));
  SC_HIP(hipMemcpyToSymbolAsync(HIP_SYMBOL(g_tmpl_count), tmpl_count_host, sizeof(tmpl_count_host), 0,
                                hipMemcpyHostToDevice, stream));
  SC_HIP(hipMemcpyToSymbolAsync(HIP_SYMBOL(g_small), small_host, sizeof(small_host), 0, hipMemcpyHostToDevice,
                                stream));
  SC_HIP(hipStreamSynchronize(stream));
  tmpl_uploaded[dev] = true;
  return SINCOSM_OK;
}

struct BatchLayout {
  size_t counter_off, order_off, arena_off, slot_bytes, total;
  int slots, npm;
};

int device_cus() {
  int dev = 0, cus = 0;
  if (hipGetDevice(&dev) != hipSuccess) return 0;
  if (hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev) != hipSuccess) return 0;
  return cus;
}

// Workspace: the queue counters (256 bytes: next entry, length, and where the
// parts of the three LDS-resident instances begin), the work queue, then one arena
// slot of 10 padded matrices of order npm per resident workgroup.
bool batch_layout(int64_t batch, int npm, int dtype, BatchLayout& L) {
  const int cus = device_cus();
  if (cus <= 0) return false;
  const size_t es = dtype == SINCOSM_F64 ? 8 : 4;
  L.npm = npm;
  L.slots = (int)std::min<int64_t>(batch, (int64_t)cus * WG_PER_CU);
  L.slot_bytes = align_up((size_t)10 * npm * npm * es, 256);
  size_t off = 0;
  L.counter_off = off; off += 256;
  L.order_off = off; off += align_up((size_t)batch * 4, 256);
  L.arena_off = off; off += (size_t)L.slots * L.slot_bytes;
  L.total = off;
  return true;
}

}  // namespace
}  // namespace sc

using namespace sc;

extern "C" {

size_t sincosm_batched_workspace_size(int64_t batch, const int32_t* n_host, int dtype, int acc, int prod) {
  (void)acc;
  if (batch <= 0 || batch > INT32_MAX || (dtype != SINCOSM_F64 && dtype != SINCOSM_F32) ||
      prod != SINCOSM_PROD_NATIVE)
    return 0;
  int nmax = NMAX;
  if (n_host) {
    nmax = 1;
    for (int64_t i = 0; i < batch; ++i) {
      if (n_host[i] < 1 || n_host[i] > NMAX) return 0;
      nmax = std::max<int>(nmax, n_host[i]);
    }
  }
  BatchLayout L;
  if (!batch_layout(batch, (nmax + 15) & ~15, dtype, L)) return 0;
  return L.total;
}

sincosm_status sincosm_eval_batched(int64_t batch, int dtype, const int32_t* n_dev, const int64_t* offset_dev,
                                    int64_t total_elems, const void* A, void* C, void* S, int acc, int prod,
                                    void* ws, size_t ws_bytes, sincosm_plan* plans_dev, void* stream_) {
  if (batch < 0 || batch > INT32_MAX || total_elems < 0) return SINCOSM_E_ARG;
  if (batch == 0) return SINCOSM_OK;
  if (acc != SINCOSM_ACC_DOUBLE && acc != SINCOSM_ACC_SINGLE) return SINCOSM_E_ARG;
  if (dtype != SINCOSM_F64 && dtype != SINCOSM_F32) return SINCOSM_E_ARG;
  if (prod != SINCOSM_PROD_NATIVE) return SINCOSM_E_UNSUPPORTED;
  if (!n_dev || !offset_dev || !A || !C || !S) return SINCOSM_E_ARG;
  if (!ws || ((uintptr_t)ws & 255u)) return SINCOSM_E_WORKSPACE;
  // the largest padded order whose slots fit the workspace (orders above it
  // are rejected on the device with SINCOSM_E_WORKSPACE)
  BatchLayout L;
  int npm = 0;
  for (int cand = NMAX; cand >= 16; cand -= 16) {
    BatchLayout t;
    if (!batch_layout(batch, cand, dtype, t)) return SINCOSM_E_HIP;
    if (t.total <= ws_bytes) {
      L = t;
      npm = cand;
      break;
    }
  }
  if (npm == 0) return SINCOSM_E_WORKSPACE;
  hipStream_t stream = (hipStream_t)stream_;
  SC_TRY(ensure_templates(stream));
  char* base = (char*)ws;
  unsigned int* counter = (unsigned int*)(base + L.counter_off);
  unsigned int* nqueue = counter + 1;
  unsigned int* nlarge = counter + 2;
  int32_t* order = (int32_t*)(base + L.order_off);
  BatchArgs a;
  a.batch = (int)batch;
  a.acc = acc;
  a.nmat = n_dev;
  a.off = offset_dev;
  a.order = order;
  a.nqueue = nqueue;
  a.A = A;
  a.C = C;
  a.S = S;
  a.plans = plans_dev;
  a.arena = base + L.arena_off;
  a.slot_bytes = (int64_t)L.slot_bytes;
  a.counter = counter;
  a.nlarge = nlarge;
  a.nmid = counter + 3;
  a.nsmall = counter + 4;
  // product mode per padded order, from the tuning table
  const Arith ar = dtype == SINCOSM_F64 ? Arith::F64 : Arith::F32;
  unsigned int lds_mask = 0u;
  for (int b = 0; b <= NMAX / 16; ++b) {
    const int tile = batched_tile(ar, 16 * b);   // 0: LDS-resident (only offered where it fits)
    a.mode[b] = (int8_t)(tile == 32 ? TILE_32 : tile == 0 ? LDS_RESIDENT : TILE_64);
    if (tile == 0 && b >= 1 && b <= NSB) lds_mask |= 1u << b;
  }
  const TimingMark t = timing_begin(SINCOSM_TIMING_BATCHED, stream);
  batched_order_kernel<<<1, ORDER_THREADS, 0, stream>>>((int)batch, n_dev, offset_dev, total_elems, npm,
                                                        lds_mask, L.slots, order, counter, plans_dev);
  // the smallest orders first: their workgroups are short, and the large
  // orders then end the call with the queue's usual largest-first tail
  const int64_t cus = device_cus();
  if (lds_mask & ((1u << 3) | (1u << 4))) {   // float32 padded orders 48, 64: one 16-wave workgroup per CU
    const int g = (int)std::min<int64_t>(batch, cus);
    batched_small_kernel<float, 64><<<g, SmallGeom<64>::NT, 0, stream>>>(a);
  }
  if (lds_mask & (1u << 2)) {   // padded order 32: 2 (float64) or 3 (float32) workgroups per CU
    const int g = (int)std::min<int64_t>(batch, cus * (dtype == SINCOSM_F64 ? 2 : 3));
    if (dtype == SINCOSM_F64) batched_small_kernel<double, 32><<<g, SmallGeom<32>::NT, 0, stream>>>(a);
    else batched_small_kernel<float, 32><<<g, SmallGeom<32>::NT, 0, stream>>>(a);
  }
  if (lds_mask & (1u << 1)) {   // padded order 16: one-wave workgroups, 6 (float64) or 10 (float32) per CU
    const int g = (int)std::min<int64_t>(batch, cus * (dtype == SINCOSM_F64 ? 6 : 10));
    if (dtype == SINCOSM_F64) batched_small_kernel<double, 16><<<g, SmallGeom<16>::NT, 0, stream>>>(a);
    else batched_small_kernel<float, 16><<<g, SmallGeom<16>::NT, 0, stream>>>(a);
  }
  if (dtype == SINCOSM_F64) batched_kernel<double><<<L.slots, BNT, 0, stream>>>(a);
  else batched_kernel<float><<<L.slots, BNT, 0, stream>>>(a);
  timing_end(t, stream);
  SC_HIP(hipGetLastError());
  return SINCOSM_OK;
}

}  // extern "C"
