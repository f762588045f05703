// Matrix products with fused linear-combination epilogues on CDNA4 MFMA.
//
// Every product of the method (the scheme products of Section 2.1 and the
// two products of each double-angle step of Section 1) is one launch of this
// kernel family. A launch computes, per problem and per output tile,
//   D = sum_seg (lscale L_seg)(rscale R_seg)
// and writes several outputs O_o = e_o D + sum_q c_oq M_q + d_o I from the
// accumulators, reading the same tile of up to MAX_IN other matrices. This is
// how the scheme's updates such as I - A_2/2 + x_8 A_4 + A_16 are fused into
// the product that produces their last term.
//
// Design for gfx950:
//  * 16x16x4 MFMA (f64 or f32); each wave owns a WTM x WTN sub-tile as
//    FM x FN MFMA blocks held in accumulator registers.
//  * Operand tiles go through LDS, double buffered, one barrier per BK step in
//    the step's last substep of MFMAs; the global loads of the next tile are
//    issued before the MFMAs of the current one so their latency hides behind
//    the matrix core. They can be loaded straight into LDS (global_load_lds),
//    with no register round trip or LDS store instructions.
//  * LDS layouts: A as [m][k] with row pitch BK+1, B as [k][n] with row pitch
//    BN+16, so the 16-lane groups that feed one MFMA read distinct banks.
//  * All operands are internal buffers padded with zeros to a multiple of the
//    tile, so the main loop has no bounds checks; only outputs carry a limit.
//  * Block index -> tile: consecutive launch indices go to different XCDs, so
//    the index is first remapped to give each XCD a contiguous range of each
//    problem's tiles, then walked in groups of 8 tile rows.
#include "common.hpp"
#include "epilogue.hpp"

#include <mutex>
#include <vector>

namespace sc {

typedef double v4d __attribute__((ext_vector_type(4)));
typedef float v4f __attribute__((ext_vector_type(4)));
typedef double v2d __attribute__((ext_vector_type(2)));

template <typename T>
struct Mma;

template <>
struct Mma<double> {
  typedef v4d acc_t;
  typedef v2d vec_t;       // 16-byte global load
  static constexpr int VEC = 2;
  __device__ static inline acc_t mma(double a, double b, acc_t c) {
    return __builtin_amdgcn_mfma_f64_16x16x4f64(a, b, c, 0, 0, 0);
  }
  // 16x16 result: lane group lg (= lane / 16), register r -> row lg + 4 r
  __device__ static inline int row_in_block(int lg, int r) { return lg + 4 * r; }
};

template <>
struct Mma<float> {
  typedef v4f acc_t;
  typedef v4f vec_t;
  static constexpr int VEC = 4;
  __device__ static inline acc_t mma(float a, float b, acc_t c) {
    return __builtin_amdgcn_mfma_f32_16x16x4f32(a, b, c, 0, 0, 0);
  }
  // 16x16 result: lane group lg, register r -> row 4 lg + r
  __device__ static inline int row_in_block(int lg, int r) { return 4 * lg + r; }
};

// Map a launch index to (problem, tile row, tile column). Consecutive launch
// indices go to different XCDs (index mod 8). When a problem's tile count is a
// multiple of 8, XCD x owns the x-th eighth of the tiles of every problem, and
// its successive workgroups alternate between the problems, so problems of
// unequal k-work are spread evenly over the XCDs.
__device__ inline void tile_coords(int np, int BM, int BN, int nprob, int& p, int& tm, int& tn) {
  const int tmc = np / BM, tnc = np / BN, tiles = tmc * tnc;
  const int b = blockIdx.x;
  int t;
  if ((tiles & 7) == 0) {
    const int j = b >> 3;
    p = j % nprob;
    t = (b & 7) * (tiles >> 3) + j / nprob;
  } else {
    p = b / tiles;
    t = b - p * tiles;
  }
  constexpr int GROUP = 8;
  const int group = t / (GROUP * tnc);
  const int first = group * GROUP;
  const int rows = (tmc - first) < GROUP ? (tmc - first) : GROUP;
  const int in_group = t - group * GROUP * tnc;
  tm = first + in_group % rows;
  tn = in_group / rows;
}

// The k loop. Each BK step is KK = BK/4 substeps of FM x FN MFMAs. The
// operand fragments of a substep are read from LDS one substep ahead (double
// buffered in registers). The loads of the next BK step are issued at the
// start of the current one; the workgroup synchronises in the step's last
// substep, and the first fragments of the next step are read while that
// substep's MFMAs run, so the barrier sits between MFMAs that are already
// queued. The segment cursor of the loads (pointers, k offset, operand scales)
// is uniform state advanced incrementally.
//
// Two ways to fill the LDS buffers:
//  * staged (DL = 0): global loads into registers; in the last substep they
//    are stored (scaled) into the other buffer, padded so that the fragment
//    reads hit distinct banks.
//  * direct (DL = 1, 2): global_load_lds_dwordx4 writes the tile straight into
//    the other buffer, 16 bytes per lane, with no register round trip and no
//    LDS store instructions; the permutation that avoids bank conflicts is
//    chosen through the source addresses, and a launch with operand scales
//    (DL = 2) applies them to the fragments after the LDS reads.
//
// LDS hazards (two buffers, barrier B_k in step k): the store or load into
// buffer (k+1)&1 happens after the wave passed B_{k-1} (staged: in step k's
// last substep; direct: at the start of step k). Every read of that buffer
// belongs to step k-1 (the prefetch after B_{k-2} and the substep reads before
// B_{k-1}), and the barrier waits for the wave's outstanding LDS reads, so
// they completed before any wave passed B_{k-1}. Before B_k each wave waits
// for its own stores or direct loads (vmcnt for the latter); the reads of
// buffer (k+1)&1 in step k+1 start after B_k. With two k groups this holds
// for each group's own pair of buffers, k counting that group's steps; the
// groups take equally many steps and share the barriers.
//
// COND: the launch is decided on the device (DevCond): every workgroup first
// reads the plan record and returns when the launch does not apply; operand
// scales marked SCALE_2_POW_MINUS_S take the record's 2^-s. Launches without
// a device plan use the COND = false kernels, which carry none of this.
template <typename T, int BM, int BN, int BK, int WGM, int WGN, int WPE, int DL, int KS, bool COND>
__global__ __launch_bounds__(WGM * WGN * KS * 64) __attribute__((amdgpu_waves_per_eu(WPE, WPE)))
void gemm_kernel(const GemmLaunch g) {
  using M = Mma<T>;
  using acc_t = typename M::acc_t;
  using vec_t = typename M::vec_t;
  constexpr int NW = WGM * WGN;   // waves of one k group
  constexpr int NT = NW * 64;     // threads of one k group
  constexpr int WTM = BM / WGM, WTN = BN / WGN;
  constexpr int FM = WTM / 16, FN = WTN / 16;
  constexpr int LDA = DL ? BK : BK + 1, LDB = DL ? BN : BN + 16;
  constexpr int VEC = M::VEC;
  constexpr int KK = BK / 4;
  constexpr int A_LOADS = BM * BK / VEC / NT;
  constexpr int B_LOADS = BK * BN / VEC / NT;
  constexpr int LDE = BN + VEC;
  constexpr int GROUP_ELEMS = 2 * (BM * LDA + BK * LDB);   // the two LDS buffers of a k group
  constexpr int STAGE_ELEMS = KS * GROUP_ELEMS;
  constexpr int RED_ELEMS = (KS - 1) * BM * BN;   // one region per group after the first
  constexpr int EPI_ELEMS = WTM * LDE;
  constexpr int SMEM_ELEMS = STAGE_ELEMS > EPI_ELEMS ? (STAGE_ELEMS > RED_ELEMS ? STAGE_ELEMS : RED_ELEMS)
                                                     : (EPI_ELEMS > RED_ELEMS ? EPI_ELEMS : RED_ELEMS);
  static_assert(FM >= 1 && FN >= 1 && WTM % 16 == 0 && WTN % 16 == 0, "wave tile");
  static_assert(A_LOADS >= 1 && A_LOADS * VEC * NT == BM * BK, "A staging");
  static_assert(B_LOADS >= 1 && B_LOADS * VEC * NT == BK * BN, "B staging");
  static_assert(BK % 8 == 0 && BK % VEC == 0 && BN % VEC == 0, "k tiling (even substep count)");
  // Direct loads: one wave instruction fills a 1 KiB chunk of LDS (64 lanes x
  // one 16-byte slot of VEC values). An A row (BK values) has QA slots and a
  // chunk holds RA rows; a B row (BN values) has QB slots and a chunk holds RB
  // rows. Rows of A repeat their bank offsets every PA rows (256 bytes: 64
  // banks of 4 bytes); the 16 columns of one B fragment span 1 / GB of the
  // banks.
  constexpr int QA = BK / VEC, QB = BN / VEC;
  constexpr int RA = 64 / QA, RB = 64 / QB;
  constexpr int PA = 256 / (BK * (int)sizeof(T)), GB = 256 / (16 * (int)sizeof(T));
  static_assert(!DL || (BK * sizeof(T) >= 64 && BK * sizeof(T) <= 128 && PA * QA == 16 &&
                        QB <= 64 && 64 % QB == 0 && A_LOADS * NW * RA == BM && B_LOADS * NW * RB == BK),
                "direct loads: 64- or 128-byte A rows, B rows that divide 1 KiB");

  static_assert(KS == 1 || KS == 2 || KS == 4, "one, two or four k groups");

  // k groups (KS = 2, 4): the waves split into KS groups of WGM x WGN waves
  // that take every KS-th k step of the same output tile, each with its own
  // LDS buffers; at the end the other groups' accumulators are added to the
  // first's through LDS in group order (a fixed order, so results are
  // deterministic; KS = 2 gives the sum it always gave).
  const int tid = threadIdx.x;
  const int lane = tid & 63, wave = tid >> 6;
  const int grp = KS > 1 ? __builtin_amdgcn_readfirstlane(wave / NW) : 0;
  const int wl = wave - grp * NW;   // wave within its group
  const int tidg = tid - grp * NT;  // thread within its group
  const int wm = wl / WGN, wn = wl % WGN;
  const int lr = lane & 15, lg = lane >> 4;

  __shared__ __attribute__((aligned(16))) T smem[SMEM_ELEMS];
  T* const As0 = smem + grp * GROUP_ELEMS;
  T* const Bs0 = As0 + 2 * BM * LDA;

  int dyn_s = 0, dyn_level = 0;
  if constexpr (COND) {
    if (!cond_applies(g.cond, dyn_s, dyn_level)) return;   // uniform: the whole workgroup leaves
  }

  const int np = g.np;
  int p, tile_m, tile_n;
  if (COND && g.cond.select) {
    tile_coords(np, BM, BN, 1, p, tile_m, tile_n);
    p = cond_problem(g.cond, g.nprob, dyn_level);
    if (p < 0) return;
  } else {
    tile_coords(np, BM, BN, g.nprob, p, tile_m, tile_n);
  }
  const Problem& P = g.prob[p];

  acc_t acc[FM][FN];
#pragma unroll
  for (int i = 0; i < FM; ++i)
#pragma unroll
    for (int j = 0; j < FN; ++j)
#pragma unroll
      for (int r = 0; r < 4; ++r) acc[i][j][r] = (T)0;

  // Global offsets of this thread's loads and their LDS places. Staged loads
  // go through registers into padded rows. A direct load writes lane l's 16
  // bytes to slot l of the wave's 1 KiB chunk, so the lane picks the source
  // that belongs there: slot q of A row r holds slot q ^ ((r / PA) % QA) of
  // that row, slot q of B row k holds column slot q ^ (sizeof(T) (k % GB)).
  // The fragment reads undo the permutation; the 16 lanes x 4 k of one read
  // then spread evenly over the 64 banks.
  int offA[A_LOADS], offB[B_LOADS], ldsA[A_LOADS], ldsB[B_LOADS];
  const int wave_u = __builtin_amdgcn_readfirstlane(wl);
#pragma unroll
  for (int i = 0; i < A_LOADS; ++i) {
    if (DL) {
      const int c = i * NW + wave_u;
      const int row = c * RA + lane / QA;
      offA[i] = row * np + VEC * ((lane % QA) ^ ((row / PA) % QA));
      ldsA[i] = c * 64 * VEC;
    } else {
      const int e = (i * NT + tidg) * VEC;
      const int r = e / BK, c = e - r * BK;
      offA[i] = r * np + c;
      ldsA[i] = r * LDA + c;
    }
  }
#pragma unroll
  for (int i = 0; i < B_LOADS; ++i) {
    if (DL) {
      const int c = i * NW + wave_u;
      const int k = c * RB + lane / QB;
      offB[i] = k * np + VEC * ((lane % QB) ^ ((int)sizeof(T) * (k % GB)));
      ldsB[i] = c * 64 * VEC;
    } else {
      const int e = (i * NT + tidg) * VEC;
      const int r = e / BN, c = e - r * BN;
      offB[i] = r * np + c;
      ldsB[i] = r * LDB + c;
    }
  }

  const int nseg = P.nseg;
  const int nks = np / BK;
  const int nkt = nseg * nks;
  const int64_t a_tile = (int64_t)tile_m * BM * np;
  const int64_t b_tile = (int64_t)tile_n * BN;

  // The launch's segments are read once; the cursors switch between them with
  // selects, so the k loop issues no scalar memory loads (they share a wait
  // counter with the LDS reads and would make the loop wait for those).
  static_assert(MAX_SEG == 3, "segment table");
  const T* segL[MAX_SEG];
  const T* segR[MAX_SEG];
  T segl[MAX_SEG], segr[MAX_SEG];
#pragma unroll
  for (int s = 0; s < MAX_SEG; ++s) {
    const int si = s < nseg ? s : 0;
    segL[s] = (const T*)P.seg[si].L + a_tile;
    segR[s] = (const T*)P.seg[si].R + b_tile;
    segl[s] = (T)(COND ? resolve_scale(P.seg[si].lscale, dyn_s) : P.seg[si].lscale);
    segr[s] = (T)(COND ? resolve_scale(P.seg[si].rscale, dyn_s) : P.seg[si].rscale);
  }
  auto pick = [](auto a0, auto a1, auto a2, int s) { return s == 0 ? a0 : (s == 1 ? a1 : a2); };

  // uniform cursor: the next tile to load
  int cseg = 0, ck0 = 0;
  const T* Lc = segL[0];
  const T* Rc = segR[0];
  T lsc = segl[0], rsc = segr[0];
  auto advance = [&]() {
    ck0 += BK;
    if (ck0 == np) {
      ck0 = 0;
      ++cseg;
      const int s = cseg < nseg ? cseg : nseg - 1;
      Lc = pick(segL[0], segL[1], segL[2], s);
      Rc = pick(segR[0], segR[1], segR[2], s);
      lsc = pick(segl[0], segl[1], segl[2], s);
      rsc = pick(segr[0], segr[1], segr[2], s);
    }
  };
  // a k group loads every KS-th step, starting at its own index
  auto advance_group = [&]() {
#pragma unroll
    for (int q = 0; q < KS; ++q) advance();
  };
  for (int q = 0; q < grp; ++q) advance();

  // staged: global -> registers (gload), registers -> LDS buffer with the
  // operand scales applied (lstore)
  T pl = (T)1, pr = (T)1;   // scales of the tile held in ra / rb
  vec_t ra[DL ? 1 : A_LOADS], rb[DL ? 1 : B_LOADS];
  auto gload = [&]() {
    const T* L = Lc + ck0;
    const T* R = Rc + (int64_t)ck0 * np;
#pragma unroll
    for (int i = 0; i < (DL ? 0 : A_LOADS); ++i) ra[i] = *(const vec_t*)(L + offA[i]);
#pragma unroll
    for (int i = 0; i < (DL ? 0 : B_LOADS); ++i) rb[i] = *(const vec_t*)(R + offB[i]);
    pl = lsc;
    pr = rsc;
    advance_group();
  };
  auto lstore = [&](int buf) {
    T* as = As0 + buf * (BM * LDA);
    T* bs = Bs0 + buf * (BK * LDB);
    if (pl != (T)1 || pr != (T)1) {
#pragma unroll
      for (int i = 0; i < (DL ? 0 : A_LOADS); ++i) ra[i] = ra[i] * pl;
#pragma unroll
      for (int i = 0; i < (DL ? 0 : B_LOADS); ++i) rb[i] = rb[i] * pr;
    }
#pragma unroll
    for (int i = 0; i < (DL ? 0 : A_LOADS); ++i)
#pragma unroll
      for (int q = 0; q < VEC; ++q) as[ldsA[i] + q] = ra[i][q];
#pragma unroll
    for (int i = 0; i < (DL ? 0 : B_LOADS); ++i) *(vec_t*)(bs + ldsB[i]) = rb[i];
  };
  // direct: global -> LDS buffer; the wave's loads complete (vmcnt) before the
  // barrier that publishes them
  auto dload = [&](int buf) {
    typedef __attribute__((address_space(3))) void lds_void;
    typedef __attribute__((address_space(1))) void glb_void;
    const T* L = Lc + ck0;
    const T* R = Rc + (int64_t)ck0 * np;
    T* as = As0 + buf * (BM * LDA);
    T* bs = Bs0 + buf * (BK * LDB);
#pragma unroll
    for (int i = 0; i < (DL ? A_LOADS : 0); ++i)
      __builtin_amdgcn_global_load_lds((glb_void*)(L + offA[i]), (lds_void*)(as + ldsA[i]), 16, 0, 0);
#pragma unroll
    for (int i = 0; i < (DL ? B_LOADS : 0); ++i)
      __builtin_amdgcn_global_load_lds((glb_void*)(R + offB[i]), (lds_void*)(bs + ldsB[i]), 16, 0, 0);
    advance_group();
  };
  auto dwait = [&]() {
    if (DL) asm volatile("s_waitcnt vmcnt(0)" ::: "memory");
  };

  // Direct loads: the lane's read offsets for each substep (A) and each
  // fragment column (B) under the permutation above. The A rows of a lane
  // differ by multiples of 16 = PA QA, so they share the permutation; its k
  // in substep kk is 4 kk + lg, and k % GB = lg % GB for B.
  int rdA[DL ? KK : 1], rdB[DL ? FN : 1];
  if (DL) {
    const int ra = wm * WTM + lr;
#pragma unroll
    for (int kk = 0; kk < (DL ? KK : 0); ++kk) {
      const int k = kk * 4 + lg;
      rdA[kk] = ra * LDA + VEC * ((k / VEC) ^ ((ra / PA) % QA)) + k % VEC;
    }
#pragma unroll
    for (int j = 0; j < (DL ? FN : 0); ++j) {
      const int col = wn * WTN + j * 16 + lr;
      rdB[j] = lg * LDB + VEC * ((col / VEC) ^ ((int)sizeof(T) * (lg % GB))) + col % VEC;
    }
  }
  // Fragment reads. With direct loads of a launch that has operand scales
  // (DL = 2) the scales of the k step the fragments belong to are applied
  // here: the same products as when staging.
  T fa[2][FM], fb[2][FN];
  auto lread = [&](int buf, int kk, T sa, T sb, T (&a)[FM], T (&b)[FN]) {
    if (DL) {
      const T* as = As0 + buf * (BM * LDA) + rdA[DL ? kk : 0];
      const T* bs = Bs0 + buf * (BK * LDB) + kk * 4 * LDB;
#pragma unroll
      for (int i = 0; i < FM; ++i) a[i] = as[i * 16 * LDA];
#pragma unroll
      for (int j = 0; j < FN; ++j) b[j] = bs[rdB[DL ? j : 0]];
      if (DL == 2) {
#pragma unroll
        for (int i = 0; i < FM; ++i) a[i] *= sa;
#pragma unroll
        for (int j = 0; j < FN; ++j) b[j] *= sb;
      }
    } else {
      (void)sa;
      (void)sb;
      const T* as = As0 + buf * (BM * LDA) + (wm * WTM + lr) * LDA + lg + kk * 4;
      const T* bs = Bs0 + buf * (BK * LDB) + (lg + kk * 4) * LDB + wn * WTN + lr;
#pragma unroll
      for (int i = 0; i < FM; ++i) a[i] = as[i * 16 * LDA];
#pragma unroll
      for (int j = 0; j < FN; ++j) b[j] = bs[j * 16];
    }
  };
  // scales of the step whose first fragments are read next (DL = 2): the
  // group's steps are KS apart, and its first one lies in segment 0
  int rseg = 0, rk = grp;
  auto next_scales = [&](T& sa, T& sb) {
#pragma unroll
    for (int q = 0; q < KS; ++q) {
      if (++rk == nks) {
        rk = 0;
        ++rseg;
      }
    }
    const int s = rseg < nseg ? rseg : nseg - 1;
    sa = pick(segl[0], segl[1], segl[2], s);
    sb = pick(segr[0], segr[1], segr[2], s);
  };

  if (nkt > 0) {
    if (DL) {
      dload(0);
    } else {
      gload();
      lstore(0);
    }
  }
  dwait();
  __syncthreads();
  T sa_c = segl[0], sb_c = segr[0];   // operand scales of the current step (DL = 2)
  if (nkt > 0) lread(0, 0, sa_c, sb_c, fa[0], fb[0]);

  // Each group takes nkt / KS steps: the padded order is a multiple of BK KS
  // (checked at launch), so nkt is too and both groups meet every barrier.
  const int nit = nkt / KS;
  for (int it = 0; it < nit; ++it) {
    const int cur = it & 1;
    T sa_n = (T)1, sb_n = (T)1;   // of the group's next step
    if (DL == 2) next_scales(sa_n, sb_n);
    if (it + 1 < nit) {
      if (DL) dload(cur ^ 1);
      else gload();
    }
#pragma unroll
    for (int kk = 0; kk < KK; ++kk) {
      const int f = kk & 1;
      if (kk + 1 < KK) {
        lread(cur, kk + 1, sa_c, sb_c, fa[f ^ 1], fb[f ^ 1]);
      } else {
        // unconditional: on the last step these move stale values that are never
        // used, and the fragment registers keep one assignment around the loop
        lstore(cur ^ 1);
        dwait();
        __syncthreads();
        lread(cur ^ 1, 0, sa_n, sb_n, fa[f ^ 1], fb[f ^ 1]);
      }
#pragma unroll
      for (int i = 0; i < FM; ++i)
#pragma unroll
        for (int j = 0; j < FN; ++j) acc[i][j] = M::mma(fa[f][i], fb[f][j], acc[i][j]);
    }
    sa_c = sa_n;
    sb_c = sb_n;
  }

  if constexpr (KS > 1) {
    // the other groups' accumulators -> LDS, group g into region g - 1
    // (element-major, so a wave's 64 lanes write consecutive slots), then
    // added to the first group's in group order
    constexpr int NACC = FM * FN * 4;
    static_assert(NACC * NT == BM * BN && RED_ELEMS <= SMEM_ELEMS, "reduction buffer");
    __syncthreads();   // every wave is done with the stage buffers
    if (grp > 0) {
      T* const red = smem + (grp - 1) * (BM * BN);
#pragma unroll
      for (int i = 0; i < FM; ++i)
#pragma unroll
        for (int j = 0; j < FN; ++j)
#pragma unroll
          for (int r = 0; r < 4; ++r) red[((i * FN + j) * 4 + r) * NT + tidg] = acc[i][j][r];
    }
    __syncthreads();
    if (grp == 0) {
#pragma unroll
      for (int q = 0; q < KS - 1; ++q)
#pragma unroll
        for (int i = 0; i < FM; ++i)
#pragma unroll
          for (int j = 0; j < FN; ++j)
#pragma unroll
            for (int r = 0; r < 4; ++r)
              acc[i][j][r] += smem[q * (BM * BN) + ((i * FN + j) * 4 + r) * NT + tidg];
    }
    __syncthreads();   // the epilogue reuses the buffer
  }
  // the epilogue's band owners are the first group's waves (the second
  // group's wave rows lie beyond WGM); all KS x NT threads write the outputs
  epilogue_bands<T, BM, BN, WGM, WGN, M, acc_t, FM, FN, KS * NT>(P, np, tile_m, tile_n, acc, smem);
}

// ----------------------------------------------------------------------------
// Tile configurations. Index -> (BM = BN, BK, wave grid, waves per SIMD).
//   0: 128 x 128, BK 16, 2 x 2 waves of 64 x 64   (large n)
//   1:  64 x  64, BK 16, 2 x 2 waves of 32 x 32   (mid n)
//   2:  32 x  32, BK 16, 2 x 2 waves of 16 x 16   (small n)
// ----------------------------------------------------------------------------
int tile_size(int tile) {
  switch (tile) {
    case 0: return 128;
    case 1: return 64;
    default: return 32;
  }
}

int choose_tile(Arith ar, int64_t n) {
  if (ar == Arith::I8X5) return n >= 1536 ? 0 : 1;   // its products need multiples of 64
  if (n >= 1536) return 0;
  if (n >= 256) return 1;
  return 2;
}

template <typename T, int BM, int BN, int BK, int WGM, int WGN, int WPE, int DL, int KS, bool COND>
static void launch_variant(const GemmLaunch& g, bool scaled, int tiles, hipStream_t stream) {
  if constexpr (DL != 0) {
    if (scaled)
      gemm_kernel<T, BM, BN, BK, WGM, WGN, WPE, 2, KS, COND><<<tiles, WGM * WGN * KS * 64, 0, stream>>>(g);
    else
      gemm_kernel<T, BM, BN, BK, WGM, WGN, WPE, 1, KS, COND><<<tiles, WGM * WGN * KS * 64, 0, stream>>>(g);
  } else {
    (void)scaled;
    gemm_kernel<T, BM, BN, BK, WGM, WGN, WPE, 0, KS, COND><<<tiles, WGM * WGN * KS * 64, 0, stream>>>(g);
  }
}

template <typename T, int BM, int BN, int BK, int WGM, int WGN, int WPE, int DL, int KS>
static sincosm_status launch_cfg(const GemmLaunch& g, hipStream_t stream) {
  const int tiles = (g.np / BM) * (g.np / BN) * (g.cond.plan && g.cond.select ? 1 : g.nprob);
  if (tiles <= 0) return SINCOSM_OK;
  if ((g.np / BK) % KS != 0) return SINCOSM_E_ARG;   // k groups need a step count divisible by KS
  bool scaled = false;
  for (int p = 0; p < g.nprob; ++p)
    for (int s = 0; s < g.prob[p].nseg; ++s)
      scaled |= g.prob[p].seg[s].lscale != 1.0 || g.prob[p].seg[s].rscale != 1.0;
  if (g.cond.plan)
    launch_variant<T, BM, BN, BK, WGM, WGN, WPE, DL, KS, true>(g, scaled, tiles, stream);
  else
    launch_variant<T, BM, BN, BK, WGM, WGN, WPE, DL, KS, false>(g, scaled, tiles, stream);
  SC_HIP(hipGetLastError());
  return SINCOSM_OK;
}


// ----------------------------------------------------------------------------
// Kernel configurations the autotuner chooses among. Each entry: tile rows and
// columns, k depth, wave grid, waves per SIMD, direct loads into LDS, k groups.
// Entries 0, 1, 2 are the defaults for the three padding granularities 128, 64
// and 32.
// ----------------------------------------------------------------------------

#define SC_CFG(T, BM, BN, BK, WGM, WGN, WPE, DL) \
  { BM, BN, BK, WGM, WGN, WPE, DL, 1, &launch_cfg<T, BM, BN, BK, WGM, WGN, WPE, DL, 1> }
#define SC_CFG_KS(T, BM, BN, BK, WGM, WGN, WPE, DL, KS) \
  { BM, BN, BK, WGM, WGN, WPE, DL, KS, &launch_cfg<T, BM, BN, BK, WGM, WGN, WPE, DL, KS> }

static const KernelCfg kF64[] = {
    SC_CFG(double, 128, 128, 16, 2, 2, 2, 0), SC_CFG(double, 64, 64, 16, 2, 2, 2, 0),
    SC_CFG(double, 32, 32, 16, 2, 2, 2, 0),   SC_CFG(double, 128, 128, 32, 2, 2, 1, 0),
    SC_CFG(double, 256, 128, 16, 4, 2, 2, 0), SC_CFG(double, 128, 128, 16, 2, 4, 2, 0),
    SC_CFG(double, 128, 64, 16, 2, 2, 2, 0),  SC_CFG(double, 64, 128, 16, 2, 2, 2, 0),
    SC_CFG(double, 128, 128, 8, 2, 2, 2, 0),  SC_CFG(double, 256, 128, 16, 4, 2, 2, 1),
    SC_CFG(double, 128, 128, 16, 2, 2, 2, 1), SC_CFG(double, 128, 128, 16, 2, 4, 2, 1),
    SC_CFG(double, 64, 64, 16, 2, 2, 2, 1),   SC_CFG(double, 128, 64, 16, 2, 2, 2, 1),
    SC_CFG(double, 64, 128, 16, 2, 2, 2, 1),
    SC_CFG_KS(double, 64, 64, 16, 2, 2, 2, 1, 2), SC_CFG_KS(double, 128, 64, 16, 2, 2, 2, 1, 2),
    SC_CFG_KS(double, 64, 64, 16, 2, 2, 2, 0, 2),
    SC_CFG_KS(double, 64, 64, 16, 2, 2, 4, 1, 4), SC_CFG_KS(double, 64, 64, 16, 2, 2, 4, 0, 4),
};
static const KernelCfg kF32[] = {
    SC_CFG(float, 128, 128, 16, 2, 2, 2, 0), SC_CFG(float, 64, 64, 16, 2, 2, 2, 0),
    SC_CFG(float, 32, 32, 32, 2, 2, 2, 0),   SC_CFG(float, 128, 128, 32, 2, 2, 2, 0),
    SC_CFG(float, 256, 128, 16, 4, 2, 2, 0), SC_CFG(float, 128, 128, 16, 2, 4, 2, 0),
    SC_CFG(float, 64, 64, 32, 2, 2, 2, 0),   SC_CFG(float, 128, 128, 32, 2, 2, 2, 1),
    SC_CFG(float, 256, 128, 16, 4, 2, 2, 1), SC_CFG(float, 128, 128, 16, 2, 2, 2, 1),
    SC_CFG(float, 64, 64, 32, 2, 2, 2, 1),
    SC_CFG_KS(float, 64, 64, 32, 2, 2, 2, 1, 2), SC_CFG_KS(float, 64, 64, 16, 2, 2, 2, 1, 2),
    SC_CFG_KS(float, 64, 64, 32, 2, 2, 4, 1, 4),
};

const KernelCfg* cfg_table(Arith ar, int& count) {
  if (ar == Arith::F64) { count = (int)(sizeof(kF64) / sizeof(kF64[0])); return kF64; }
  if (ar == Arith::F32) { count = (int)(sizeof(kF32) / sizeof(kF32[0])); return kF32; }
  count = 0;
  return nullptr;
}

// Launch class of a product launch for the tuning table: 0 one problem with at
// most one k-segment, 1 several problems of equal k-work, 2 the rest.
static int launch_class(const GemmLaunch& g) {
  if (g.cond.plan && g.cond.select) return 0;   // one of the problems runs, each a single product
  if (g.nprob <= 1) return g.prob[0].nseg <= 1 ? 0 : 2;
  for (int p = 1; p < g.nprob; ++p)
    if (g.prob[p].nseg != g.prob[0].nseg) return 2;
  return 1;
}

// Operand scales that are powers of two (with sign) commute with every
// rounding of a product: the sum over k of (ls a)(rs b) is exactly ls rs times
// the unscaled sum, away from overflow and the subnormal range. When all
// k-segments of a problem carry one such factor ls rs, it moves into the
// coefficients e_o of that problem's outputs (O_o = e_o D + ...) and the
// kernels run without operand scaling; the results are the same. The factor
// is kept within 2^-60 .. 2^60 so the unscaled accumulation stays far from
// the float32 overflow threshold for the plans' operands.
static bool pow2_scale(double x) {
  int e = 0;
  return x != 0.0 && fabs(frexp(x, &e)) == 0.5;
}

static bool fold_scales(const GemmLaunch& g, GemmLaunch& out) {
  bool changed = false;
  out = g;
  for (int p = 0; p < g.nprob; ++p) {
    const Problem& P = g.prob[p];
    if (P.nseg == 0) continue;
    const double f = P.seg[0].lscale * P.seg[0].rscale;
    bool scaled = false, ok = fabs(f) >= 0x1p-60 && fabs(f) <= 0x1p60;
    for (int s = 0; ok && s < P.nseg; ++s) {
      ok = pow2_scale(P.seg[s].lscale) && pow2_scale(P.seg[s].rscale) && P.seg[s].lscale * P.seg[s].rscale == f;
      scaled |= P.seg[s].lscale != 1.0 || P.seg[s].rscale != 1.0;
    }
    if (!ok || !scaled) continue;
    Problem& Q = out.prob[p];
    for (int s = 0; s < Q.nseg; ++s) Q.seg[s].lscale = Q.seg[s].rscale = 1.0;
    for (int o = 0; o < Q.nout; ++o) Q.out[o].e *= f;
    changed = true;
  }
  return changed;
}

sincosm_status launch_gemm(Arith ar, int tile, const GemmLaunch& g0, hipStream_t stream, void* scratch) {
  if (g0.np % tile_size(tile) != 0) return SINCOSM_E_ARG;
  if (ar == Arith::I8X5) {
    bool products = false;
    for (int p = 0; p < g0.nprob; ++p) products |= g0.prob[p].nseg > 0;
    if (products) return launch_gemm_i8x5(g0, scratch, stream);
    ar = Arith::F64;   // epilogue only: float64 storage
  }
  GemmLaunch folded;
  const GemmLaunch& g = fold_scales(g0, folded) ? folded : g0;
  if (ar == Arith::BF16X3) return launch_gemm_bf16x3(tile, g, stream);
  int count = 0;
  const KernelCfg* t = cfg_table(ar, count);
  if (!t) return SINCOSM_E_UNSUPPORTED;
  int idx = tuned_cfg(ar, launch_class(g), g.np);
  if (idx < 0 || idx >= count || g.np % t[idx].bm != 0 || g.np % t[idx].bn != 0 ||
      (g.np / t[idx].bk) % t[idx].ks != 0)
    idx = tile;
  return t[idx].fn(g, stream);
}

}  // namespace sc
