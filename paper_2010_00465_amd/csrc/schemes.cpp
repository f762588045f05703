// Host side of sincosm_eval: validation, workspace layout, plan read-back and
// the launch sequences of the four schemes and of the double-angle steps.
//
// Scheme launch sequences (X = 2^-s A is never formed: the factor goes into
// the operand scales of the first and last products; Y = X^2 is the paper's
// A_2, Y2 its A_4, and so on). "->" lists the outputs written by the fused
// epilogue of that product.
//
// 3 products (Algorithm3cA, Algorithm3sA):
//   G1 Y = (sA)(sA)                       -> Y
//   G2 Y Y  -> C = I - Y/2 + Y2/24,  V = I - Y/6 + Y2/120
//   G3 S = (sA) V
// 4 products (Algorithm4cA, Algorithm4sA):
//   G1 Y;  G2 Y2 = Y Y -> Y2, W = -Y/6! + Y2/8!, Pc = I - Y/2 + Y2/24, Ps = I - Y/6 + Y2/120
//   G3 Y4 = Y2 W -> C = Pc + Y4, V = Ps + (6!/7!) Y4
//   G4 S = (sA) V
// 5 products (Algorithm4cA, Algorithm5sA; extended plan only):
//   G1 Y;  G2 Y2 = Y Y -> Y2, W = -Y/6! + Y2/8!, Ws = -Y/7! + Y2/9!, Pc = I - Y/2 + Y2/24,
//        Ps = I - Y/6 + Y2/120
//   G3 Y4 = Y2 W  -> C = Pc + Y4
//   G4 Y4s = Y2 Ws -> V = Ps + Y4s
//   G5 S = (sA) V
// 6 products (Algorithm6cA with eq:cosm8, Algorithm6sA):
//   G1 Y;  G2 Y2 = Y Y -> Y2, W = x1 Y + x2 Y2
//   G3 Y4 = Y2 W (paper A_8) -> Y4, L = x3 Y2 + Y4, R = x4 I + x5 Y + x6 Y2 + x7 Y4,
//        Pc = I - Y/2 + x8 Y2, Q = z5 I + z5 Y + z6 Y2 + z7 Y4, P = z0 I + z1 Y + z2 Y2 + z3 Y4
//   G4 T = L R (A_16) -> C = Pc + T, Q += z8 C, P += z4 C
//   G5 U = Q Y4 (C_24) -> V = P + U
//   G6 S = (sA) V
// 7 products (Algorithm7cA with Coefs7cA, Algorithm7sA with Coefs7sA):
//   G1 Y;  G2 Y2 = Y Y
//   G3 Y3 = Y2 Y (A_6) -> C_j = a0j I + a1j Y + a2j Y2 + a3j Y3 (j = 1..4),
//        P = z0 I + z1 Y + z2 Y2 + z3 Y3, Q = z6 I + z7 Y + z8 Y2 + z9 Y3
//   G4 K = C4 C4 -> Y6 = C3 + K (A_12), L = C2 + Y6
//   G5 T = L Y6 (A_24) -> C = C1 + T, Q += z10 Y6 + z11 C, P += z4 Y6 + z5 C
//   G6 U = Q C (C_48) -> V = P + U
//   G7 S = (sA) V
// Double angle (Section 1), s times, from the old pair:
//   one launch, two problems sharing the left operand S:
//   [P | Q] = S [S | C] -> C' = I - 2 P, S' = 2 Q.
#include <math.h>
#include <stdlib.h>
#include <string.h>

#include <mutex>

#include <cstdio>
#include <cstdlib>

#include "schemes.hpp"
#include "coeffs.hpp"

namespace sc {

// ----------------------------------------------------------------------------
// Problem builders
// ----------------------------------------------------------------------------
Problem make_problem(int nvalid) {
  Problem p;
  memset(&p, 0, sizeof(p));
  p.nvalid = nvalid;
  return p;
}

void add_seg(Problem& p, const void* L, const void* R, int64_t ld, double lsc, double rsc) {
  if (p.nseg >= MAX_SEG) abort();
  Seg& s = p.seg[p.nseg++];
  s.L = L; s.R = R; s.ldl = ld; s.ldr = ld; s.lscale = lsc; s.rscale = rsc;
}

void add_in(Problem& p, const void* m, int64_t ld) {
  if (p.nin >= MAX_IN) abort();  // launch sequences are fixed; overflow is a programming error
  p.in[p.nin].p = m;
  p.in[p.nin].ld = ld;
  p.nin++;
}


void add_out(Problem& p, const Target& t, double e, double d, std::initializer_list<double> c) {
  if (p.nout >= MAX_OUT || c.size() > (size_t)MAX_IN) abort();
  EpiOut& o = p.out[p.nout++];
  o.p = t.p; o.ld = t.ld; o.lim = t.lim; o.f64 = t.f64 ? 1 : 0;
  o.e = e; o.d = d;
  int q = 0;
  for (double v : c) o.c[q++] = v;
  for (; q < MAX_IN; ++q) o.c[q] = 0.0;
}

GemmLaunch two(const Problem& p0, const Problem& p1, int np) {
  GemmLaunch g;
  memset(&g, 0, sizeof(g));
  g.np = np;
  g.nprob = 2;
  g.prob[0] = p0;
  g.prob[1] = p1;
  return g;
}

GemmLaunch three(const Problem& p0, const Problem& p1, const Problem& p2, int np) {
  GemmLaunch g;
  memset(&g, 0, sizeof(g));
  g.np = np;
  g.nprob = 3;
  g.prob[0] = p0;
  g.prob[1] = p1;
  g.prob[2] = p2;
  return g;
}

GemmLaunch one(const Problem& p, int np) {
  GemmLaunch g;
  memset(&g, 0, sizeof(g));
  g.np = np;
  g.nprob = 1;
  g.prob[0] = p;
  return g;
}

// ----------------------------------------------------------------------------
// Workspace layout of sincosm_eval
// ----------------------------------------------------------------------------

bool modes_for(int64_t n, int dtype, int prod, Modes& m) {
  m.user_f64 = dtype == SINCOSM_F64;
  if (dtype == SINCOSM_F64) {
    m.sq = Arith::F64; m.sq_f64 = true;
    if (prod == SINCOSM_PROD_NATIVE) { m.poly = Arith::F64; m.poly_f64 = true; }
    else if (prod == SINCOSM_PROD_I8X5) {
      if (n > 16384) return false;   // int32 accumulation of the slice products
      m.poly = Arith::I8X5; m.poly_f64 = true;
    }
    else if (prod == SINCOSM_PROD_F32) { m.poly = Arith::F32; m.poly_f64 = false; }
    else if (prod == SINCOSM_PROD_BF16X3) { m.poly = Arith::BF16X3; m.poly_f64 = false; }
    else return false;
  } else if (dtype == SINCOSM_F32) {
    m.sq = Arith::F32; m.sq_f64 = false;
    if (prod == SINCOSM_PROD_NATIVE || prod == SINCOSM_PROD_F32) { m.poly = Arith::F32; m.poly_f64 = false; }
    else if (prod == SINCOSM_PROD_BF16X3) { m.poly = Arith::BF16X3; m.poly_f64 = false; }
    else return false;
  } else {
    return false;
  }
  m.tile = choose_tile(m.poly, n);
  const int ts = tile_size(m.tile);
  m.np = (n + ts - 1) / ts * ts;
  return true;
}


Layout layout_for(const Modes& m) {
  Layout L;
  const size_t np2 = (size_t)m.np * (size_t)m.np;
  const size_t pe = m.poly_f64 ? 8 : 4, se = m.sq_f64 ? 8 : 4;
  size_t off = 0;
  L.norm_off = off; off += align_up(norm_scratch_bytes(m.np), 256);
  L.ap_off = off; off += align_up(np2 * pe, 256);
  for (int i = 0; i < 9; ++i) { L.w_off[i] = off; off += align_up(np2 * pe, 256); }
  for (int i = 0; i < 4; ++i) { L.q_off[i] = off; off += align_up(np2 * se, 256); }
  L.i8_off = off;
  if (m.poly == Arith::I8X5) off += align_up(i8x5_scratch_bytes(m.np), 256);
  L.total = off;
  return L;
}

// Pinned host slots for the plan read-back: one block of PLAN_SLOTS pairs,
// allocated on first use and kept for the life of the process (a bounded,
// one-time allocation); a call holds one slot while it copies and waits. When
// every slot is held (more concurrent callers than slots) the copy goes
// through a stack buffer instead (pageable memory: the same result, a staged
// copy).
constexpr int PLAN_SLOTS = 64;
std::mutex plan_slot_mu;
sincosm_plan* plan_slots = nullptr;
bool plan_slot_busy[PLAN_SLOTS];

// SINCOSM_LOG set to a non-empty value other than "0": every plan read back
// to the host is printed to stderr, one line per call (read once).
static bool plan_log_on() {
  static const bool on = [] {
    const char* v = std::getenv("SINCOSM_LOG");
    return v && v[0] && !(v[0] == '0' && v[1] == 0);
  }();
  return on;
}

sincosm_status read_plan(const sincosm_plan* dev, sincosm_plan* host, hipStream_t stream, int count,
                         const char* who, int64_t n) {
  if (count < 1 || count > 2) return SINCOSM_E_ARG;
  int slot = -1;
  {
    std::lock_guard<std::mutex> g(plan_slot_mu);
    if (!plan_slots) SC_HIP(hipHostMalloc((void**)&plan_slots, PLAN_SLOTS * 2 * sizeof(sincosm_plan),
                                          hipHostMallocDefault));
    for (int i = 0; i < PLAN_SLOTS && slot < 0; ++i)
      if (!plan_slot_busy[i]) { plan_slot_busy[i] = true; slot = i; }
  }
  sincosm_plan local[2];
  sincosm_plan* buf = slot >= 0 ? plan_slots + 2 * slot : local;
  hipError_t e = hipMemcpyAsync(buf, dev, count * sizeof(sincosm_plan), hipMemcpyDeviceToHost, stream);
  if (e == hipSuccess) e = hipStreamSynchronize(stream);
  if (e == hipSuccess)
    for (int i = 0; i < count; ++i) host[i] = buf[i];
  if (slot >= 0) {
    std::lock_guard<std::mutex> g(plan_slot_mu);
    plan_slot_busy[slot] = false;
  }
  if (e == hipSuccess && plan_log_on())
    std::fprintf(stderr, "[sincosm] %s n=%lld: level %d s %d products %d norm1 %.6e status %d\n",
                 who ? who : "plan", (long long)n, host[0].level, host[0].s, host[0].products, host[0].norm1,
                 host[0].status);
  return e == hipSuccess ? SINCOSM_OK : SINCOSM_E_HIP;
}

bool overlaps(const void* a, int64_t lda, const void* b, int64_t ldb, int64_t n, size_t es) {
  const char* a0 = (const char*)a;
  const char* a1 = a0 + ((size_t)(n - 1) * lda + n) * es;
  const char* b0 = (const char*)b;
  const char* b1 = b0 + ((size_t)(n - 1) * ldb + n) * es;
  return a0 < b1 && b0 < a1;
}

// ----------------------------------------------------------------------------
// Scheme launch sequences.
// ----------------------------------------------------------------------------

Target internal(void* p, const Modes& m, bool f64) { return Target{p, m.np, (int)m.np, f64}; }

sincosm_status gemm(Run& r, Arith ar, const GemmLaunch& g0, int kind) {
  if (r.rec) {
    if (r.rec->count >= 8) return SINCOSM_E_ARG;
    r.rec->launches[r.rec->count++] = g0;
    return SINCOSM_OK;
  }
  GemmLaunch dg;
  const GemmLaunch* gp = &g0;
  if (r.cond.plan) {
    dg = g0;
    dg.cond = r.cond;
    gp = &dg;
  }
  const GemmLaunch& g = *gp;
  if (!r.timed) return launch_gemm(ar, r.m->tile, g, r.stream, r.i8ws);
  if (kind < 0) kind = g.nprob == 2 ? SINCOSM_TIMING_SQUARING : SINCOSM_TIMING_SCHEME;
  const TimingMark t = timing_begin(kind, r.stream);
  const sincosm_status st = launch_gemm(ar, r.m->tile, g, r.stream, r.i8ws);
  timing_end(t, r.stream);
  return st;
}

sincosm_status first_product(Run& r, double sx) {
  if (r.y_ready) return SINCOSM_OK;
  const Modes& m = *r.m;
  Problem p = make_problem((int)r.n);
  add_seg(p, r.Ap, r.Ap, m.np, sx, sx);
  add_out(p, internal(r.W[0], m, m.poly_f64), 1.0, 0.0, {});
  return gemm(r, m.poly, one(p, (int)m.np));
}

sincosm_status scheme3(Run& r, double sx) {
  const Modes& m = *r.m;
  const int64_t np = m.np;
  const int nv = (int)r.n;
  const bool pf = m.poly_f64;
  SC_TRY(first_product(r, sx));
  Problem p = make_problem(nv);
  add_seg(p, r.W[0], r.W[0], np);
  add_in(p, r.W[0], np);
  add_out(p, r.Cout, 1.0 / 24.0, 1.0, {-0.5});
  add_out(p, internal(r.W[1], m, pf), 1.0 / 120.0, 1.0, {-1.0 / 6.0});
  SC_TRY(gemm(r, m.poly, one(p, (int)np)));
  p = make_problem(nv);
  add_seg(p, r.Ap, r.W[1], np, sx, 1.0);
  add_out(p, r.Sout, 1.0, 0.0, {});
  return gemm(r, m.poly, one(p, (int)np));
}

sincosm_status scheme4(Run& r, double sx) {
  const Modes& m = *r.m;
  const int64_t np = m.np;
  const int nv = (int)r.n;
  const bool pf = m.poly_f64;
  SC_TRY(first_product(r, sx));
  Problem p = make_problem(nv);
  add_seg(p, r.W[0], r.W[0], np);
  add_in(p, r.W[0], np);
  add_out(p, internal(r.W[1], m, pf), 1.0, 0.0, {});
  add_out(p, internal(r.W[2], m, pf), 1.0 / 40320.0, 0.0, {-1.0 / 720.0});
  add_out(p, internal(r.W[3], m, pf), 1.0 / 24.0, 1.0, {-0.5});
  add_out(p, internal(r.W[4], m, pf), 1.0 / 120.0, 1.0, {-1.0 / 6.0});
  SC_TRY(gemm(r, m.poly, one(p, (int)np)));
  p = make_problem(nv);
  add_seg(p, r.W[1], r.W[2], np);
  add_in(p, r.W[3], np);
  add_in(p, r.W[4], np);
  add_out(p, r.Cout, 1.0, 0.0, {1.0, 0.0});
  add_out(p, internal(r.W[4], m, pf), 1.0 / 7.0, 0.0, {0.0, 1.0});
  SC_TRY(gemm(r, m.poly, one(p, (int)np)));
  p = make_problem(nv);
  add_seg(p, r.Ap, r.W[4], np, sx, 1.0);
  add_out(p, r.Sout, 1.0, 0.0, {});
  return gemm(r, m.poly, one(p, (int)np));
}

sincosm_status scheme5(Run& r, double sx) {
  const Modes& m = *r.m;
  const int64_t np = m.np;
  const int nv = (int)r.n;
  const bool pf = m.poly_f64;
  SC_TRY(first_product(r, sx));
  Problem p = make_problem(nv);
  add_seg(p, r.W[0], r.W[0], np);
  add_in(p, r.W[0], np);
  add_out(p, internal(r.W[1], m, pf), 1.0, 0.0, {});
  add_out(p, internal(r.W[2], m, pf), 1.0 / 40320.0, 0.0, {-1.0 / 720.0});
  add_out(p, internal(r.W[5], m, pf), 1.0 / 362880.0, 0.0, {-1.0 / 5040.0});
  add_out(p, internal(r.W[3], m, pf), 1.0 / 24.0, 1.0, {-0.5});
  add_out(p, internal(r.W[4], m, pf), 1.0 / 120.0, 1.0, {-1.0 / 6.0});
  SC_TRY(gemm(r, m.poly, one(p, (int)np)));
  p = make_problem(nv);
  add_seg(p, r.W[1], r.W[2], np);
  add_in(p, r.W[3], np);
  add_out(p, r.Cout, 1.0, 0.0, {1.0});
  SC_TRY(gemm(r, m.poly, one(p, (int)np)));
  p = make_problem(nv);
  add_seg(p, r.W[1], r.W[5], np);
  add_in(p, r.W[4], np);
  add_out(p, internal(r.W[4], m, pf), 1.0, 0.0, {1.0});
  SC_TRY(gemm(r, m.poly, one(p, (int)np)));
  p = make_problem(nv);
  add_seg(p, r.Ap, r.W[4], np, sx, 1.0);
  add_out(p, r.Sout, 1.0, 0.0, {});
  return gemm(r, m.poly, one(p, (int)np));
}

sincosm_status scheme6(Run& r, double sx) {
  const Modes& m = *r.m;
  const int64_t np = m.np;
  const int nv = (int)r.n;
  const bool pf = m.poly_f64;
  const Coeffs& k = coeffs();
  const double* x = k.x;   // x[1..8]
  const double* z = k.z6;  // z[0..8]
  SC_TRY(first_product(r, sx));
  // G2: Y2 = Y Y -> Y2, W = x1 Y + x2 Y2
  Problem p = make_problem(nv);
  add_seg(p, r.W[0], r.W[0], np);
  add_in(p, r.W[0], np);
  add_out(p, internal(r.W[1], m, pf), 1.0, 0.0, {});
  add_out(p, internal(r.W[2], m, pf), x[2], 0.0, {x[1]});
  SC_TRY(gemm(r, m.poly, one(p, (int)np)));
  // G3: Y4 = Y2 W; inputs Y (W0), Y2 (W1)
  p = make_problem(nv);
  add_seg(p, r.W[1], r.W[2], np);
  add_in(p, r.W[0], np);
  add_in(p, r.W[1], np);
  add_out(p, internal(r.W[3], m, pf), 1.0, 0.0, {});                 // Y4
  add_out(p, internal(r.W[4], m, pf), 1.0, 0.0, {0.0, x[3]});        // L
  add_out(p, internal(r.W[5], m, pf), x[7], x[4], {x[5], x[6]});     // R
  add_out(p, internal(r.W[6], m, pf), 0.0, 1.0, {-0.5, x[8]});       // Pc
  add_out(p, internal(r.W[7], m, pf), z[7], z[5], {z[5], z[6]});     // Q
  add_out(p, internal(r.W[8], m, pf), z[3], z[0], {z[1], z[2]});     // P
  SC_TRY(gemm(r, m.poly, one(p, (int)np)));
  // G4: T = L R; inputs Pc (W6), Q (W7), P (W8)
  p = make_problem(nv);
  add_seg(p, r.W[4], r.W[5], np);
  add_in(p, r.W[6], np);
  add_in(p, r.W[7], np);
  add_in(p, r.W[8], np);
  add_out(p, r.Cout, 1.0, 0.0, {1.0, 0.0, 0.0});                    // C = Pc + T
  add_out(p, internal(r.W[7], m, pf), z[8], 0.0, {z[8], 1.0, 0.0});  // Q + z8 C
  add_out(p, internal(r.W[8], m, pf), z[4], 0.0, {z[4], 0.0, 1.0});  // P + z4 C
  SC_TRY(gemm(r, m.poly, one(p, (int)np)));
  // G5: U = Q Y4 -> V = P + U
  p = make_problem(nv);
  add_seg(p, r.W[7], r.W[3], np);
  add_in(p, r.W[8], np);
  add_out(p, internal(r.W[8], m, pf), 1.0, 0.0, {1.0});
  SC_TRY(gemm(r, m.poly, one(p, (int)np)));
  // G6: S = (sA) V
  p = make_problem(nv);
  add_seg(p, r.Ap, r.W[8], np, sx, 1.0);
  add_out(p, r.Sout, 1.0, 0.0, {});
  return gemm(r, m.poly, one(p, (int)np));
}

sincosm_status scheme7(Run& r, double sx) {
  const Modes& m = *r.m;
  const int64_t np = m.np;
  const int nv = (int)r.n;
  const bool pf = m.poly_f64;
  const Coeffs& k = coeffs();
  const double(*a)[5] = k.a;  // a[i][j], i = 0..3, j = 1..4
  const double* z = k.z7;     // z[0..11]
  SC_TRY(first_product(r, sx));
  // G2: Y2 = Y Y
  Problem p = make_problem(nv);
  add_seg(p, r.W[0], r.W[0], np);
  add_out(p, internal(r.W[1], m, pf), 1.0, 0.0, {});
  SC_TRY(gemm(r, m.poly, one(p, (int)np)));
  // G3: Y3 = Y2 Y; inputs Y (W0), Y2 (W1)
  p = make_problem(nv);
  add_seg(p, r.W[1], r.W[0], np);
  add_in(p, r.W[0], np);
  add_in(p, r.W[1], np);
  for (int j = 1; j <= 4; ++j)
    add_out(p, internal(r.W[1 + j], m, pf), a[3][j], a[0][j], {a[1][j], a[2][j]});  // C_j -> W2..W5
  add_out(p, internal(r.W[6], m, pf), z[3], z[0], {z[1], z[2]});                  // P
  add_out(p, internal(r.W[7], m, pf), z[9], z[6], {z[7], z[8]});                  // Q
  SC_TRY(gemm(r, m.poly, one(p, (int)np)));
  // G4: K = C4 C4; inputs C3 (W4), C2 (W3) -> Y6 = C3 + K (W4), L = C2 + Y6 (W3)
  p = make_problem(nv);
  add_seg(p, r.W[5], r.W[5], np);
  add_in(p, r.W[4], np);
  add_in(p, r.W[3], np);
  add_out(p, internal(r.W[4], m, pf), 1.0, 0.0, {1.0, 0.0});
  add_out(p, internal(r.W[3], m, pf), 1.0, 0.0, {1.0, 1.0});
  SC_TRY(gemm(r, m.poly, one(p, (int)np)));
  // G5: T = L Y6; inputs C1 (W2), Y6 (W4), Q (W7), P (W6)
  p = make_problem(nv);
  add_seg(p, r.W[3], r.W[4], np);
  add_in(p, r.W[2], np);
  add_in(p, r.W[4], np);
  add_in(p, r.W[7], np);
  add_in(p, r.W[6], np);
  add_out(p, internal(r.W[8], m, pf), 1.0, 0.0, {1.0, 0.0, 0.0, 0.0});      // C (operand of G6)
  add_out(p, r.Cout, 1.0, 0.0, {1.0, 0.0, 0.0, 0.0});                       // C (result)
  add_out(p, internal(r.W[7], m, pf), z[11], 0.0, {z[11], z[10], 1.0, 0.0}); // Q + z10 Y6 + z11 C
  add_out(p, internal(r.W[6], m, pf), z[5], 0.0, {z[5], z[4], 0.0, 1.0});    // P + z4 Y6 + z5 C
  SC_TRY(gemm(r, m.poly, one(p, (int)np)));
  // G6: U = Q C -> V = P + U (W6)
  p = make_problem(nv);
  add_seg(p, r.W[7], r.W[8], np);
  add_in(p, r.W[6], np);
  add_out(p, internal(r.W[6], m, pf), 1.0, 0.0, {1.0});
  SC_TRY(gemm(r, m.poly, one(p, (int)np)));
  // G7: S = (sA) V
  p = make_problem(nv);
  add_seg(p, r.Ap, r.W[6], np, sx, 1.0);
  add_out(p, r.Sout, 1.0, 0.0, {});
  return gemm(r, m.poly, one(p, (int)np));
}

sincosm_status run_scheme(Run& r, int level, double sx) {
  switch (level) {
    case 3: return scheme3(r, sx);
    case 4: return scheme4(r, sx);
    case 5: return scheme5(r, sx);
    case 6: return scheme6(r, sx);
    default: return scheme7(r, sx);
  }
}

// One double-angle step: from (Sc, Cc) write C' = I - 2 Sc Sc, S' = 2 Sc Cc.
sincosm_status double_angle(Run& r, const void* Sc, const void* Cc, const Target& Cn, const Target& Sn) {
  const Modes& m = *r.m;
  GemmLaunch g;
  memset(&g, 0, sizeof(g));
  g.np = (int)m.np;
  g.nprob = 2;
  Problem p0 = make_problem((int)r.n);
  add_seg(p0, Sc, Sc, m.np);
  add_out(p0, Cn, -2.0, 1.0, {});
  Problem p1 = make_problem((int)r.n);
  add_seg(p1, Sc, Cc, m.np);
  add_out(p1, Sn, 2.0, 0.0, {});
  g.prob[0] = p0;
  g.prob[1] = p1;
  return gemm(r, m.sq, g);
}

}  // namespace sc
