/*
 * sincosm.h - C ABI of the MI355X (gfx950) library for the simultaneous
 * matrix cosine and sine of a real dense matrix.
 *
 * Method: Seydaoglu, Bader, Blanes, Casas, "Computing the matrix sine and
 * cosine simultaneously with a reduced number of products" (arXiv
 * 2010.00465). For a real n x n matrix A the library returns C = cos(A) and
 * S = sin(A) (Section 2.1, definitions of T^c_{2m} and T^s_{2m+1}) by
 *   1. theta = ||A||_1 (maximum absolute column sum), in float64 on device;
 *   2. choosing a scheme with 3, 4, 6 or 7 products and a scaling power s
 *      from the bounds of Tables 1 (double) / 2 (single): the plan minimises
 *      the product count Pi + 2 s, with s the smallest integer >= 0 such that
 *      theta 2^-s does not exceed the scheme's bound, ties to the smaller s;
 *   3. evaluating the factorized Taylor scheme of Section 2.1 on X = 2^-s A;
 *   4. s double-angle steps cos 2X = I - 2 sin^2 X, sin 2X = 2 sin X cos X
 *      (Section 1), two products each.
 *
 * Conventions for every call below:
 *  - Matrices are row-major with a leading dimension (elements between the
 *    starts of consecutive rows) >= n. The 1-norm is the maximum absolute
 *    COLUMN sum of the logical matrix.
 *  - Pointers named A, C, S, Gc, Gs, gA, ws and *_dev are DEVICE pointers on
 *    the current HIP device; pointers named *_host are host pointers.
 *  - `stream` is a hipStream_t passed as void*; NULL means the default
 *    stream. Work is enqueued on it. sincosm_eval and sincosm_backward read
 *    the 24-byte plan back to the host (one stream synchronisation) before
 *    they enqueue the products, so they return after the plan is known (so
 *    do sincosm_wave_eval, sincosm_wave_block_eval and sincosm_expi_eval);
 *    the *_async variants decide the plan on the device and never wait.
 *  - The caller owns every buffer. The library allocates no device memory:
 *    each call takes a workspace whose size the matching *_workspace_size
 *    query returns. Results are deterministic (bitwise) for identical inputs,
 *    settings and device.
 *  - Errors in arguments are returned synchronously and leave outputs
 *    untouched. n = 0 is a no-op returning SINCOSM_OK.
 *  - Environment: SINCOSM_LOG set to a value other than "" or "0" prints
 *    one line to stderr for every plan read back to the host (the calls that
 *    wait for their plan: entry name, n, level, s, products, norm1, status);
 *    it is read once, at the first such call.
 */
#ifndef SINCOSM_H
#define SINCOSM_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef enum {
  SINCOSM_OK = 0,
  SINCOSM_E_ARG = -1,         /* bad size, leading dimension, null or aliased pointer, bad enum */
  SINCOSM_E_UNSUPPORTED = -2, /* combination not provided (see each call) */
  SINCOSM_E_WORKSPACE = -3,   /* workspace missing or smaller than the query's size */
  SINCOSM_E_NONFINITE = -4,   /* A holds Inf/NaN (or its 1-norm overflows): outputs set to NaN */
  SINCOSM_E_HIP = -5,         /* a HIP runtime call failed */
  SINCOSM_E_PLAN = -6,        /* a caller's plan does not cover ||A||_1: outputs set to NaN */
  SINCOSM_E_TOO_LARGE = -7,   /* the matrix needs more workspace than the library's static scratch */
  SINCOSM_E_SCALING = -8      /* the plan needs more double-angle steps than the call allowed: NaN outputs */
} sincosm_status;

/* Storage type of A, C, S and of the gradients. */
typedef enum { SINCOSM_F64 = 0, SINCOSM_F32 = 1 } sincosm_dtype;

/* Accuracy target of the plan: Table 1 bounds (u = 2^-53) or Table 2 (u = 2^-24). */
typedef enum { SINCOSM_ACC_DOUBLE = 0, SINCOSM_ACC_SINGLE = 1 } sincosm_accuracy;

/* Flag OR-ed into `acc` of sincosm_plan_host, sincosm_plan_device, sincosm_eval and
 * sincosm_expi_eval: the plan also considers the 5-product scheme of Section 2.1
 * (the 4-product cosine T^c_8 of Algorithm4cA with the order-nine sine T^s_9 of
 * Algorithm5sA; combined bound = the printed T^c_8 bound, 1.1495e-1 double /
 * 8.5756e-1 single, since its sine bound is larger). It is chosen only where it
 * saves a product: ||A||_1 in (8.0438e-2, 1.1495e-1] double, (7.492e-1, 8.5756e-1]
 * single. Without the flag the plan uses exactly the schemes of Tables 1-2. The
 * batched, backward and wave entries reject the flag (SINCOSM_E_ARG). */
enum { SINCOSM_PLAN_EXTENDED = 16 };

/* Flag OR-ed into `acc` of sincosm_eval only: plan on theta' = min(||A||_1,
 * ||A^2||_1^(1/2)) instead of ||A||_1 (not in the paper; the remedy for the
 * overscaling Section 4 observes on [[1, lambda], [0, -1]], whose square is I).
 * A^2 is the first product every scheme forms anyway: it is computed unscaled
 * before the plan, its 1-norm taken on the device, and after the plan it is
 * scaled by 4^-s (exact) and reused, so the product count stays Pi + 2 s. Cost:
 * one more O(n^2) norm pass and scaling pass. The cosine's truncation bound
 * holds as for Tables 1-2 (the scheme is a polynomial in A^2); the sine's
 * becomes u ||X|| / theta_level relative to X = 2^-s A. plan_host->norm1
 * reports theta'. If A^2 overflows, theta' = ||A||_1 and A^2 is recomputed from
 * the scaled operands (one extra product). Rejected elsewhere (SINCOSM_E_ARG). */
enum { SINCOSM_PLAN_REFINED = 32 };

/* Arithmetic of the polynomial-phase products (the scheme of step 3):
 *  NATIVE - the storage type (float64 MFMA for F64, float32 MFMA for F32);
 *  F32    - float32 MFMA products and float32 intermediates;
 *  BF16X3 - each float32 operand split as hi + lo (hi = bf16(x), lo = bf16(x - hi)),
 *           products hi*hi + hi*lo + lo*hi on bf16 MFMA with float32 accumulation.
 *  I8X5   - float64 storage and float64 intermediates and epilogues; each product
 *           on the int8 matrix cores by error-free splitting (Ozaki's scheme): the
 *           left operand's rows and the right operand's columns are scaled by
 *           powers of two and written as five 7-bit digits, the 15 digit products
 *           of weight 2^-14 ... 2^-42 accumulate exactly in int32 and are combined
 *           in float64. Elementwise product error at most
 *           2^-34 (rowmax|X| colsum|Y| + rowsum|X| colmax|Y|) for the digits cut
 *           off, plus 2^-31 n rowmax|X| colmax|Y| for the digit products left out
 *           (reached only when digits agree in sign throughout; for uncorrelated
 *           digits those sums grow like n^(1/2) and the first term dominates):
 *           inside the single-accuracy bound u = 2^-24 of Table 2, not the
 *           double one. dtype F64 only, n <= 16384 (for the wave block entries
 *           the order of A: their products are n x n). Accepted by every
 *           single-matrix entry point, device-planned ones included (each int8
 *           kernel honours the launch's plan record), and by sincosm_matmul,
 *           where a row of X or a column of Y holding Inf or NaN gives a NaN row
 *           or column of Z; the batched and reverse passes return
 *           SINCOSM_E_UNSUPPORTED.
 * The 1-norm, the plan and the double-angle steps always run in the storage
 * type (float64 for F64). */
typedef enum { SINCOSM_PROD_NATIVE = 0, SINCOSM_PROD_F32 = 1, SINCOSM_PROD_BF16X3 = 2,
               SINCOSM_PROD_I8X5 = 3 } sincosm_prod;

/* The plan chosen for one matrix. level in {3,4,6,7} (= products of the
 * scheme; also 5 with SINCOSM_PLAN_EXTENDED; 2..5 for the wave entries),
 * s = number of double-angle steps, products = level + 2 s, status =
 * SINCOSM_OK or SINCOSM_E_NONFINITE, norm1 = ||A||_1 as computed on device. */
typedef struct {
  int32_t level;
  int32_t s;
  int32_t products;
  int32_t status;
  double norm1;
} sincosm_plan;

/* Plan for a given 1-norm, computed on the host with the same rule and
 * constants as the device (Tables 1-2; the 7-product sine bound in double is
 * 1.8548, re-derived from the printed coefficients). Pure function.
 * Returns SINCOSM_E_ARG for a bad `acc` or a null `out`; a NaN/Inf/negative
 * norm gives status SINCOSM_E_NONFINITE in *out and return SINCOSM_OK. */
sincosm_status sincosm_plan_host(double norm1, int acc, sincosm_plan* out);

/* Human-readable text for a status code (static storage). */
const char* sincosm_strerror(int status);

/* The plan sincosm_eval would use for A (1-norm and rule on the device),
 * read back to *plan_host. ws: sincosm_plan_workspace_size(n) bytes, 256-byte
 * aligned. acc may carry SINCOSM_PLAN_EXTENDED (not SINCOSM_PLAN_REFINED, which
 * needs a product). Returns SINCOSM_OK also for non-finite input (status in
 * the plan). */
size_t sincosm_plan_workspace_size(int64_t n);
sincosm_status sincosm_plan_device(int64_t n, int dtype, const void* A, int64_t lda, int acc,
                                   void* ws, size_t ws_bytes, sincosm_plan* plan_host, void* stream);

/* Bytes of workspace sincosm_eval needs for this n and settings (0 for n <= 0);
 * the same size serves sincosm_wave_eval, sincosm_wave_block_eval and
 * sincosm_expi_eval. `acc` does not change it. */
size_t sincosm_workspace_size(int64_t n, int dtype, int acc, int prod);

/* cos(A) and sin(A) of one n x n matrix (Sections 1 and 2.1, Tables 1-2).
 *  A (lda), C (ldc), S (lds): device matrices of type `dtype`; A is read only;
 *  C and S must not overlap each other or A.
 *  ws / ws_bytes: device workspace of at least sincosm_workspace_size(...) bytes,
 *  256-byte aligned.
 *  plan_host: optional host pointer receiving the plan used.
 *  Supported: dtype F64 with prod NATIVE, F32, BF16X3 or I8X5 (n <= 16384);
 *  dtype F32 with prod NATIVE (= F32) or BF16X3. acc may be DOUBLE or SINGLE in every case, with
 *  SINCOSM_PLAN_EXTENDED and/or SINCOSM_PLAN_REFINED OR-ed in.
 *  Returns SINCOSM_E_NONFINITE (after filling C and S with NaN) when A holds
 *  Inf or NaN. */
sincosm_status sincosm_eval(int64_t n, int dtype, const void* A, int64_t lda,
                            void* C, int64_t ldc, void* S, int64_t lds,
                            int acc, int prod, void* ws, size_t ws_bytes,
                            sincosm_plan* plan_host, void* stream);

/* sincosm_eval with the plan given by the caller (host pointer plan_in: level
 * and s, e.g. sincosm_plan_host of a known bound on ||A||_1, or the plan of an
 * earlier call). Nothing is read back, so the call only enqueues kernels on
 * `stream` (no synchronisation, no allocation) and can be captured in a HIP
 * graph; the launches are those sincosm_eval makes for the same plan, so the
 * results are bitwise the same. The 1-norm is still computed on the device and
 * the plan checked against it: it covers A when ||A||_1 2^-s <= theta of its
 * level (Tables 1-2 of the accuracy `acc`). When it does not, or A holds Inf or
 * NaN, C and S are filled with NaN after the products.
 *  plan_in (host, read): level in {3, 4, 6, 7} (5 with SINCOSM_PLAN_EXTENDED
 *  in acc), 0 <= s <= 1100; other fields are ignored.
 *  plan_dev (device, nullable): receives {level, s, products, status, norm1}
 *  of this call once the stream reaches it; status SINCOSM_OK,
 *  SINCOSM_E_PLAN or SINCOSM_E_NONFINITE.
 *  acc: SINCOSM_ACC_DOUBLE or SINGLE, optionally | SINCOSM_PLAN_EXTENDED (the
 *  refined-norm flag is not accepted). Other arguments as sincosm_eval.
 *  Returns SINCOSM_E_ARG for a bad plan_in, otherwise the argument and
 *  workspace errors of sincosm_eval; the status of the check is on the device. */
sincosm_status sincosm_eval_planned(int64_t n, int dtype, const void* A, int64_t lda,
                                    void* C, int64_t ldc, void* S, int64_t lds,
                                    int acc, int prod, const sincosm_plan* plan_in,
                                    void* ws, size_t ws_bytes, sincosm_plan* plan_dev,
                                    void* stream);

/* sincosm_eval with the plan decided on the device: the call only enqueues
 * kernels on `stream` (no read-back, no synchronisation, no allocation), so it
 * can be captured in a HIP graph without knowing the plan (Tables 1-2 applied
 * to ||A||_1 on the device). It enqueues a fixed sequence: the 1-norm and the
 * plan (2 launches), the schemes' shared first product, the other products of
 * the four schemes packed into 6 launches (7 with SINCOSM_PLAN_EXTENDED) whose
 * workgroups compute the product of the plan's level, s_max double-angle
 * steps whose workgroups return at once beyond the plan's s, and a copy of
 * the result into C and S. The products computed are those sincosm_eval
 * computes for the same plan, with the 2^-s scales resolved on the device, so
 * the results are bitwise those of sincosm_eval.
 *  s_max: 0 <= s_max <= 1100, the largest number of double-angle steps the
 *  call may need; a plan with s > s_max gives status SINCOSM_E_SCALING and C
 *  and S filled with NaN (double table: s_max = k covers ||A||_1 <=
 *  1.8548 * 2^k). Each unused step costs one launch that does no work.
 *  plan_dev (device, nullable): receives the plan record {level, s, products,
 *  status, norm1} once the stream reaches it; status SINCOSM_OK,
 *  SINCOSM_E_NONFINITE (C, S = NaN) or SINCOSM_E_SCALING (C, S = NaN).
 *  acc: DOUBLE or SINGLE, optionally | SINCOSM_PLAN_EXTENDED (the refined-norm
 *  flag is not accepted). Other arguments, the workspace and the synchronous
 *  argument errors as sincosm_eval. */
sincosm_status sincosm_eval_async(int64_t n, int dtype, const void* A, int64_t lda,
                                  void* C, int64_t ldc, void* S, int64_t lds,
                                  int acc, int prod, int32_t s_max, void* ws, size_t ws_bytes,
                                  sincosm_plan* plan_dev, void* stream);

/* Size in bytes of the static device scratch array behind
 * sincosm_eval_planned_noalloc (one per GPU the library runs on, held until
 * the process ends). */
#define SINCOSM_NOALLOC_SCRATCH_BYTES (32u << 20)

/* sincosm_eval_planned without a workspace argument, for callers that cannot
 * allocate device memory (code under HIP graph capture, tight serving loops,
 * harnesses that forbid hipMalloc). The workspace is a static device array of
 * SINCOSM_NOALLOC_SCRATCH_BYTES bytes that the library holds per GPU; the call
 * makes no hipMalloc, hipFree or other allocating call, no synchronisation and
 * records no timing events. Arguments, launches, results (bitwise) and errors
 * are those of sincosm_eval_planned; in addition it returns SINCOSM_E_TOO_LARGE
 * (nothing enqueued) when sincosm_workspace_size(n, dtype, acc, prod) exceeds
 * the scratch size (float64 storage with native products up to n = 512,
 * float32 storage up to n = 768).
 * Every call on a GPU shares that GPU's array, which keeps the last call's
 * contents: calls that overlap in time on one GPU (other streams, other host
 * threads) race and give undefined results; calls ordered on one stream are
 * safe. */
sincosm_status sincosm_eval_planned_noalloc(int64_t n, int dtype, const void* A, int64_t lda,
                                            void* C, int64_t ldc, void* S, int64_t lds,
                                            int acc, int prod, const sincosm_plan* plan_in,
                                            sincosm_plan* plan_dev, void* stream);

/* Plan of the wave-equation schemes for a given ||B||_1, B = t^2 A (host, pure).
 * level in {2,3,4,5} (= products of the Section 2.2 scheme), s = number of
 * double-angle steps (t halved s times, so B is quartered s times), products =
 * level + 2 s, norm1 = ||B||_1. The bounds on ||B||_1 per scheme (the paper
 * prints none for these schemes) are derived from the scheme polynomials as
 * for Tables 1-2: double {3.4458e-3, 1.3213e-2, 9.6251e-1, 3.6404}, single
 * {5.2237e-1, 7.354e-1, 8.9612, 21.848}. Same rule as sincosm_plan_host
 * otherwise (least Pi + 2 s, ties to the smaller s; non-finite norm gives
 * status SINCOSM_E_NONFINITE). Returns SINCOSM_E_ARG for a bad `acc`/null `out`. */
sincosm_status sincosm_wave_plan_host(double normB, int acc, sincosm_plan* out);

/* Wave-equation pair (Sections 1 and 2.2): for y'' + A y = 0,
 *   C = c(t^2 A) = cos(t sqrt A) = sum_k (-1)^k (t^2 A)^k / (2k)!,
 *   S = s(t, A)  = sin(t sqrt A) / sqrt A = t sum_k (-1)^k (t^2 A)^k / (2k+1)!,
 * both entire in A, so no square root of A is formed and A may be any real
 * matrix. The factorized schemes use B = t^2 A in place of A^2 and the
 * scalar t in place of the sine's final factor A (2, 3, 4 or 5 products);
 * the double-angle step is c(4 t^2 A) = 2 c(t^2 A)^2 - I, s(2t, A) =
 * 2 s(t, A) c(t^2 A). The pair solves y(t) = C y(0) + S y'(0).
 *  t: finite scalar (t = 0 gives C = I, S = 0; negative t negates S).
 *  Buffers, dtype/prod combinations, workspace (sincosm_workspace_size(n,
 *  dtype, acc, prod) bytes, 256-byte aligned), aliasing rules, plan_host and
 *  errors as for sincosm_eval; *plan_host receives the wave plan (norm1 =
 *  ||t^2 A||_1). Non-finite t is SINCOSM_E_ARG; t^2 A with Inf/NaN (including
 *  overflow of t^2) gives SINCOSM_E_NONFINITE with C and S filled with NaN. */
sincosm_status sincosm_wave_eval(int64_t n, int dtype, const void* A, int64_t lda, double t,
                                 void* C, int64_t ldc, void* S, int64_t lds,
                                 int acc, int prod, void* ws, size_t ws_bytes,
                                 sincosm_plan* plan_host, void* stream);

/* Block propagator of the wave system (eq:symplectic, Section 1): y'' + A y = 0
 * written as (y, y')' = M (y, y'), M = [[0, I], [-A, 0]], has
 *   E = e^{tM} = [[c(t^2 A), s(t, A)], [-A s(t, A), c(t^2 A)]].
 * Computed as sincosm_wave_eval does, plus one product A s(t, A) whose
 * epilogue writes all four n x n blocks of E (2n x 2n, row-major, leading
 * dimension lde >= 2n, type `dtype`). E must not overlap A. Plan, workspace
 * (sincosm_workspace_size(n, dtype, acc, prod)), dtype/prod combinations and
 * errors as for sincosm_wave_eval; the wave plan's product count does not
 * include the extra product. Non-finite input: E filled with NaN,
 * SINCOSM_E_NONFINITE. */
sincosm_status sincosm_wave_block_eval(int64_t n, int dtype, const void* A, int64_t lda, double t,
                                       void* E, int64_t lde, int acc, int prod, void* ws,
                                       size_t ws_bytes, sincosm_plan* plan_host, void* stream);

/* sincosm_wave_eval and sincosm_wave_block_eval with the plan decided on the
 * device (the wave plan of ||t^2 A||_1): the calls only enqueue kernels on
 * `stream` (no read-back, no synchronisation, no allocation; graph-capturable).
 * Fixed sequence: the 1-norm and plan (2 launches), B_s = 4^-s t^2 A formed in
 * place (1 launch), the products of the four wave schemes packed into 5 slot
 * launches whose workgroups compute the product of the plan's level, s_max
 * double-angle steps that return at once beyond the plan's s, then the copy
 * into C and S (block form: one launch that moves the pair to fixed buffers,
 * one padded copy of A, the product A s(t, A) writing E, and a NaN fill that
 * acts only on a failed plan). The sine is carried as s / t_s through the
 * steps (t_s = 2^-s t; the step becomes S' = S C) and multiplied by t at the
 * end, so C is bitwise that of the synchronous call and S agrees with it to
 * rounding (not bitwise).
 *  s_max: 0 <= s_max <= 1100; a plan with s > s_max gives status
 *  SINCOSM_E_SCALING in the plan record and NaN outputs (double table: s_max =
 *  k covers ||t^2 A||_1 <= 3.6404 * 4^k).
 *  plan_dev (device, nullable): receives the plan record; status SINCOSM_OK,
 *  SINCOSM_E_NONFINITE or SINCOSM_E_SCALING (outputs NaN for the last two).
 *  Other arguments, workspace and synchronous argument errors as the
 *  synchronous calls. */
sincosm_status sincosm_wave_eval_async(int64_t n, int dtype, const void* A, int64_t lda, double t,
                                       void* C, int64_t ldc, void* S, int64_t lds,
                                       int acc, int prod, int32_t s_max, void* ws, size_t ws_bytes,
                                       sincosm_plan* plan_dev, void* stream);
sincosm_status sincosm_wave_block_eval_async(int64_t n, int dtype, const void* A, int64_t lda,
                                             double t, void* E, int64_t lde, int acc, int prod,
                                             int32_t s_max, void* ws, size_t ws_bytes,
                                             sincosm_plan* plan_dev, void* stream);

/* Unitary propagator of i u' = A u for real A (eq:unitary, Section 1):
 *   U = e^{-itA} = cos(tA) - i sin(tA),
 * from the cos/sin method on X = tA (the copy of A is multiplied by t in
 * float64 as it is read; the plan is that of sincosm_eval for ||tA||_1), so
 * every product is real and each double-angle step costs two real products.
 *  U: n x n complex, interleaved (real, imaginary) pairs of `dtype` (complex128
 *     for F64, complex64 for F32), leading dimension ldu >= n in complex
 *     elements, aligned to one complex element; must not overlap A.
 *  t: finite scalar; non-finite t is SINCOSM_E_ARG.
 * Workspace sincosm_workspace_size(n, dtype, acc, prod); dtype/prod, plan_host
 * and errors as for sincosm_eval (non-finite tA: U filled with NaN,
 * SINCOSM_E_NONFINITE). */
sincosm_status sincosm_expi_eval(int64_t n, int dtype, const void* A, int64_t lda, double t,
                                 void* U, int64_t ldu, int acc, int prod, void* ws, size_t ws_bytes,
                                 sincosm_plan* plan_host, void* stream);

/* sincosm_expi_eval with the plan decided on the device (that of
 * sincosm_eval_async for ||tA||_1): the same fixed launch sequence as
 * sincosm_eval_async on the padded copy of tA, ending in one pass that writes
 * U = C - i S (or NaN) from the ping-pong pair the plan's s selects. The
 * result is bitwise that of sincosm_expi_eval. s_max, plan_dev and its
 * statuses as sincosm_eval_async (s_max = k covers ||tA||_1 <= 1.8548 * 2^k
 * for the double table); other arguments and errors as sincosm_expi_eval. */
sincosm_status sincosm_expi_eval_async(int64_t n, int dtype, const void* A, int64_t lda, double t,
                                       void* U, int64_t ldu, int acc, int prod, int32_t s_max,
                                       void* ws, size_t ws_bytes, sincosm_plan* plan_dev, void* stream);

/* Batched evaluation of many independent matrices of uneven orders
 * (1 <= n <= 256), each with its own plan (as sincosm_eval would choose it:
 * Tables 1-2 on its own 1-norm), packed row-major with leading dimension n.
 *
 * sincosm_batched_workspace_size - bytes of workspace for `batch` matrices
 *   whose orders are at most max(n_host[i]) (n_host: host array of the
 *   orders, read during the call; NULL sizes for any order up to 256). It
 *   grows with the batch only by 4 bytes per matrix (the work queue): each
 *   resident workgroup owns one slot of 10 padded matrices. Returns 0 for
 *   batch <= 0, an order outside 1..256, a bad dtype or prod other than NATIVE.
 * sincosm_eval_batched - cos and sin of every matrix. n_dev[i] (int32) and
 *   offset_dev[i] (int64, in elements; the same offsets for A, C and S) are
 *   DEVICE arrays of `batch` entries; A, C and S hold at least total_elems
 *   elements each. Everything is checked on the device: an entry whose order
 *   lies outside 1..256, or whose n x n elements do not lie inside
 *   [0, total_elems), is skipped with status SINCOSM_E_ARG in its plan record;
 *   an order beyond the largest one the workspace's slots hold is skipped with
 *   SINCOSM_E_WORKSPACE; a matrix with Inf/NaN gets NaN outputs and status
 *   SINCOSM_E_NONFINITE. The call enqueues a fixed sequence of two launches
 *   (entry checks and the largest-first work queue in one workgroup, then the
 *   persistent kernel; one or two more when the tuning table routes small
 *   padded orders to the LDS-resident kernels, which run before the persistent
 *   one), reads nothing back and returns SINCOSM_OK for any
 *   entry values, so it can be captured in a HIP graph and replayed with new
 *   values in A, n_dev and offset_dev.
 *   ws / ws_bytes: 256-byte aligned; the size query's value for the batch
 *   (a smaller workspace holds smaller orders only; none at all:
 *   SINCOSM_E_WORKSPACE). dtype F64 or F32 with prod NATIVE (other products:
 *   SINCOSM_E_UNSUPPORTED). plans_dev: optional device array of `batch`
 *   sincosm_plan. Calls that overlap on one workspace race. */
size_t sincosm_batched_workspace_size(int64_t batch, const int32_t* n_host, int dtype,
                                      int acc, int prod);
sincosm_status sincosm_eval_batched(int64_t batch, int dtype, const int32_t* n_dev,
                                    const int64_t* offset_dev, int64_t total_elems,
                                    const void* A, void* C, void* S, int acc, int prod,
                                    void* ws, size_t ws_bytes, sincosm_plan* plans_dev,
                                    void* stream);

/* Bytes of workspace sincosm_backward needs for order n and `s` double-angle
 * steps (s from the forward call's plan; the backward rejects a larger s), and
 * that sincosm_backward_async needs for s_max = s. */
size_t sincosm_backward_workspace_size(int64_t n, int dtype, int acc, int32_t s);

/* Gradient of L(A) = <Gc, cos A> + <Gs, sin A> (Frobenius inner products)
 * with respect to A, for the function the forward computes (same plan):
 *  gA = adjoint of the map A -> (C, S) applied to (Gc, Gs).
 *  Gc (ldgc), Gs (ldgs): device matrices; either may be NULL (= zero).
 *  gA (ldga): device output, must not overlap the inputs.
 *  dtype F64 only (prod NATIVE). The reverse pass runs through the s
 *  double-angle steps (their inputs recomputed and kept in the workspace)
 *  and through the scheme's products, two products per forward product.
 *  Returns SINCOSM_E_NONFINITE (gA filled with NaN) for Inf/NaN input. */
sincosm_status sincosm_backward(int64_t n, int dtype, const void* A, int64_t lda,
                                const void* Gc, int64_t ldgc, const void* Gs, int64_t ldgs,
                                void* gA, int64_t ldga, int acc, void* ws, size_t ws_bytes,
                                sincosm_plan* plan_host, void* stream);

/* sincosm_backward with the plan decided on the device: the call only enqueues
 * kernels on `stream` (no read-back, no synchronisation), so it can be captured
 * in a HIP graph without knowing the plan. The forward recomputation and the
 * reverse pass run as a fixed launch sequence whose launches read the plan
 * record and return at once where they do not apply (another level; a
 * double-angle step beyond the plan's s), as in sincosm_eval_async; the
 * products computed are those of sincosm_backward, so gA is bitwise the same.
 *  s_max: 0 <= s_max <= 1100, the largest number of double-angle steps the
 *  call allows; the workspace must hold
 *  sincosm_backward_workspace_size(n, dtype, acc, s_max) bytes. A plan with
 *  s > s_max gives status SINCOSM_E_SCALING and gA filled with NaN.
 *  plan_dev (device, nullable): receives the plan record once the stream
 *  reaches it (status SINCOSM_OK, SINCOSM_E_NONFINITE or SINCOSM_E_SCALING;
 *  gA is NaN for the latter two). Other arguments and the synchronous argument
 *  errors as sincosm_backward. */
sincosm_status sincosm_backward_async(int64_t n, int dtype, const void* A, int64_t lda,
                                      const void* Gc, int64_t ldgc, const void* Gs, int64_t ldgs,
                                      void* gA, int64_t ldga, int acc, int32_t s_max, void* ws,
                                      size_t ws_bytes, sincosm_plan* plan_dev, void* stream);

/* Building block exposed for tests and measurement: Z = X Y for n x n
 * matrices with the same kernels and padding sincosm_eval uses
 * (dtype F64 / F32, prod as in sincosm_eval). ws: sincosm_matmul_workspace_size bytes. */
size_t sincosm_matmul_workspace_size(int64_t n, int dtype, int prod);
sincosm_status sincosm_matmul(int64_t n, int dtype, const void* X, int64_t ldx,
                              const void* Y, int64_t ldy, void* Z, int64_t ldz, int prod,
                              void* ws, size_t ws_bytes, void* stream);

/* Instrumentation: when enabled, every product launch of the library is
 * bracketed by two HIP events on its stream, tagged by class:
 *   SINCOSM_TIMING_SCHEME   - a product of the scheme (one problem per launch),
 *   SINCOSM_TIMING_SQUARING - a double-angle step (one launch, 2 products),
 *   SINCOSM_TIMING_BACKWARD - a product of the reverse pass,
 *   SINCOSM_TIMING_BATCHED  - a launch of the batched path.
 * sincosm_timing_enable(1) starts recording (discarding earlier records),
 * (0) stops. sincosm_timing_read waits for the recorded events of one class
 * and returns their summed duration in ms and their number. Host-side state,
 * thread-safe, intended for measurement runs. */
enum { SINCOSM_TIMING_SCHEME = 0, SINCOSM_TIMING_SQUARING = 1, SINCOSM_TIMING_BACKWARD = 2,
       SINCOSM_TIMING_BATCHED = 3 };
sincosm_status sincosm_timing_enable(int on);
sincosm_status sincosm_timing_read(int kind, double* total_ms, int64_t* count);

/* Autotuning of the product kernel. `arith` is 0 for float64 products, 1 for
 * float32 products. Each arithmetic offers a list of kernel configurations
 * (tile rows, tile columns, k depth, wave rows, wave columns, waves per SIMD,
 * 1 if operand tiles are loaded straight into LDS, number of k groups that
 * split the k steps of a tile -> info[0..7]; info must hold 8 entries);
 * entries 0, 1 and 2 are the defaults for padding
 * granularities 128, 64 and 32. sincosm_tune_set makes launches of that
 * arithmetic whose padded order lies in [np_lo, np_hi] use configuration idx
 * (later entries win; idx = -1 removes the overlapping entries); a
 * configuration whose tile does not divide the padded order is ignored for it.
 * With SINCOSM_TUNE_MULTI OR-ed into `arith`, sincosm_tune_set addresses the
 * table used by launches of several problems with equal k-work (the
 * double-angle steps); with SINCOSM_TUNE_UNEVEN, the table of the remaining
 * launches: problems of unequal k-work or one problem with several k-segments
 * (the reverse pass). Such launches use the plain table where their own has
 * no entry. With SINCOSM_TUNE_BATCHED, the entries choose how
 * sincosm_eval_batched runs a matrix's products by padded order: configuration
 * 0 is 64 x 64 output tiles (the default), 1 is 32 x 32 (both with the
 * per-matrix workspace in the caller's workspace), 2 keeps the whole
 * per-matrix workspace in LDS (kernels of their own for padded orders up to
 * 32 in float64 and 64 in float32; larger orders given 2 use 64 x 64); all
 * three give bitwise the same results. The choice is read when sincosm_eval_batched is called (a captured
 * graph keeps the choice made at capture). More than one flag is an error. Host-side state shared by all
 * devices, thread-safe; results do not depend on it beyond rounding order. */
enum { SINCOSM_TUNE_MULTI = 16, SINCOSM_TUNE_UNEVEN = 32, SINCOSM_TUNE_BATCHED = 64 };
int sincosm_tune_num_configs(int arith);
sincosm_status sincosm_tune_config_info(int arith, int idx, int32_t* info);
sincosm_status sincosm_tune_set(int arith, int64_t np_lo, int64_t np_hi, int idx);
/* The configuration index the table gives for padded order np in the table
 * `arith` addresses (flags as for sincosm_tune_set; launches of several or
 * unequal problems fall back to the plain table as the launches do), or -1
 * when no entry covers it (the launch then uses its default) or `arith` is
 * invalid. */
int sincosm_tune_lookup(int arith, int64_t np);

#ifdef __cplusplus
}
#endif

#endif /* SINCOSM_H */
