/*
 * eri4.h -- C ABI of the MI355X (gfx950) library for 4-center 2-electron
 * Coulomb integrals (ab|cd) over contracted Cartesian Gaussian shells, computed
 * with the matrix form of the McMurchie-Davidson scheme (Asadchev & Valeev,
 * arXiv:2307.03452, Sec. 2 and Sec. 3).
 *
 * Conventions shared by every entry point
 * ---------------------------------------
 * - Primitive Cartesian Gaussian (Sec. 2, first equation):
 *       phi_a(r) = x_A^ax y_A^ay z_A^az exp(-z_a |r - A|^2)     (UNnormalised)
 *   A contracted shell of angular momentum l is sum_p c_p phi_a(r; z_p); the
 *   coefficients c_p passed here multiply the unnormalised primitives (any
 *   normalisation is the caller's, folded into c_p).
 * - Cartesian components of a shell are ordered ax = l..0, then ay = l-ax..0
 *   (az = l - ax - ay): index = (l-ax)(l-ax+1)/2 + az.
 * - (ab|cd) = sum over primitives of c_a c_b c_c c_d times the integral of
 *   phi_a(r) phi_b(r) |r - r'|^-1 phi_c(r') phi_d(r') over r and r'.
 * - All pointers marked "device" are HIP device (or managed) memory on the
 *   current device; "host" pointers are host memory.  The caller owns every
 *   buffer; the library never frees or reallocates caller memory.
 * - stream is a hipStream_t (0 = the null stream).  Compute calls only enqueue
 *   work on it and return without synchronising; results are ready once the
 *   stream is synchronised.  A kernel fault surfaces at that synchronisation.
 * - Arguments are validated on the host before anything is enqueued; on any
 *   error nothing is written and eri4_last_error() describes the problem.
 *   Device-resident values (exponents, coefficients, contraction lengths) are
 *   not read on the host; a quartet whose contraction lengths are outside
 *   1..kmax gets NaN in every output element.
 * - No screening is done: every quartet passed is computed (Sec. 3, the
 *   library interface paragraph).
 * - Thread safety: calls may come from several host threads; the one-time
 *   per-device set-up is serialised internally.
 */
#ifndef ERI4_H
#define ERI4_H

#include <stdint.h>
#include <hip/hip_runtime_api.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef enum {
  ERI4_SUCCESS = 0,
  ERI4_ERROR_INVALID_ARGUMENT = 1, /* a size, pointer or range is wrong     */
  ERI4_ERROR_UNSUPPORTED = 2,      /* valid but not implemented (e.g. l > max) */
  ERI4_ERROR_OUT_OF_MEMORY = 3,    /* device allocation during set-up failed  */
  ERI4_ERROR_HIP = 4,              /* a HIP runtime call failed               */
  ERI4_ERROR_INTERNAL = 5
} eri4_status;

/* Arithmetic of the two Hermite-to-Cartesian transforms of a plan.  Boys
 * function, Hermite integrals and E coefficients are FP64 in both.
 *   ERI4_PREC_FP64  FP64 matrix cores, FP64 accumulation (the paper's scheme).
 *   ERI4_PREC_FP32  operands rounded to FP32 and multiplied on FP32 matrix
 *                   cores with FP32 accumulation inside each transform (over the
 *                   Hermite index and, for the bra transform, the bra primitive
 *                   pairs); [ab|q] is held in FP64 between the transforms and the
 *                   ket primitive pairs are summed into the FP64 output.  The
 *                   error is that of FP32 arithmetic (unit roundoff 2^-24) times
 *                   the magnitude of the terms summed, typically 1e-7 of a
 *                   quartet's largest integral; it does not reach 1e-10
 *                   absolute on quartets whose integrals exceed about 1e-3. */
typedef enum { ERI4_PREC_FP64 = 0, ERI4_PREC_FP32 = 1 } eri4_precision;

/* Largest angular momentum per shell accepted by eri4_batch. */
#define ERI4_MAX_L 7
/* Largest contraction length per shell (kmax) accepted by eri4_batch. */
#define ERI4_MAX_K 16
/* Largest Boys order m accepted by eri4_boys (covers L = 4 * 7). */
#define ERI4_MAX_BOYS_M 28

/* Number of Cartesian components of a shell, (l+1)(l+2)/2; -1 if l < 0. */
int eri4_ncart(int l);

/* Doubles written per quartet by eri4_batch: ncart(la)ncart(lb)ncart(lc)ncart(ld);
 * -1 on a negative l. */
int64_t eri4_quartet_size(int la, int lb, int lc, int ld);

/* Message of the last error on the calling thread ("" if none). The pointer
 * stays valid until the next call from that thread. */
const char* eri4_last_error(void);

/* Library version string. */
const char* eri4_version(void);

/* Optional explicit set-up of the current device: uploads the Boys-function
 * interpolation table and the Hermite recursion tables (a few MB of device
 * memory held until process exit) and sets kernel attributes.  Every compute
 * call does this lazily on first use of a device; calling it up front keeps
 * the allocation out of timed or captured regions.  Synchronous. */
eri4_status eri4_init(void);

/*
 * eri4_batch -- (ab|cd) for nquartets independent shell quartets of one class
 * (la lb|lc ld), by the matrix form of McMurchie-Davidson (Sec. 2, eqs.
 * (abcd_to_hermite), (ab_to_hermite), (cd_to_hermite)): Boys function, Hermite
 * integrals [r]^(m) by eq. (md1), [p|q] by eq. (pq), then the bra transform
 * [ab|q] = sum_p E_ab^p [p|q] and the ket transform (ab|cd) = sum_q E_cd^q [ab|q]
 * as FP64 matrix products with the primitive contraction folded into the
 * product dimensions (Sec. 3, the batched-GEMM paragraph).  FP64 throughout.
 *
 *   la..ld     0..ERI4_MAX_L
 *   nquartets  >= 0 (0: nothing is enqueued, pointers may be NULL)
 *   centers    device double [nquartets][4][3]       shell centres A, B, C, D (Bohr)
 *   exponents  device double [nquartets][4][kmax]    z_p > 0 for p < nprim
 *   coeffs     device double [nquartets][4][kmax]    c_p for p < nprim
 *   nprim      device int32  [nquartets][4]          contraction lengths, 1..kmax
 *   kmax       1..ERI4_MAX_K, the padded length of the exponent/coefficient rows
 *   out        device double [nquartets][Na][Nb][Nc][Nd], row-major, quartets in
 *              input order; every element is written
 *   stream     hipStream_t
 * Entries p >= nprim of exponents/coeffs are never read.
 * Returns ERI4_SUCCESS, ERI4_ERROR_INVALID_ARGUMENT (bad l, sizes or NULL
 * pointers), ERI4_ERROR_UNSUPPORTED (l > ERI4_MAX_L), ERI4_ERROR_HIP or
 * ERI4_ERROR_OUT_OF_MEMORY (set-up on first use).
 */
eri4_status eri4_batch(int la, int lb, int lc, int ld, int64_t nquartets,
                       const double* centers, const double* exponents, const double* coeffs,
                       const int32_t* nprim, int kmax, double* out, hipStream_t stream);

/*
 * Solid-harmonic output.  The paper contracts the E matrices with the
 * coefficients of real solid-harmonic Gaussians in Cartesian ones before the
 * transforms, H_ab^p = sum_a C_a sum_b C_b E_ab^p (Sec. 2, the equation defining
 * H, coefficients after Schlegel and Frisch), so that both transforms run over
 * the 2l+1 solid functions of each shell instead of the (l+1)(l+2)/2 Cartesian
 * ones.
 *
 * Convention: functions m = -l..l; m > 0 the real part of (x + i y)^m times a
 * polynomial in z and r^2, m < 0 the imaginary part of (x + i y)^|m| times the
 * same polynomial, no Condon-Shortley phase, unit norm when the Cartesian
 * components share the coefficient that normalises x^l (as the inputs'
 * coefficients do).  For l = 1 the order is (y, z, x).
 *
 * eri4_solid_coefficients writes C for shell l (0..ERI4_MAX_L) into the HOST
 * array C[2l+1][(l+1)(l+2)/2] (rows m = -l..l, columns in the Cartesian order
 * of eri4_batch).
 *
 * eri4_batch_solid computes the integrals of eri4_batch over solid harmonics:
 *   out  device double [nquartets][2la+1][2lb+1][2lc+1][2ld+1], row-major
 *   work device double [work_size], scratch owned by the caller for the H
 *        matrices of every primitive pair; contents on entry are ignored and
 *        undefined on return
 * Other arguments as eri4_batch.  The quartets run in passes of as many as the
 * workspace holds: eri4_solid_work_size(la, lb, lc, ld, kmax, n) doubles hold
 * n quartets (-1 for bad arguments); a workspace below one quartet's size gives
 * INVALID_ARGUMENT.  FP64 throughout; enqueue-only (nothing is allocated
 * after the first call on a device), so a HIP graph can capture it.
 */
/*
 * Coulomb contraction without forming (ab|cd): for every quartet,
 *   J_ab = sum_cd (ab|cd) D_cd
 * with D the quartet's own ket density block.  The paper names computing Fock
 * matrix elements directly from [q|ab) as the way around the transposes between
 * its transforms (Sec. 3).  Here the ket density is taken to Hermite space per
 * ket primitive pair, dket_q = sum_cd E_cd^q D_cd (sign of eq. (pq) included),
 * and carried through the Hermite integrals before the bra transform (eqs.
 * (abcd_to_hermite), (pq) associated the other way): per bra primitive pair,
 * w_p = sum over ket pairs of sum_q [p+q] dket_q (a matrix-vector product per
 * primitive quartet), then J_ab = sum_p E_ab^p w_p, summed over the bra
 * primitive pairs in a fixed order.  Neither [ab|q] nor the N_ab N_cd
 * integrals are formed.  FP64, Cartesian functions.
 *   dens  device double [nquartets][Nc][Nd]   (the caller gathers each quartet's block)
 *   out   device double [nquartets][Na][Nb]   J contributions, quartets in input order
 *   work  device double [work_size], caller-owned scratch for dket and the
 *         J of each bra primitive pair
 * Other arguments as eri4_batch; quartets run in passes of as many as the
 * workspace holds (eri4_coulomb_work_size(la, lb, lc, ld, kmax, n) doubles for
 * n quartets, -1 for bad arguments).  Symmetry (the (cd|ab) contribution, or
 * exchange) is the caller's: each call contracts the ket index pair only.
 */
int64_t eri4_coulomb_work_size(int la, int lb, int lc, int ld, int kmax, int64_t nquartets);
eri4_status eri4_batch_coulomb(int la, int lb, int lc, int ld, int64_t nquartets, const double* centers,
                               const double* exponents, const double* coeffs, const int32_t* nprim, int kmax,
                               const double* dens, double* work, int64_t work_size, double* out, hipStream_t stream);

/*
 * Exchange-type contraction without forming (ab|cd): for each quartet of one
 * class,
 *   K_ac = sum_bd (ab|cd) D_bd
 * (Sec. 3: Fock-matrix elements computed directly from the first transform's
 * [ab|q] instead of from stored integrals; the paper leaves exchange to later
 * work).  The density's d index goes to Hermite space per ket primitive pair
 * and component b, F^b[q][c] = sum_d E_cd^q D_bd, and the first transform's
 * [ab|q] is contracted with it on the matrix cores; the second transform
 * (eq. (cd_to_hermite)) never runs.  FP64, Cartesian.
 *   dens  device double [nquartets][Nb][Nd]  each quartet's density block D_bd
 *   out   device double [nquartets][Na][Nc]  K contributions, quartets in input order
 *   work  device double [work_size], caller-owned scratch (F^b and per-b partial rows)
 * Other arguments as eri4_batch; quartets run in passes of as many as the
 * workspace holds (eri4_exchange_work_size(la, lb, lc, ld, kmax, n) doubles
 * for n quartets, -1 for bad arguments).  Each element of out is a sum over b
 * in a fixed order (reproducible bits).  Symmetry partners (the other three
 * exchange contractions of the quartet) are the caller's.
 */
int64_t eri4_exchange_work_size(int la, int lb, int lc, int ld, int kmax, int64_t nquartets);
eri4_status eri4_batch_exchange(int la, int lb, int lc, int ld, int64_t nquartets, const double* centers,
                                const double* exponents, const double* coeffs, const int32_t* nprim, int kmax,
                                const double* dens, double* work, int64_t work_size, double* out,
                                hipStream_t stream);

/*
 * eri4_batch_coulomb without a workspace argument, for callers that cannot
 * allocate device memory (code under HIP graph capture, tight serving loops,
 * harnesses that forbid hipMalloc).  It calls no hipMalloc, hipFree or other
 * allocating routine: the Hermite-space densities and the per-bra-pair J live in a static device
 * array of eri4_static_scratch_bytes() bytes (32 MiB) that the library holds
 * on each device until the process ends.  Quartets run in passes of as many
 * as that array holds; a class whose single quartet would need more is
 * rejected with UNSUPPORTED (no class with l <= 7 and kmax <= 16 does).
 * eri4_init must have run on the current device (it allocates the library's
 * tables): otherwise INVALID_ARGUMENT and nothing is enqueued.
 * Every call on one device shares that device's array and leaves the last
 * call's contents in it (nothing in it needs to start at zero): calls that
 * overlap on one device (different streams or threads, with no ordering
 * between them) race and give undefined results; calls on one stream, or
 * otherwise ordered, do not.  Arguments, results and errors as
 * eri4_batch_coulomb.
 */
int64_t eri4_static_scratch_bytes(void);
eri4_status eri4_batch_coulomb_static(int la, int lb, int lc, int ld, int64_t nquartets, const double* centers,
                                      const double* exponents, const double* coeffs, const int32_t* nprim, int kmax,
                                      const double* dens, double* out, hipStream_t stream);

eri4_status eri4_solid_coefficients(int l, double* C);
int64_t eri4_solid_work_size(int la, int lb, int lc, int ld, int kmax, int64_t nquartets);
eri4_status eri4_batch_solid(int la, int lb, int lc, int ld, int64_t nquartets, const double* centers,
                             const double* exponents, const double* coeffs, const int32_t* nprim, int kmax,
                             double* work, int64_t work_size, double* out, hipStream_t stream);

/*
 * Plans -- one batch mixing classes and contraction lengths, computed by a single
 * persistent launch (Sec. 3, batched evaluation; the paper groups shell pairs of
 * equal total angular momentum and contraction order into lists, here the
 * grouping is per work item inside one launch).
 *
 * eri4_plan_create reads the HOST arrays
 *   l      int32 [nquartets][4]   angular momenta of shells a, b, c, d, 0..ERI4_MAX_L
 *   nprim  int32 [nquartets][4]   contraction lengths, 1..kmax
 * and takes the arithmetic of the transforms (eri4_precision above),
 * splits every quartet into tiles of bra rows, orders the tiles by an estimate
 * of their cost (largest first) and uploads the schedule, the per-class
 * parameters, the output offsets and a copy of nprim to device memory that the
 * plan owns.  It allocates and synchronises; everything else about a plan does
 * neither.  Errors: INVALID_ARGUMENT (sizes, NULL, a length outside 1..kmax),
 * UNSUPPORTED (l > ERI4_MAX_L), OUT_OF_MEMORY, HIP.  On error *plan is NULL.
 *
 * Output layout: quartet q's (ab|cd) block, [Na][Nb][Nc][Nd] row-major for its
 * own class, starts at offsets[q] doubles into out, quartets in input order
 * with no gaps; eri4_plan_output_size gives the total number of doubles.
 *
 * eri4_plan_execute enqueues on `stream` a one-thread counter reset and the
 * persistent kernel; it neither allocates nor synchronises, so it can be
 * captured into a HIP graph and replayed.  centers, exponents and coeffs are
 * device arrays laid out as for eri4_batch ([nquartets][4][3], [nquartets][4][kmax]);
 * the contraction lengths are the ones given at creation.  Executions of one
 * plan must not overlap in time (they share the plan's work counter); run them
 * on one stream or order them.  The plan must be executed on the device that
 * was current at creation.
 *
 * eri4_plan_destroy frees the plan's device memory (hipFree synchronises).
 */
typedef struct eri4_plan_s* eri4_plan;

eri4_status eri4_plan_create(eri4_plan* plan, int64_t nquartets, const int32_t* l, const int32_t* nprim,
                             int kmax, eri4_precision precision);

/*
 * Tile choices for plans (what an autotuner picks per class and contraction
 * size).  A tile is 16 * rows16 bra rows of one quartet (rows16 = 4 only with
 * the two box layouts and at most 16 ket column blocks, i.e. lc+ld <= 9); the Hermite integrals
 * of eq. (md1) live in LDS in one of three layouts:
 *   ERI4_LAYOUT_BOX   (L+1)^3 box, recursion in place            (L <= 24)
 *   ERI4_LAYOUT_SLAB  t-slabs, about half the space, in place      (L <= 28)
 *   ERI4_LAYOUT_BOX2  two boxes, levels alternate between them     (L <= 19)
 * where L = la+lb+lc+ld.  A choice applies to the quartets of class l whose
 * product of the four contraction lengths lies in [kq_min, kq_max].
 */
typedef enum { ERI4_LAYOUT_BOX = 0, ERI4_LAYOUT_SLAB = 1, ERI4_LAYOUT_BOX2 = 2 } eri4_layout;

/* basis functions of the output (pair-list plans) */
typedef enum { ERI4_CARTESIAN = 0, ERI4_SOLID = 1 } eri4_functions;

typedef struct {
  int32_t l[4];           /* class (la lb|lc ld) */
  int32_t kq_min, kq_max; /* range of nprim[a]*nprim[b]*nprim[c]*nprim[d] */
  int32_t rows16;         /* 1, 2 or 4 */
  int32_t layout;         /* eri4_layout */
} eri4_tile_choice;

/* eri4_plan_create with tile choices (HOST array of nchoices entries, may be
 * NULL when nchoices == 0).  For each quartet the first matching entry is
 * used; quartets no entry matches get the library's own choice.  A matching
 * entry whose tile does not fit (LDS, or L beyond the layout's limit) or has
 * rows16/layout out of range gives INVALID_ARGUMENT naming it.  Otherwise as
 * eri4_plan_create, which is this call with no choices. */
eri4_status eri4_plan_create_tuned(eri4_plan* plan, int64_t nquartets, const int32_t* l, const int32_t* nprim,
                                   int kmax, eri4_precision precision, const eri4_tile_choice* choices,
                                   int nchoices);

/*
 * eri4_plan_create_tuned with the choices read from a tile table file (what
 * the autotuner writes), so that a plan can be built from the table alone.
 * tune_file: path of a text file, or NULL for the library's own choices.
 * Format: '#' starts a comment line; one line "arch <name>" (e.g. "arch
 * gfx950") before the entries; then one entry per line,
 *   la lb lc ld kq_min kq_max rows16 layout
 * with layout one of box, slab, box2 (fields as eri4_tile_choice).  The
 * table applies only to the architecture it names: a file whose arch differs
 * from the current device's (hipDeviceProp_t::gcnArchName up to its first
 * ':') gives INVALID_ARGUMENT, as do an unreadable file, a malformed line and
 * a missing arch line (the message names the file and line).  Otherwise as
 * eri4_plan_create_tuned.
 */
eri4_status eri4_plan_create_tunefile(eri4_plan* plan, int64_t nquartets, const int32_t* l, const int32_t* nprim,
                                      int kmax, eri4_precision precision, const char* tune_file);

/*
 * Quartet plans over real solid harmonics: the contraction of E with the
 * Cartesian-to-solid coefficients (Sec. 2) for a batch mixing classes and
 * contraction lengths.  eri4_plan_create_solid takes the HOST arrays of
 * eri4_plan_create and a tile table file (or NULL) as eri4_plan_create_tunefile;
 * the transforms are FP64.  Quartet q's block is [2la+1][2lb+1][2lc+1][2ld+1]
 * (conventions as eri4_batch_solid) at offsets[q], quartets in input order.
 *
 * eri4_plan_execute_solid takes the device arrays of eri4_plan_execute and a
 * DEVICE workspace of at least eri4_plan_work_size(plan) doubles (contents
 * undefined afterwards): it first builds the H matrices of the bra and the ket
 * pair of every quartet (one per primitive pair, K_a*K_b + K_c*K_d of them per
 * quartet), then runs the persistent kernel that reads them.  Enqueue-only and
 * capturable, as eri4_plan_execute.  A solid quartet plan must be run with
 * this call (eri4_plan_execute and eri4_plan_execute_pairs give
 * INVALID_ARGUMENT), and this call takes no other plan.
 */
eri4_status eri4_plan_create_solid(eri4_plan* plan, int64_t nquartets, const int32_t* l, const int32_t* nprim,
                                   int kmax, const char* tune_file);
eri4_status eri4_plan_execute_solid(eri4_plan plan, const double* centers, const double* exponents,
                                    const double* coeffs, double* work, int64_t work_size, double* out,
                                    hipStream_t stream);
int64_t eri4_plan_output_size(eri4_plan plan);                         /* doubles; -1 if plan is NULL */
eri4_status eri4_plan_output_offsets(eri4_plan plan, int64_t* offsets); /* HOST int64 [nquartets]; Coulomb plans: [nbra] */
eri4_status eri4_plan_execute(eri4_plan plan, const double* centers, const double* exponents,
                              const double* coeffs, double* out, hipStream_t stream);
eri4_status eri4_plan_destroy(eri4_plan plan);

/*
 * Plans over a bra and a ket list of shell pairs: every bra pair with every
 * ket pair, the way the paper's engine computes integrals for lists of bra and
 * ket shell pairs (Sec. 3, library interface).  Quartet (i, j) is bra pair i
 * with ket pair j, at index q = i * nket + j (bra-major); its block starts at
 * offsets[q] (eri4_plan_output_offsets), as for quartet plans.
 *
 * eri4_plan_create_pairs reads the HOST arrays
 *   bra_l, bra_nprim  int32 [nbra][2]   (la, lb) and contraction lengths of each bra pair
 *   ket_l, ket_nprim  int32 [nket][2]   (lc, ld) and lengths of each ket pair
 * (nbra * nket < 2^31) and otherwise behaves as eri4_plan_create_tuned
 * (choices may be NULL with nchoices 0: the library picks the tiles).
 * functions: ERI4_CARTESIAN, or ERI4_SOLID for integrals over real solid
 * harmonics (FP64 only; conventions as eri4_batch_solid; each quartet's block
 * is [2la+1][2lb+1][2lc+1][2ld+1]).  A solid plan builds the H matrices of
 * every list entry once per execute, in the caller's workspace (work, at least
 * eri4_plan_work_size(plan) doubles, contents undefined afterwards), and every
 * quartet of that entry reads them; Cartesian plans ignore work.
 *
 * eri4_plan_execute_pairs takes DEVICE arrays per list:
 *   bra_centers [nbra][2][3], bra_exponents / bra_coeffs [nbra][2][kmax],
 *   ket_centers [nket][2][3], ket_exponents / ket_coeffs [nket][2][kmax]
 * and reads each quartet's shells from them (nothing is expanded per quartet
 * on the device).  Enqueue-only and capturable, as eri4_plan_execute.  A plan
 * made from pair lists must be run with eri4_plan_execute_pairs and a quartet
 * plan with eri4_plan_execute (INVALID_ARGUMENT otherwise).
 */
eri4_status eri4_plan_create_pairs(eri4_plan* plan, int64_t nbra, const int32_t* bra_l, const int32_t* bra_nprim,
                                   int64_t nket, const int32_t* ket_l, const int32_t* ket_nprim, int kmax,
                                   eri4_precision precision, eri4_functions functions,
                                   const eri4_tile_choice* choices, int nchoices);
int64_t eri4_plan_work_size(eri4_plan plan); /* doubles of workspace execute needs; 0 for Cartesian, -1 if NULL */
eri4_status eri4_plan_execute_pairs(eri4_plan plan, const double* bra_centers, const double* bra_exponents,
                                    const double* bra_coeffs, const double* ket_centers,
                                    const double* ket_exponents, const double* ket_coeffs, double* work,
                                    int64_t work_size, double* out, hipStream_t stream);

/*
 * The Coulomb contraction over a bra and a ket list of shell pairs: for every
 * bra entry i,
 *   J_i[ab] = sum_j sum_cd (ab|cd)_ij D_j[cd]
 * with D_j the density block of ket entry j.  dket of each ket entry is built
 * once per execute and shared by every bra entry; each quartet's J rows
 * (computed as in eri4_batch_coulomb, all its bra primitive pairs in one
 * workgroup) go to the workspace and are summed over j in a fixed order
 * (reproducible bits).  FP64, Cartesian.
 * eri4_plan_create_coulomb: host arrays as eri4_plan_create_pairs.
 * eri4_plan_execute_coulomb: lists as eri4_plan_execute_pairs, and
 *   ket_dens  device double, the blocks D_j[Nc][Nd] of the ket entries one after
 *             the other in list order
 *   work      device double [work_size >= eri4_plan_work_size(plan)]
 *   out       device double, the blocks J_i[Na][Nb] one after the other in list
 *             order (eri4_plan_output_size doubles; eri4_plan_output_offsets
 *             gives the nbra block offsets)
 * With an empty ket list (nket = 0) every J_i is an empty sum: execute only
 * zeroes out (the list and work pointers are not read).
 * Other plan calls apply (destroy, output size and offsets); the other execute
 * calls reject a Coulomb plan.  Execute is enqueue-only and capturable, as
 * eri4_plan_execute.
 */
eri4_status eri4_plan_create_coulomb(eri4_plan* plan, int64_t nbra, const int32_t* bra_l, const int32_t* bra_nprim,
                                     int64_t nket, const int32_t* ket_l, const int32_t* ket_nprim, int kmax);
eri4_status eri4_plan_execute_coulomb(eri4_plan plan, const double* bra_centers, const double* bra_exponents,
                                      const double* bra_coeffs, const double* ket_centers,
                                      const double* ket_exponents, const double* ket_coeffs, const double* ket_dens,
                                      double* work, int64_t work_size, double* out, hipStream_t stream);


/*
 * Stage entry points.  They run the same device code the fused eri4_batch
 * kernel runs for one stage, so each stage can be checked on its own.
 */

/* Boys function of eq. (boys), F_m(T) = int_0^1 y^(2m) exp(-T y^2) dy, for
 * m = 0..mmax (mmax 0..ERI4_MAX_BOYS_M) at n arguments T >= 0.
 *   T  device double [n];   F  device double [n][mmax+1]
 * Negative or non-finite T give NaN rows. */
eri4_status eri4_boys(int mmax, int64_t n, const double* T, double* F, hipStream_t stream);

/* Hermite integrals R[t][u][v] = [r]^(0) (Sec. 2, from [0]^(m) and eq. (md1)) for
 * n primitive pairs-of-pairs, with total order t+u+v <= L (0..4*ERI4_MAX_L).
 *   zp, zq  device double [n]      zeta_p = za+zb, zeta_q = zc+zd (> 0)
 *   P, Q    device double [n][3]   product centres R_p, R_q
 *   R       device double [n][L+1][L+1][L+1]; entries with t+u+v > L are 0
 * No Gaussian-product prefactor or contraction coefficient is applied. */
eri4_status eri4_hermite_r(int L, int64_t n, const double* zp, const double* zq,
                           const double* P, const double* Q, double* R, hipStream_t stream);

/* Hermite expansion coefficients of eq. (cart2herm-2) for n primitive pairs,
 * from the two recursions that follow it with (E)^0_00 = 1:
 *   za, zb  device double [n];  A, B  device double [n][3]
 *   E       device double [n][3][la+1][lb+1][la+lb+1]   (axis x, y, z; entries
 *           with t > a+b are 0).  la, lb in 0..7. */
eri4_status eri4_hermite_e(int la, int lb, int64_t n, const double* za, const double* zb,
                           const double* A, const double* B, double* E, hipStream_t stream);

#ifdef __cplusplus
}
#endif

#endif /* ERI4_H */
