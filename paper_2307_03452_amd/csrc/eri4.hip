// eri4.hip -- host side of liberi4's C ABI (gfx950), and the small stage
// kernels.  The fused and plan kernels live in eri4_device.h and are compiled
// in eri4_fused.hip, eri4_plan64.hip and eri4_plan32.hip.
//
// (ab|cd) over contracted Cartesian Gaussians by the matrix form of the
// McMurchie-Davidson scheme (Asadchev & Valeev, Sec. 2 and Sec. 3).
#include <hip/hip_runtime.h>

#include <algorithm>
#include <array>
#include <cmath>
#include <cstdarg>
#include <cstdio>
#include <cstring>
#include <deque>
#include <map>
#include <mutex>
#include <new>
#include <numeric>
#include <string>
#include <vector>

#include "eri4.h"
#include "eri4_device.h"
#include "eri4_internal.h"
#include "eri4_launch.h"

namespace eri4 {
void make_boys_table(std::vector<double>& tab);
void make_rtabs(std::vector<uint32_t>& tab, std::vector<int>& start);
void make_solid_table(std::vector<double>& tab);
void solid_dense(int l, double* C);

__global__ void reset_counter_kernel(int* counter) {
  if (threadIdx.x == 0) counter[0] = 0;
}

// out[0..n) = 0 (a kernel rather than a memset, so that graph captures of the
// calls that use it stay correct on replay)
__global__ void zero_fill_kernel(double* __restrict__ out, int64_t n) {
  for (int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; i < n; i += (int64_t)gridDim.x * blockDim.x)
    out[i] = 0.0;
}

// ---------------------------------------------------------------------------
// stage kernels (same device code as the fused kernel)
// ---------------------------------------------------------------------------

__global__ void boys_kernel(int mmax, int64_t n, const double* __restrict__ T, double* __restrict__ F,
                            const double* __restrict__ tab) {
  const int64_t g = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  const int64_t total = n * (mmax + 1);
  if (g >= total) return;
  const int64_t i = g / (mmax + 1);
  const int m = (int)(g - i * (mmax + 1));
  F[g] = boys_fm(m, T[i], tab);
}

__global__ __launch_bounds__(kThreads, 1) void hermite_r_kernel(
    int L, bool slab, const double* __restrict__ zp, const double* __restrict__ zq, const double* __restrict__ P,
    const double* __restrict__ Q, double* __restrict__ R, const double* __restrict__ boys_tab,
    const uint2* __restrict__ rtab_L) {
  extern __shared__ __align__(16) unsigned char lds[];
  double* baseM = (double*)lds;
  double* pq = baseM + 32;
  double* box = baseM + 36;
  const int tid = threadIdx.x;
  const int64_t it = blockIdx.x;
  const int n1 = L + 1;
  const double a = zp[it], b = zq[it];
  double PQ[3];
  for (int x = 0; x < 3; ++x) PQ[x] = P[it * 3 + x] - Q[it * 3 + x];
  if (tid < 3) pq[tid] = PQ[tid];
  if (tid <= L) {
    const double rho = a * b / (a + b);
    const double T = rho * (PQ[0] * PQ[0] + PQ[1] * PQ[1] + PQ[2] * PQ[2]);
    double pw = 1.0;
    for (int mm = 0; mm < tid; ++mm) pw *= -2.0 * rho;
    baseM[tid] = pw * (2.0 * pow(M_PI, 2.5) / (a * b * sqrt(a + b))) * boys_fm(tid, T, boys_tab);
  }
  uint2 rent[kRPerThread];
  load_rtab(rent, rtab_L, L, tid);
  __syncthreads();
  hermite_r_lds(box, baseM, L, pq, rent, tid);
  double* o = R + it * (int64_t)n1 * n1 * n1;
  for (int e = tid; e < n1 * n1 * n1; e += kThreads) {
    const int t = e / (n1 * n1), u = (e / n1) % n1, v = e % n1;
    o[e] = (t + u + v <= L) ? box[r_offset(slab, L, t, u, v)] : 0.0;
  }
}

__global__ void hermite_e_kernel(int la, int lb, const double* __restrict__ za, const double* __restrict__ zb,
                                 const double* __restrict__ A, const double* __restrict__ B,
                                 double* __restrict__ E) {
  extern __shared__ __align__(16) unsigned char lds[];
  double* tabs = (double*)lds;
  const int lane = threadIdx.x;
  const int64_t it = blockIdx.x;
  const int trow = odd_row(la + lb + 2);
  const int taxis = ((la + 1) * (lb + 1) + 1) * trow;
  double* pair = tabs + 3 * taxis;
  if (lane == 0) {
    double Av[3], Bv[3];
    for (int x = 0; x < 3; ++x) {
      Av[x] = A[it * 3 + x];
      Bv[x] = B[it * 3 + x];
    }
    make_pair(pair, za[it], zb[it], 1.0, 1.0, Av, Bv);
  }
  __syncthreads();
  build_etab(tabs, la, lb, trow, taxis, 0.5 / pair[0], pair + 5, pair + 8, false, lane);
  __syncthreads();
  const int nt = la + lb + 1;
  const int per_axis = (la + 1) * (lb + 1) * nt;
  double* o = E + it * 3 * per_axis;
  for (int e = lane; e < 3 * per_axis; e += blockDim.x) {
    const int axis = e / per_axis, rem = e - axis * per_axis;
    const int ab = rem / nt, t = rem - ab * nt;
    o[e] = tabs[axis * taxis + ab * trow + t];
  }
}

// ---------------------------------------------------------------------------
// host side
// ---------------------------------------------------------------------------

namespace {

thread_local std::string g_err;

eri4_status fail(eri4_status s, const char* fmt, ...) {
  char buf[512];
  va_list ap;
  va_start(ap, fmt);
  vsnprintf(buf, sizeof buf, fmt, ap);
  va_end(ap);
  g_err = buf;
  return s;
}

// Device scratch of the no-allocation Coulomb call (eri4_batch_coulomb_static):
// the Hermite-space ket densities of one pass of quartets.  Each device holds
// its own copy until the process ends.  Host code must never pass this name to
// a kernel or a copy (on the host it is only a stand-in, not a device address):
// it uses the address that hipGetSymbolAddress returned for the current device
// (DeviceState::scratch), taken once per device in ensure_device.
constexpr int64_t kStaticScratchDoubles = (int64_t)4 << 20;  // 32 MiB
static __device__ __align__(256) double scratch[kStaticScratchDoubles];

struct DeviceState {
  bool ready = false;
  double* scratch = nullptr;  // this device's address of `scratch`
  double* boys = nullptr;
  uint2* rtab = nullptr;
  double* stab = nullptr;  // solid-harmonic coefficients (make_solid_table)
  int rstart[2 * (kMaxL + 1)] = {0};  // [layout][L], in uint2 entries
};

std::mutex g_mu;
std::deque<DeviceState> g_dev;  // a deque: growing it keeps pointers to existing entries valid

#define HIP_TRY(call)                                                                     \
  do {                                                                                    \
    hipError_t e_ = (call);                                                               \
    if (e_ != hipSuccess) return fail(ERI4_ERROR_HIP, "%s: %s", #call, hipGetErrorString(e_)); \
  } while (0)

eri4_status set_attrs() {
  HIP_TRY(fused_set_attrs());
  HIP_TRY(small_set_attrs());
  HIP_TRY(solid_set_attrs());
  HIP_TRY(plan_solid_set_attrs());
  HIP_TRY(coulomb_set_attrs());
  HIP_TRY(exchange_set_attrs());
  HIP_TRY(plan_coulomb_set_attrs());
  HIP_TRY(plan_set_attrs_f64());
  HIP_TRY(plan_set_attrs_f32());
  HIP_TRY(plan_set_attrs_f64p());
  HIP_TRY(plan_set_attrs_f32p());
  HIP_TRY(hipFuncSetAttribute((const void*)hermite_r_kernel, hipFuncAttributeMaxDynamicSharedMemorySize,
                              kMaxLdsBytes));
  return ERI4_SUCCESS;
}

eri4_status ensure_device(DeviceState** st) {
  int dev = 0;
  HIP_TRY(hipGetDevice(&dev));
  std::lock_guard<std::mutex> lk(g_mu);
  if ((int)g_dev.size() <= dev) g_dev.resize(dev + 1);
  DeviceState& d = g_dev[dev];
  if (!d.ready) {
    static std::vector<double> boys;
    static std::vector<uint32_t> rt;
    static std::vector<int> rs;
    static std::vector<double> st;
    if (boys.empty()) {
      make_boys_table(boys);
      make_rtabs(rt, rs);
      make_solid_table(st);
    }
    if ((int)rt.size() != 2 * 2 * kRtabEntries) return fail(ERI4_ERROR_INTERNAL, "recursion table size mismatch");
    if (hipMalloc(&d.boys, boys.size() * sizeof(double)) != hipSuccess)
      return fail(ERI4_ERROR_OUT_OF_MEMORY, "device allocation of the Boys table failed");
    if (hipMalloc(&d.rtab, rt.size() * sizeof(uint32_t)) != hipSuccess)
      return fail(ERI4_ERROR_OUT_OF_MEMORY, "device allocation of the recursion tables failed");
    HIP_TRY(hipMemcpy(d.boys, boys.data(), boys.size() * sizeof(double), hipMemcpyHostToDevice));
    HIP_TRY(hipMemcpy(d.rtab, rt.data(), rt.size() * sizeof(uint32_t), hipMemcpyHostToDevice));
    if (hipMalloc(&d.stab, st.size() * sizeof(double)) != hipSuccess)
      return fail(ERI4_ERROR_OUT_OF_MEMORY, "device allocation of the solid-harmonic table failed");
    HIP_TRY(hipMemcpy(d.stab, st.data(), st.size() * sizeof(double), hipMemcpyHostToDevice));
    for (int i = 0; i < 2 * (kMaxL + 1); ++i) d.rstart[i] = rs[i];
    HIP_TRY(hipGetSymbolAddress((void**)&d.scratch, HIP_SYMBOL(scratch)));
    eri4_status s = set_attrs();
    if (s != ERI4_SUCCESS) return s;
    d.ready = true;
  }
  *st = &d;
  return ERI4_SUCCESS;
}

int align16(int x) { return (x + 15) & ~15; }

// Class parameters and LDS layout for a tile of rb*16 bra rows.  xs: row
// stride of the [ab|q] staging area in doubles (0: 16 * nqb + 2, every column
// the first transform's accumulators hold).
ClassParams make_params(int la, int lb, int lc, int ld, int kmax, int rb, bool slab, bool box2, int xs = 0) {
  ClassParams p{};
  p.rb = rb;
  p.slab = slab ? 1 : 0;
  p.la = la; p.lb = lb; p.lc = lc; p.ld = ld;
  p.na = ncart(la); p.nb = ncart(lb); p.nc = ncart(lc); p.nd = ncart(ld);
  p.nab = p.na * p.nb; p.ncd = p.nc * p.nd;
  p.Lb = la + lb; p.Lk = lc + ld; p.L = p.Lb + p.Lk;
  p.np = nherm(p.Lb); p.nq = nherm(p.Lk);
  p.np4 = (p.np + 3) & ~3; p.nq4 = (p.nq + 3) & ~3;
  p.nqb = (p.nq + 15) / 16;
  p.ncdb = (p.ncd + 15) / 16;
  p.nrt = (p.nab + 16 * rb - 1) / (16 * rb);
  p.S1 = box_s1(p.L); p.S2 = box_s2(p.L);
  p.tbrow = odd_row(p.Lb + 2); p.tkrow = odd_row(p.Lk + 2);
  p.tbaxis = ((la + 1) * (lb + 1) + 1) * p.tbrow;
  p.tkaxis = ((lc + 1) * (ld + 1) + 1) * p.tkrow;
  p.xs = xs > 0 ? xs : 16 * p.nqb + 2;
  p.kmax = kmax;
  int off = 0;
  p.o_shell = off; off = align16(off + (12 + 8 * kmax) * 8 + 4 * 4);
  p.o_base = off;  off = align16(off + 96 * 8);  // [0]^(m), ket pair, bra pair, P-Q
  p.o_ptab = off;  off = align16(off + p.np4 * 8);
  p.o_qtab = off;  off = align16(off + 16 * p.nqb * 8);
  p.o_union = off;
  const int box_b = r_cells(slab, p.L) * 8;
  p.lay = slab ? kLaySlab : (box2 ? kLayBox2 : kLayBox);
  // phase 1: R box, bra tables[, second R box]
  p.o_box1 = off + align16(box_b) + align16(3 * p.tbaxis * 8);
  const int ph1 = box2 ? p.o_box1 - off + box_b : align16(box_b) + 3 * p.tbaxis * 8;
  const int xb = align16(rb * 16 * p.xs * 8);
  const int ph2 = xb + 3 * p.tkaxis * 8;
  p.o_brae = off + align16(box_b);
  p.o_kete = off + xb;
  off = align16(off + (ph1 > ph2 ? ph1 : ph2));
  p.lds_bytes = off;
  return p;
}

// Class parameters for one tile height and R layout, if they fit (limit:
// bytes of LDS available for the dynamic area; column blocks per wave within
// what the kernel bodies are instantiated for).
bool try_params(int la, int lb, int lc, int ld, int kmax, int rb, int lay, const DeviceState* d, int limit,
                ClassParams* out) {
  const bool slab = lay == kLaySlab, two = lay == kLayBox2;
  if ((rb != 1 && rb != 2 && rb != 4) || lay < kLayBox || lay > kLayBox2) return false;
  if (rb == 4 && slab) return false;  // 64-row tiles are built for the box layouts
  if (two && la + lb + lc + ld > kBox2LMax) return false;
  ClassParams p = make_params(la, lb, lc, ld, kmax, rb, slab, two);
  const int maxc = rb == 4 ? 2 : (slab && rb == 1 ? kMaxC1 : 4);
  if (p.lds_bytes > limit || p.L > kMaxL || (p.nqb + 7) / 8 > maxc) return false;
  if (!slab && p.L > kBoxLMax) return false;  // the box recursion holds kRPerBox entries per thread
  p.rtab_off = d ? d->rstart[(slab ? 1 : 0) * (kMaxL + 1) + p.L] : 0;
  *out = p;
  return true;
}

// The library's own choice: the first that fits of two boxes (64-row tiles,
// then 32, then 16), box (the same), slab (32, 16).
bool pick_params(int la, int lb, int lc, int ld, int kmax, const DeviceState* d, int limit, ClassParams* out) {
  static const int order[8][2] = {{4, kLayBox2}, {2, kLayBox2}, {1, kLayBox2}, {4, kLayBox},
                                  {2, kLayBox},  {1, kLayBox},  {2, kLaySlab}, {1, kLaySlab}};
  for (const auto& o : order)
    if (try_params(la, lb, lc, ld, kmax, o[0], o[1], d, limit, out)) return true;
  return false;
}

// The low-l kernels: one wave per quartet for kets of at most four [ab|q]
// column blocks, four waves for more.
bool small_four_waves(const ClassParams& p) { return p.nqb > 4; }

// The low-l kernels' parameters for classes whose shells all have l <=
// kSmallLMax: box layout, rb = bra row blocks per pass (at most 3, with at
// most 12 first-transform accumulator blocks of 16 x 16, spread evenly over
// the passes: (fd|fd)'s 4 row blocks run as 2 + 2, not 3 + 1).  The [ab|q]
// rows hold only the nq4 columns the second transform reads (the kernels
// store no others); the one-wave kernel keeps the recursion table for L in
// the last align16(8 nherm(L)) bytes.
bool small_params(int la, int lb, int lc, int ld, int kmax, const DeviceState* d, ClassParams* out) {
  if (la > kSmallLMax || lb > kSmallLMax || lc > kSmallLMax || ld > kSmallLMax) return false;
  const int nrb = (ncart(la) * ncart(lb) + 15) / 16, nqb = (nherm(lc + ld) + 15) / 16;
  int rg = std::min(nrb, 3);
  while (rg > 1 && rg * nqb > 12) --rg;
  const int passes = (nrb + rg - 1) / rg;
  rg = (nrb + passes - 1) / passes;
  const int nq4 = (nherm(lc + ld) + 3) & ~3;
  ClassParams p = make_params(la, lb, lc, ld, kmax, rg, false, false, nq4 + 2);
  if (!small_four_waves(p)) p.lds_bytes += align16(8 * nherm(p.L));
  if (p.lds_bytes > kSmallLdsMax || p.nqb > 6) return false;
  p.rtab_off = d ? d->rstart[p.L] : 0;
  *out = p;
  return true;
}

// Solid-harmonic output: the library's tile for the class, with rows and
// columns over the 2l+1 real solid harmonics of each shell; hbs / hks doubles
// of H per bra / ket primitive pair (rows padded to whole tiles, columns to
// whole 16-column blocks, k to the padded Hermite counts).
void to_solid(ClassParams* p) {
  p->na = 2 * p->la + 1; p->nb = 2 * p->lb + 1; p->nc = 2 * p->lc + 1; p->nd = 2 * p->ld + 1;
  p->nab = p->na * p->nb;
  p->ncd = p->nc * p->nd;
  p->nrt = (p->nab + 16 * p->rb - 1) / (16 * p->rb);
  p->ncdb = (p->ncd + 15) / 16;
}

bool solid_params(int la, int lb, int lc, int ld, int kmax, const DeviceState* d, ClassParams* p, int64_t* hbs,
                  int64_t* hks) {
  if (!pick_params(la, lb, lc, ld, kmax, d, kMaxLdsBytes, p)) return false;
  to_solid(p);
  *hbs = (int64_t)p->nrt * p->rb * 16 * p->np4;
  *hks = (int64_t)p->ncdb * 16 * p->nq4;
  return true;
}

}  // namespace
}  // namespace eri4

using namespace eri4;

extern "C" {

int eri4_ncart(int l) { return l < 0 ? -1 : ncart(l); }

int64_t eri4_quartet_size(int la, int lb, int lc, int ld) {
  if (la < 0 || lb < 0 || lc < 0 || ld < 0) return -1;
  return (int64_t)ncart(la) * ncart(lb) * ncart(lc) * ncart(ld);
}

const char* eri4_last_error(void) { return g_err.c_str(); }

const char* eri4_version(void) { return "eri4 0.1 (gfx950, FP64 MFMA matrix McMurchie-Davidson)"; }

eri4_status eri4_init(void) {
  g_err.clear();
  DeviceState* d;
  return ensure_device(&d);
}

eri4_status eri4_batch(int la, int lb, int lc, int ld, int64_t nquartets, const double* centers,
                       const double* exponents, const double* coeffs, const int32_t* nprim, int kmax,
                       double* out, hipStream_t stream) {
  g_err.clear();
  if (la < 0 || lb < 0 || lc < 0 || ld < 0)
    return fail(ERI4_ERROR_INVALID_ARGUMENT, "angular momenta must be >= 0 (got %d %d %d %d)", la, lb, lc, ld);
  if (la > ERI4_MAX_L || lb > ERI4_MAX_L || lc > ERI4_MAX_L || ld > ERI4_MAX_L)
    return fail(ERI4_ERROR_UNSUPPORTED, "angular momentum above %d is not supported (got %d %d %d %d)",
                ERI4_MAX_L, la, lb, lc, ld);
  if (nquartets < 0) return fail(ERI4_ERROR_INVALID_ARGUMENT, "nquartets must be >= 0");
  if (kmax < 1 || kmax > ERI4_MAX_K)
    return fail(ERI4_ERROR_INVALID_ARGUMENT, "kmax must be in 1..%d (got %d)", ERI4_MAX_K, kmax);
  if (nquartets == 0) return ERI4_SUCCESS;
  if (!centers || !exponents || !coeffs || !nprim || !out)
    return fail(ERI4_ERROR_INVALID_ARGUMENT, "NULL buffer pointer");
  DeviceState* d;
  eri4_status s = ensure_device(&d);
  if (s != ERI4_SUCCESS) return s;
  ClassParams p;
  if (small_params(la, lb, lc, ld, kmax, d, &p)) {
    const int64_t qchunk = (int64_t)1 << 24;  // grid of qchunk workgroups of at most 256 threads
    for (int64_t q0 = 0; q0 < nquartets; q0 += qchunk) {
      const int64_t nq = std::min(qchunk, nquartets - q0);
      // four waves per quartet for kets with more than four [ab|q] column
      // blocks, one wave otherwise (measured: (ff|ff) 10-16% faster on four
      // waves at K_bra K_ket = 1, 5 and 25; (dd|dd) faster on one wave)
      const bool four = small_four_waves(p);
      const Tables tb{d->boys, d->rtab};
      const hipError_t e = four ? small4_launch(p, nq, stream, tb, centers, exponents, coeffs, nprim, out, q0)
                                : small_launch(p, nq, stream, tb, centers, exponents, coeffs, nprim, out, q0);
      if (e != hipSuccess) return fail(ERI4_ERROR_HIP, "kernel launch: %s", hipGetErrorString(e));
    }
    return ERI4_SUCCESS;
  }
  if (!pick_params(la, lb, lc, ld, kmax, d, kMaxLdsBytes, &p))
    return fail(ERI4_ERROR_UNSUPPORTED, "class (%d %d|%d %d) does not fit in LDS", la, lb, lc, ld);
  const int64_t max_blocks = (int64_t)1 << 30;
  const int64_t qchunk = max_blocks / p.nrt;
  for (int64_t q0 = 0; q0 < nquartets; q0 += qchunk) {
    const int64_t nq = (nquartets - q0 < qchunk) ? nquartets - q0 : qchunk;
    const dim3 grid((unsigned)(nq * p.nrt));
    const hipError_t e =
        fused_launch(p, grid, stream, Tables{d->boys, d->rtab}, centers, exponents, coeffs, nprim, out, q0);
    if (e != hipSuccess) return fail(ERI4_ERROR_HIP, "kernel launch: %s", hipGetErrorString(e));
  }
  return ERI4_SUCCESS;
}

static eri4_status check_class(int la, int lb, int lc, int ld, int64_t nquartets, int kmax) {
  if (la < 0 || lb < 0 || lc < 0 || ld < 0)
    return fail(ERI4_ERROR_INVALID_ARGUMENT, "angular momenta must be >= 0 (got %d %d %d %d)", la, lb, lc, ld);
  if (la > ERI4_MAX_L || lb > ERI4_MAX_L || lc > ERI4_MAX_L || ld > ERI4_MAX_L)
    return fail(ERI4_ERROR_UNSUPPORTED, "angular momentum above %d is not supported (got %d %d %d %d)",
                ERI4_MAX_L, la, lb, lc, ld);
  if (nquartets < 0) return fail(ERI4_ERROR_INVALID_ARGUMENT, "nquartets must be >= 0");
  if (kmax < 1 || kmax > ERI4_MAX_K)
    return fail(ERI4_ERROR_INVALID_ARGUMENT, "kmax must be in 1..%d (got %d)", ERI4_MAX_K, kmax);
  return ERI4_SUCCESS;
}

eri4_status eri4_solid_coefficients(int l, double* C) {
  g_err.clear();
  if (l < 0 || l > ERI4_MAX_L) return fail(ERI4_ERROR_INVALID_ARGUMENT, "l must be in 0..%d (got %d)", ERI4_MAX_L, l);
  if (!C) return fail(ERI4_ERROR_INVALID_ARGUMENT, "NULL output array");
  solid_dense(l, C);
  return ERI4_SUCCESS;
}

int64_t eri4_solid_work_size(int la, int lb, int lc, int ld, int kmax, int64_t nquartets) {
  if (check_class(la, lb, lc, ld, nquartets, kmax) != ERI4_SUCCESS) return -1;
  ClassParams p;
  int64_t hbs, hks;
  if (!solid_params(la, lb, lc, ld, kmax, nullptr, &p, &hbs, &hks)) return -1;
  return nquartets * kmax * kmax * (hbs + hks);
}

eri4_status eri4_batch_solid(int la, int lb, int lc, int ld, int64_t nquartets, const double* centers,
                             const double* exponents, const double* coeffs, const int32_t* nprim, int kmax,
                             double* work, int64_t work_size, double* out, hipStream_t stream) {
  g_err.clear();
  eri4_status st = check_class(la, lb, lc, ld, nquartets, kmax);
  if (st != ERI4_SUCCESS) return st;
  if (nquartets == 0) return ERI4_SUCCESS;
  if (!centers || !exponents || !coeffs || !nprim || !out || !work)
    return fail(ERI4_ERROR_INVALID_ARGUMENT, "NULL buffer pointer");
  ClassParams p;
  int64_t hbs, hks;
  if (!solid_params(la, lb, lc, ld, kmax, nullptr, &p, &hbs, &hks))
    return fail(ERI4_ERROR_UNSUPPORTED, "class (%d %d|%d %d) does not fit in LDS", la, lb, lc, ld);
  // quartets per pass: what the workspace holds (H of every primitive pair),
  // within the grid limits
  const int64_t perq = (int64_t)kmax * kmax * (hbs + hks);
  int64_t chunk = work_size / perq;
  if (chunk < 1)
    return fail(ERI4_ERROR_INVALID_ARGUMENT, "workspace of %lld doubles is below one quartet's %lld",
                (long long)work_size, (long long)perq);
  DeviceState* d;
  st = ensure_device(&d);
  if (st != ERI4_SUCCESS) return st;
  (void)solid_params(la, lb, lc, ld, kmax, d, &p, &hbs, &hks);  // the same tile, with the device's table offsets
  chunk = std::min<int64_t>(chunk, std::min<int64_t>(((int64_t)1 << 30) / p.nrt, INT32_MAX));
  double* hbra = work;
  for (int64_t q0 = 0; q0 < nquartets; q0 += chunk) {
    const int64_t nq = std::min(chunk, nquartets - q0);
    double* hket = hbra + nq * kmax * kmax * hbs;
    hipError_t e = solid_h_launch(p, nq, stream, centers, exponents, coeffs, nprim, d->stab, hbra, hket, q0, hbs, hks);
    if (e == hipSuccess)
      e = solid_launch(p, dim3((unsigned)(nq * p.nrt)), stream, Tables{d->boys, d->rtab}, centers, exponents, coeffs,
                       nprim, out, q0, hbra, hket, hbs, hks);
    if (e != hipSuccess) return fail(ERI4_ERROR_HIP, "kernel launch: %s", hipGetErrorString(e));
  }
  return ERI4_SUCCESS;
}

// Parameters and LDS layout of the Coulomb (J-engine) kernels: the R box of
// the first layout that fits (two boxes up to L = kBox2LMax, one box up to
// kBoxLMax, else slab), the bra tables, and the w buffer (inside the R box when
// that is large enough: w is written after the last recursion of a bra pair).
// No [ab|q] tile and no ket tables.
bool jengine_params(int la, int lb, int lc, int ld, int kmax, const DeviceState* d, ClassParams* out) {
  const int L = la + lb + lc + ld;
  if (L > kMaxL) return false;
  static const int order[3] = {kLayBox2, kLayBox, kLaySlab};
  for (int lay : order) {
    const bool slab = lay == kLaySlab, two = lay == kLayBox2;
    if ((two && L > kBox2LMax) || (lay == kLayBox && L > kBoxLMax)) continue;
    ClassParams p = make_params(la, lb, lc, ld, kmax, 1, slab, two);
    const int box_b = r_cells(slab, L) * 8;
    p.o_brae = p.o_union + align16(box_b);
    p.o_box1 = p.o_brae + align16(3 * p.tbaxis * 8);
    int end = p.o_box1 + (two ? align16(box_b) : 0);
    if (box_b >= kJw * 8) {
      p.o_jw = p.o_union;
    } else {
      p.o_jw = end;
      end += kJw * 8;
    }
    p.o_kete = p.o_union;  // unused
    p.lds_bytes = end;
    p.nrt = 1;
    if (p.lds_bytes > kMaxLdsBytes - 64) continue;
    p.rtab_off = d ? d->rstart[(slab ? 1 : 0) * (kMaxL + 1) + L] : 0;
    *out = p;
    return true;
  }
  return false;
}

// ds: doubles of one ket primitive pair's dket; ps: of one bra pair's J^ij.
static bool coulomb_params(int la, int lb, int lc, int ld, int kmax, const DeviceState* d, ClassParams* p,
                           int64_t* ds, int64_t* ps) {
  if (!jengine_params(la, lb, lc, ld, kmax, d, p)) return false;
  *ds = 16 * (int64_t)p->nqb;
  *ps = p->nab;
  return true;
}

int64_t eri4_coulomb_work_size(int la, int lb, int lc, int ld, int kmax, int64_t nquartets) {
  if (check_class(la, lb, lc, ld, nquartets, kmax) != ERI4_SUCCESS) return -1;
  ClassParams p;
  int64_t ds, ps;
  if (!coulomb_params(la, lb, lc, ld, kmax, nullptr, &p, &ds, &ps)) return -1;
  return nquartets * kmax * kmax * (ds + ps);
}

// J for nquartets quartets in passes of as many as the workspace (work_size
// doubles) holds the Hermite-space densities and per-bra-pair J of: per pass,
// the density kernel, the J-engine kernel and the sum over bra pairs.
// Arguments already checked; d is initialised.
static eri4_status coulomb_passes(int la, int lb, int lc, int ld, int64_t nquartets, const double* centers,
                                  const double* exponents, const double* coeffs, const int32_t* nprim, int kmax,
                                  const double* dens, double* work, int64_t work_size, double* out,
                                  hipStream_t stream, const DeviceState* d) {
  ClassParams p;
  int64_t ds, ps;
  if (!coulomb_params(la, lb, lc, ld, kmax, d, &p, &ds, &ps))
    return fail(ERI4_ERROR_UNSUPPORTED, "class (%d %d|%d %d) does not fit in LDS", la, lb, lc, ld);
  const int64_t kk2 = (int64_t)kmax * kmax;
  const int64_t perq = kk2 * (ds + ps);
  int64_t chunk = work_size / perq;
  if (chunk < 1)
    return fail(ERI4_ERROR_INVALID_ARGUMENT, "workspace of %lld doubles is below one quartet's %lld",
                (long long)work_size, (long long)perq);
  chunk = std::min<int64_t>(chunk, ((int64_t)1 << 22) / kk2);  // grid of chunk * kmax^2 workgroups
  for (int64_t q0 = 0; q0 < nquartets; q0 += chunk) {
    const int64_t nq = std::min(chunk, nquartets - q0);
    double* part = work + nq * kk2 * ds;
    hipError_t e = coulomb_dket_launch(p, nq, stream, centers, exponents, coeffs, nprim, dens, work, q0, ds);
    if (e == hipSuccess)
      e = coulomb_launch(p, nq, stream, Tables{d->boys, d->rtab}, centers, exponents, coeffs, nprim, part, out, q0,
                         work, ds);
    if (e != hipSuccess) return fail(ERI4_ERROR_HIP, "kernel launch: %s", hipGetErrorString(e));
  }
  return ERI4_SUCCESS;
}

eri4_status eri4_batch_coulomb(int la, int lb, int lc, int ld, int64_t nquartets, const double* centers,
                               const double* exponents, const double* coeffs, const int32_t* nprim, int kmax,
                               const double* dens, double* work, int64_t work_size, double* out, hipStream_t stream) {
  g_err.clear();
  eri4_status st = check_class(la, lb, lc, ld, nquartets, kmax);
  if (st != ERI4_SUCCESS) return st;
  if (nquartets == 0) return ERI4_SUCCESS;
  if (!centers || !exponents || !coeffs || !nprim || !dens || !out || !work)
    return fail(ERI4_ERROR_INVALID_ARGUMENT, "NULL buffer pointer");
  ClassParams p;
  int64_t ds, ps;
  if (!coulomb_params(la, lb, lc, ld, kmax, nullptr, &p, &ds, &ps))
    return fail(ERI4_ERROR_UNSUPPORTED, "class (%d %d|%d %d) does not fit in LDS", la, lb, lc, ld);
  if (work_size < (int64_t)kmax * kmax * (ds + ps))
    return fail(ERI4_ERROR_INVALID_ARGUMENT, "workspace of %lld doubles is below one quartet's %lld",
                (long long)work_size, (long long)kmax * kmax * (ds + ps));
  DeviceState* d;
  st = ensure_device(&d);
  if (st != ERI4_SUCCESS) return st;
  return coulomb_passes(la, lb, lc, ld, nquartets, centers, exponents, coeffs, nprim, kmax, dens, work, work_size,
                        out, stream, d);
}

// Exchange contraction: the library's tile for the class, with the bra rows
// ordered (b, a) and a padded to whole 16-row blocks (one b per block); fbs
// doubles of F^b per ket primitive pair and b, ps doubles of partial rows
// y^b per quartet.
static bool exchange_params(int la, int lb, int lc, int ld, int kmax, const DeviceState* d, ClassParams* p,
                            int64_t* fbs, int64_t* ps) {
  if (!pick_params(la, lb, lc, ld, kmax, d, kMaxLdsBytes, p)) return false;
  const int blocks = p->nb * ((p->na + 15) / 16);
  p->nrt = (blocks + p->rb - 1) / p->rb;
  *fbs = (int64_t)((p->nc + 15) / 16) * 16 * p->nq4;
  *ps = (int64_t)p->nb * p->na * p->nc;
  return true;
}

int64_t eri4_exchange_work_size(int la, int lb, int lc, int ld, int kmax, int64_t nquartets) {
  if (check_class(la, lb, lc, ld, nquartets, kmax) != ERI4_SUCCESS) return -1;
  ClassParams p;
  int64_t fbs, ps;
  if (!exchange_params(la, lb, lc, ld, kmax, nullptr, &p, &fbs, &ps)) return -1;
  return nquartets * ((int64_t)kmax * kmax * p.nb * fbs + ps);
}

eri4_status eri4_batch_exchange(int la, int lb, int lc, int ld, int64_t nquartets, const double* centers,
                                const double* exponents, const double* coeffs, const int32_t* nprim, int kmax,
                                const double* dens, double* work, int64_t work_size, double* out,
                                hipStream_t stream) {
  g_err.clear();
  eri4_status st = check_class(la, lb, lc, ld, nquartets, kmax);
  if (st != ERI4_SUCCESS) return st;
  if (nquartets == 0) return ERI4_SUCCESS;
  if (!centers || !exponents || !coeffs || !nprim || !dens || !out || !work)
    return fail(ERI4_ERROR_INVALID_ARGUMENT, "NULL buffer pointer");
  ClassParams p;
  int64_t fbs, ps;
  if (!exchange_params(la, lb, lc, ld, kmax, nullptr, &p, &fbs, &ps))
    return fail(ERI4_ERROR_UNSUPPORTED, "class (%d %d|%d %d) does not fit in LDS", la, lb, lc, ld);
  const int64_t perq = (int64_t)kmax * kmax * p.nb * fbs + ps;
  int64_t chunk = work_size / perq;
  if (chunk < 1)
    return fail(ERI4_ERROR_INVALID_ARGUMENT, "workspace of %lld doubles is below one quartet's %lld",
                (long long)work_size, (long long)perq);
  DeviceState* d;
  st = ensure_device(&d);
  if (st != ERI4_SUCCESS) return st;
  (void)exchange_params(la, lb, lc, ld, kmax, d, &p, &fbs, &ps);
  chunk = std::min<int64_t>(chunk, std::min<int64_t>(((int64_t)1 << 30) / p.nrt, INT32_MAX));
  for (int64_t q0 = 0; q0 < nquartets; q0 += chunk) {
    const int64_t nq = std::min(chunk, nquartets - q0);
    double* fb = work;
    double* part = work + nq * (int64_t)kmax * kmax * p.nb * fbs;
    const hipError_t e = exchange_launch(p, nq, stream, Tables{d->boys, d->rtab}, centers, exponents, coeffs, nprim,
                                         dens, fb, fbs, part, out, q0);
    if (e != hipSuccess) return fail(ERI4_ERROR_HIP, "kernel launch: %s", hipGetErrorString(e));
  }
  return ERI4_SUCCESS;
}

int64_t eri4_static_scratch_bytes(void) { return kStaticScratchDoubles * (int64_t)sizeof(double); }

eri4_status eri4_batch_coulomb_static(int la, int lb, int lc, int ld, int64_t nquartets, const double* centers,
                                      const double* exponents, const double* coeffs, const int32_t* nprim, int kmax,
                                      const double* dens, double* out, hipStream_t stream) {
  g_err.clear();
  eri4_status st = check_class(la, lb, lc, ld, nquartets, kmax);
  if (st != ERI4_SUCCESS) return st;
  if (nquartets == 0) return ERI4_SUCCESS;
  if (!centers || !exponents || !coeffs || !nprim || !dens || !out)
    return fail(ERI4_ERROR_INVALID_ARGUMENT, "NULL buffer pointer");
  ClassParams p;
  int64_t ds, ps;
  if (!coulomb_params(la, lb, lc, ld, kmax, nullptr, &p, &ds, &ps))
    return fail(ERI4_ERROR_UNSUPPORTED, "class (%d %d|%d %d) does not fit in LDS", la, lb, lc, ld);
  if ((int64_t)kmax * kmax * (ds + ps) > kStaticScratchDoubles)
    return fail(ERI4_ERROR_UNSUPPORTED, "one quartet's Hermite-space densities and partial J (%lld doubles) exceed "
                "the %lld-double static scratch", (long long)kmax * kmax * (ds + ps),
                (long long)kStaticScratchDoubles);
  // no initialisation here: that allocates the tables (eri4_init must have run)
  int dev = 0;
  HIP_TRY(hipGetDevice(&dev));
  const DeviceState* d = nullptr;
  {
    std::lock_guard<std::mutex> lk(g_mu);
    if (dev < (int)g_dev.size() && g_dev[dev].ready) d = &g_dev[dev];
  }
  if (!d)
    return fail(ERI4_ERROR_INVALID_ARGUMENT, "the library is not initialised on device %d: call eri4_init there "
                "first (it allocates; this call does not)", dev);
  return coulomb_passes(la, lb, lc, ld, nquartets, centers, exponents, coeffs, nprim, kmax, dens, d->scratch,
                        kStaticScratchDoubles, out, stream, d);
}

// ---------------------------------------------------------------------------
// plans: many classes and contraction lengths in one persistent launch
// ---------------------------------------------------------------------------

struct eri4_plan_s {
  int device = 0;
  int64_t nq = 0;
  int kmax = 1;
  int nitems = 0;
  int nclasses = 0;
  int lds_bytes = 0;
  int grid = 0;
  bool f32 = false;  // ERI4_PREC_FP32
  bool pairs = false;  // made from a bra and a ket list of shell pairs
  int64_t nbra = 0, nket = 0;
  bool solid = false;  // solid-harmonic output
  int64_t work = 0;    // doubles of caller workspace for the H matrices
  int64_t nentries = 0;      // solid plans: list entries whose H is built (2 per quartet for quartet plans)
  int hlds = 0;              // solid plans: dynamic LDS of the H builder (its largest entry)
  int32_t* d_pl = nullptr;   // per list entry: l of its two shells (bra entries first)
  int32_t* d_pn = nullptr;   // per list entry: contraction lengths
  int64_t* d_hoff = nullptr; // per list entry: where its H matrices start in the workspace
  bool coul = false;         // Coulomb contraction over the lists (eri4_plan_create_coulomb)
  int64_t dket_size = 0;     // doubles of the workspace holding the ket entries' dket
  int64_t ket_dens_size = 0; // doubles of ket_dens (all ket entries' blocks)
  std::vector<int64_t> ooff; // output offsets per bra entry (Coulomb plans)
  int64_t* d_doff = nullptr;   // per ket entry: its density block in ket_dens
  int64_t* d_dkoff = nullptr;  // per ket entry: its dket in the workspace
  int64_t* d_joff = nullptr;   // per bra entry: its J block in out
  int64_t out_size = 0;
  std::vector<int64_t> qoff;
  ClassParams* d_classes = nullptr;
  int2* d_items = nullptr;
  int64_t* d_qoff = nullptr;
  int32_t* d_nprim = nullptr;
  int* d_counter = nullptr;
};

static void plan_free(eri4_plan_s* p) {
  if (!p) return;
  if (p->d_classes) (void)hipFree(p->d_classes);
  if (p->d_items) (void)hipFree(p->d_items);
  if (p->d_qoff) (void)hipFree(p->d_qoff);
  if (p->d_nprim) (void)hipFree(p->d_nprim);
  if (p->d_counter) (void)hipFree(p->d_counter);
  if (p->d_pl) (void)hipFree(p->d_pl);
  if (p->d_pn) (void)hipFree(p->d_pn);
  if (p->d_hoff) (void)hipFree(p->d_hoff);
  if (p->d_doff) (void)hipFree(p->d_doff);
  if (p->d_dkoff) (void)hipFree(p->d_dkoff);
  if (p->d_joff) (void)hipFree(p->d_joff);
  delete p;
}

eri4_status eri4_plan_create(eri4_plan* plan, int64_t nquartets, const int32_t* l, const int32_t* nprim, int kmax,
                             eri4_precision precision) {
  return eri4_plan_create_tuned(plan, nquartets, l, nprim, kmax, precision, nullptr, 0);
}

static_assert(ERI4_LAYOUT_BOX == kLayBox && ERI4_LAYOUT_SLAB == kLaySlab && ERI4_LAYOUT_BOX2 == kLayBox2,
              "public and internal layout codes agree");

// Plan over quartets given by l / nprim; pairs: the shells will come from a
// bra and a ket list (quartet q = bra pair q / nket with ket pair q % nket).
static eri4_status plan_create(eri4_plan* plan, int64_t nquartets, const int32_t* l, const int32_t* nprim, int kmax,
                               eri4_precision precision, const eri4_tile_choice* choices, int nchoices, bool pairs,
                               int64_t nbra, int64_t nket, bool solid, bool coul = false) {
  if (!plan) return fail(ERI4_ERROR_INVALID_ARGUMENT, "NULL plan pointer");
  *plan = nullptr;
  if (precision != ERI4_PREC_FP64 && precision != ERI4_PREC_FP32)
    return fail(ERI4_ERROR_INVALID_ARGUMENT, "unknown precision %d", (int)precision);
  if (nquartets < 0 || nquartets > ((int64_t)1 << 31) - 1)
    return fail(ERI4_ERROR_INVALID_ARGUMENT, "nquartets must be in 0..2^31-1");
  if (kmax < 1 || kmax > ERI4_MAX_K)
    return fail(ERI4_ERROR_INVALID_ARGUMENT, "kmax must be in 1..%d (got %d)", ERI4_MAX_K, kmax);
  if (nquartets > 0 && (!l || !nprim)) return fail(ERI4_ERROR_INVALID_ARGUMENT, "NULL host array");
  for (int64_t i = 0; i < 4 * nquartets; ++i) {
    if (l[i] < 0) return fail(ERI4_ERROR_INVALID_ARGUMENT, "negative angular momentum at quartet %lld", (long long)(i / 4));
    if (l[i] > ERI4_MAX_L)
      return fail(ERI4_ERROR_UNSUPPORTED, "angular momentum %d above %d at quartet %lld", l[i], ERI4_MAX_L,
                  (long long)(i / 4));
    if (nprim[i] < 1 || nprim[i] > kmax)
      return fail(ERI4_ERROR_INVALID_ARGUMENT, "contraction length %d outside 1..%d at quartet %lld", nprim[i], kmax,
                  (long long)(i / 4));
  }
  if (nchoices < 0 || (nchoices > 0 && !choices))
    return fail(ERI4_ERROR_INVALID_ARGUMENT, "tile choices: NULL array or negative count");
  // entries of the choice table per class, in table order
  std::vector<std::vector<int>> choices_of(8 * 8 * 8 * 8);
  for (int i = 0; i < nchoices; ++i) {
    const eri4_tile_choice& c = choices[i];
    if (c.rows16 != 1 && c.rows16 != 2 && c.rows16 != 4)
      return fail(ERI4_ERROR_INVALID_ARGUMENT, "tile choice %d: rows16 must be 1, 2 or 4 (got %d)", i, c.rows16);
    if (c.layout < ERI4_LAYOUT_BOX || c.layout > ERI4_LAYOUT_BOX2)
      return fail(ERI4_ERROR_INVALID_ARGUMENT, "tile choice %d: unknown layout %d", i, c.layout);
    if (c.kq_min > c.kq_max)
      return fail(ERI4_ERROR_INVALID_ARGUMENT, "tile choice %d: kq_min %d above kq_max %d", i, c.kq_min, c.kq_max);
    for (int x = 0; x < 4; ++x)
      if (c.l[x] < 0 || c.l[x] > ERI4_MAX_L)
        return fail(ERI4_ERROR_INVALID_ARGUMENT, "tile choice %d: angular momentum %d out of range", i, c.l[x]);
    choices_of[((c.l[0] * 8 + c.l[1]) * 8 + c.l[2]) * 8 + c.l[3]].push_back(i);
  }
  int device = 0;
  HIP_TRY(hipGetDevice(&device));
  DeviceState* d;
  eri4_status st = ensure_device(&d);
  if (st != ERI4_SUCCESS) return st;
  eri4_plan_s* p = new (std::nothrow) eri4_plan_s();
  if (!p) return fail(ERI4_ERROR_OUT_OF_MEMORY, "host allocation failed");
  p->device = device;
  p->nq = nquartets;
  p->kmax = kmax;
  p->f32 = precision == ERI4_PREC_FP32;
  p->pairs = pairs;
  p->nbra = nbra;
  p->nket = nket;
  p->solid = solid;
  p->coul = coul;
  // dynamic LDS available next to the persistent kernel's static LDS
  const int limit = kMaxLdsBytes - 64;

  // groups of quartets with the same class and tile choice (the first matching
  // entry of the table, or none), keyed by class * (nchoices + 1) + entry + 1
  std::map<int64_t, int> group_of;
  std::vector<int> qcls(nquartets);
  std::vector<std::array<int, 5>> keys;  // la, lb, lc, ld, entry (-1: none)
  for (int64_t q = 0; q < nquartets; ++q) {
    const int key = ((l[4 * q] * 8 + l[4 * q + 1]) * 8 + l[4 * q + 2]) * 8 + l[4 * q + 3];
    const int64_t kq = (int64_t)nprim[4 * q] * nprim[4 * q + 1] * nprim[4 * q + 2] * nprim[4 * q + 3];
    int entry = -1;
    for (int i : choices_of[key])
      if (kq >= choices[i].kq_min && kq <= choices[i].kq_max) {
        entry = i;
        break;
      }
    const int64_t gkey = (int64_t)key * (nchoices + 1) + entry + 1;
    auto it = group_of.find(gkey);
    if (it == group_of.end()) {
      it = group_of.emplace(gkey, (int)keys.size()).first;
      keys.push_back({l[4 * q], l[4 * q + 1], l[4 * q + 2], l[4 * q + 3], entry});
    }
    qcls[q] = it->second;
  }
  if (keys.size() > 32767) {
    plan_free(p);
    return fail(ERI4_ERROR_INVALID_ARGUMENT, "too many (class, tile choice) groups");
  }
  // per group: tile height and R layout (the table's, or see pick_params)
  std::vector<ClassParams> cps(keys.size());
  for (size_t c = 0; c < keys.size(); ++c) {
    const auto& k = keys[c];
    if (coul) {
      if (!jengine_params(k[0], k[1], k[2], k[3], kmax, d, &cps[c])) {
        plan_free(p);
        return fail(ERI4_ERROR_UNSUPPORTED, "class (%d %d|%d %d) does not fit in LDS", k[0], k[1], k[2], k[3]);
      }
    } else if (k[4] >= 0) {
      const eri4_tile_choice& ch = choices[k[4]];
      if (!try_params(k[0], k[1], k[2], k[3], kmax, ch.rows16, ch.layout, d, limit, &cps[c])) {
        plan_free(p);
        return fail(ERI4_ERROR_INVALID_ARGUMENT, "tile choice %d (rows16 %d, layout %d) does not fit class (%d %d|%d %d)",
                    k[4], ch.rows16, ch.layout, k[0], k[1], k[2], k[3]);
      }
    } else if (!pick_params(k[0], k[1], k[2], k[3], kmax, d, limit, &cps[c])) {
      plan_free(p);
      return fail(ERI4_ERROR_UNSUPPORTED, "class (%d %d|%d %d) does not fit in LDS", k[0], k[1], k[2], k[3]);
    }
  }
  if (solid)
    for (ClassParams& c : cps) to_solid(&c);  // rows and columns over solid functions; same tile and LDS
  p->nclasses = (int)keys.size();
  for (const ClassParams& c : cps) p->lds_bytes = std::max(p->lds_bytes, c.lds_bytes);

  // output offsets in input order, and work items with their cost
  p->qoff.resize(nquartets);
  int64_t off = 0;
  std::vector<int2> items;
  std::vector<double> cost;
  for (int64_t q = 0; q < nquartets; ++q) {
    const ClassParams& c = cps[qcls[q]];
    p->qoff[q] = off;
    off += coul ? (int64_t)c.nab : (int64_t)c.nab * c.ncd;  // Coulomb plans: J rows per quartet
    const double kb = (double)nprim[4 * q] * nprim[4 * q + 1], kk = (double)nprim[4 * q + 2] * nprim[4 * q + 3];
    if (coul) {
      // one item per quartet (J-engine): per primitive quartet the recursion
      // and the matrix-vector product, per bra pair the bra transform
      cost.push_back(kb * kk * (8000.0 + 4.0 * nherm(c.L) + (double)c.np * c.nq / 128.0) +
                     kb * (double)c.nab * c.np / 256.0 + 4000.0);
      items.push_back(make_int2((int)q, qcls[q] << 16));
      continue;
    }
    for (int rt = 0; rt < c.nrt; ++rt) {
      const int rows = 16 * std::min(c.rb, (c.nab - rt * c.rb * 16 + 15) / 16);
      // MFMA cycles of the two transforms at 128 FLOP/clk per CU, plus a
      // latency-bound estimate for Boys and the recursion per primitive quartet
      const double g1 = 2.0 * rows * c.np4 * 16.0 * c.nqb * kb * kk;
      const double g2 = 2.0 * rows * c.nq4 * 16.0 * c.ncdb * kk;
      cost.push_back((g1 + g2) / 128.0 + kb * kk * (8000.0 + 4.0 * nherm(c.L)) + 4000.0);
      items.push_back(make_int2((int)q, rt | (qcls[q] << 16)));
    }
  }
  p->out_size = off;
  std::vector<int> order(items.size());
  std::iota(order.begin(), order.end(), 0);
  std::stable_sort(order.begin(), order.end(), [&](int a, int b) { return cost[a] > cost[b]; });
  std::vector<int2> sorted(items.size());
  for (size_t i = 0; i < order.size(); ++i) sorted[i] = items[order[i]];
  if (sorted.size() > (size_t)INT32_MAX) {
    plan_free(p);
    return fail(ERI4_ERROR_INVALID_ARGUMENT, "too many work items");
  }
  p->nitems = (int)sorted.size();

  int ncu = 0, per_cu = 0;
  HIP_TRY(hipDeviceGetAttribute(&ncu, hipDeviceAttributeMultiprocessorCount, p->device));
  const hipError_t oe = p->coul ? plan_coulomb_occupancy(p->lds_bytes, &per_cu)
                        : p->solid ? plan_solid_occupancy(p->pairs, p->lds_bytes, &per_cu)
                        : p->pairs ? (p->f32 ? plan_occupancy_f32p(p->lds_bytes, &per_cu)
                                           : plan_occupancy_f64p(p->lds_bytes, &per_cu))
                                 : (p->f32 ? plan_occupancy_f32(p->lds_bytes, &per_cu)
                                           : plan_occupancy_f64(p->lds_bytes, &per_cu));
  if (oe != hipSuccess || per_cu < 1) per_cu = 1;
  p->grid = (int)std::min<int64_t>(std::max(p->nitems, 1), (int64_t)ncu * per_cu);

  const bool ok = hipMalloc(&p->d_classes, std::max<size_t>(1, cps.size()) * sizeof(ClassParams)) == hipSuccess &&
                  hipMalloc(&p->d_items, std::max<size_t>(1, sorted.size()) * sizeof(int2)) == hipSuccess &&
                  hipMalloc(&p->d_qoff, std::max<int64_t>(1, nquartets) * sizeof(int64_t)) == hipSuccess &&
                  hipMalloc(&p->d_nprim, std::max<int64_t>(1, 4 * nquartets) * sizeof(int32_t)) == hipSuccess &&
                  hipMalloc(&p->d_counter, 64) == hipSuccess;
  if (!ok) {
    plan_free(p);
    return fail(ERI4_ERROR_OUT_OF_MEMORY, "device allocation for the plan failed");
  }
  hipError_t e = hipSuccess;
  if (!cps.empty()) e = hipMemcpy(p->d_classes, cps.data(), cps.size() * sizeof(ClassParams), hipMemcpyHostToDevice);
  if (e == hipSuccess && !sorted.empty())
    e = hipMemcpy(p->d_items, sorted.data(), sorted.size() * sizeof(int2), hipMemcpyHostToDevice);
  if (e == hipSuccess && nquartets > 0)
    e = hipMemcpy(p->d_qoff, p->qoff.data(), nquartets * sizeof(int64_t), hipMemcpyHostToDevice);
  if (e == hipSuccess && nquartets > 0)
    e = hipMemcpy(p->d_nprim, nprim, 4 * nquartets * sizeof(int32_t), hipMemcpyHostToDevice);
  if (e != hipSuccess) {
    plan_free(p);
    return fail(ERI4_ERROR_HIP, "plan upload: %s", hipGetErrorString(e));
  }
  *plan = p;
  return ERI4_SUCCESS;
}

eri4_status eri4_plan_create_tuned(eri4_plan* plan, int64_t nquartets, const int32_t* l, const int32_t* nprim,
                                   int kmax, eri4_precision precision, const eri4_tile_choice* choices,
                                   int nchoices) {
  g_err.clear();
  return plan_create(plan, nquartets, l, nprim, kmax, precision, choices, nchoices, false, 0, 0, false);
}

// Tile table file (format in eri4.h) -> choices; checks the arch line against
// the current device.
static eri4_status read_tile_table(const char* path, std::vector<eri4_tile_choice>* out) {
  FILE* f = std::fopen(path, "r");
  if (!f) return fail(ERI4_ERROR_INVALID_ARGUMENT, "tile table %s: cannot open it", path);
  int dev = 0;
  hipDeviceProp_t prop;
  if (hipGetDevice(&dev) != hipSuccess || hipGetDeviceProperties(&prop, dev) != hipSuccess) {
    std::fclose(f);
    return fail(ERI4_ERROR_HIP, "tile table %s: no device properties", path);
  }
  std::string devarch(prop.gcnArchName);
  devarch = devarch.substr(0, devarch.find(':'));
  char line[512];
  int lineno = 0;
  bool have_arch = false;
  eri4_status st = ERI4_SUCCESS;
  while (st == ERI4_SUCCESS && std::fgets(line, sizeof line, f)) {
    ++lineno;
    char* p = line;
    while (*p == ' ' || *p == '\t') ++p;
    if (*p == '#' || *p == '\n' || *p == '\r' || *p == 0) continue;
    char word[64];
    if (std::sscanf(p, "arch %63s", word) == 1 && std::strncmp(p, "arch", 4) == 0) {
      if (devarch != word)
        st = fail(ERI4_ERROR_INVALID_ARGUMENT, "tile table %s is for %s, the device is %s", path, word,
                  devarch.c_str());
      have_arch = true;
      continue;
    }
    eri4_tile_choice c{};
    char lay[16];
    int n = 0;
    if (std::sscanf(p, "%d %d %d %d %d %d %d %15s %n", &c.l[0], &c.l[1], &c.l[2], &c.l[3], &c.kq_min, &c.kq_max,
                    &c.rows16, lay, &n) != 8 || p[n] != 0) {
      st = fail(ERI4_ERROR_INVALID_ARGUMENT, "tile table %s line %d: expected 'la lb lc ld kq_min kq_max rows16 "
                "layout'", path, lineno);
      break;
    }
    if (!have_arch) {
      st = fail(ERI4_ERROR_INVALID_ARGUMENT, "tile table %s line %d: entry before the arch line", path, lineno);
      break;
    }
    if (!std::strcmp(lay, "box")) c.layout = ERI4_LAYOUT_BOX;
    else if (!std::strcmp(lay, "slab")) c.layout = ERI4_LAYOUT_SLAB;
    else if (!std::strcmp(lay, "box2")) c.layout = ERI4_LAYOUT_BOX2;
    else {
      st = fail(ERI4_ERROR_INVALID_ARGUMENT, "tile table %s line %d: unknown layout %s", path, lineno, lay);
      break;
    }
    out->push_back(c);
  }
  std::fclose(f);
  if (st == ERI4_SUCCESS && !have_arch) st = fail(ERI4_ERROR_INVALID_ARGUMENT, "tile table %s: no arch line", path);
  return st;
}

eri4_status eri4_plan_create_tunefile(eri4_plan* plan, int64_t nquartets, const int32_t* l, const int32_t* nprim,
                                      int kmax, eri4_precision precision, const char* tune_file) {
  g_err.clear();
  if (!plan) return fail(ERI4_ERROR_INVALID_ARGUMENT, "NULL plan pointer");
  *plan = nullptr;
  std::vector<eri4_tile_choice> choices;
  if (tune_file) {
    const eri4_status st = read_tile_table(tune_file, &choices);
    if (st != ERI4_SUCCESS) return st;
  }
  return plan_create(plan, nquartets, l, nprim, kmax, precision, choices.data(), (int)choices.size(), false, 0, 0,
                     false);
}

int64_t eri4_plan_output_size(eri4_plan plan) { return plan ? plan->out_size : -1; }

eri4_status eri4_plan_output_offsets(eri4_plan plan, int64_t* offsets) {
  g_err.clear();
  if (!plan) return fail(ERI4_ERROR_INVALID_ARGUMENT, "NULL plan");
  const std::vector<int64_t>& o = plan->coul ? plan->ooff : plan->qoff;
  if (!o.empty() && !offsets) return fail(ERI4_ERROR_INVALID_ARGUMENT, "NULL offsets array");
  std::copy(o.begin(), o.end(), offsets);
  return ERI4_SUCCESS;
}

// Enqueue the counter reset and the persistent kernel of a plan.
static eri4_status plan_launch(eri4_plan plan, const Shells& shl, double* work, int64_t work_size, double* out,
                               hipStream_t stream) {
  if (plan->nitems == 0) return ERI4_SUCCESS;
  if (!shl.centers || !shl.exps || !shl.coefs || !out || (plan->pairs && (!shl.kcenters || !shl.kexps || !shl.kcoefs)))
    return fail(ERI4_ERROR_INVALID_ARGUMENT, "NULL buffer pointer");
  if (plan->solid && (!work || work_size < plan->work))
    return fail(ERI4_ERROR_INVALID_ARGUMENT, "workspace of %lld doubles is below the plan's %lld",
                (long long)(work ? work_size : 0), (long long)plan->work);
  int dev = 0;
  HIP_TRY(hipGetDevice(&dev));
  if (dev != plan->device)
    return fail(ERI4_ERROR_INVALID_ARGUMENT, "plan was made for device %d, current device is %d", plan->device, dev);
  DeviceState* d;
  eri4_status st = ensure_device(&d);
  if (st != ERI4_SUCCESS) return st;
  if (plan->solid)
    HIP_TRY(solid_hpairs_launch(plan->pairs ? plan->nbra : -1, plan->nentries, plan->kmax, plan->hlds, stream, plan->d_pl,
                                plan->d_pn, shl, plan->d_hoff, d->stab, work));
  hipLaunchKernelGGL(reset_counter_kernel, dim3(1), dim3(64), 0, stream, plan->d_counter);
  HIP_TRY(hipGetLastError());
  const PlanArgs a{plan->d_classes, plan->d_items, plan->nitems, plan->d_qoff, plan->d_nprim, plan->d_counter, shl,
                   out};
  const Tables t{d->boys, d->rtab};
  const dim3 grid(plan->grid);
  if (plan->solid)
    HIP_TRY(plan_solid_launch(plan->pairs, grid, plan->lds_bytes, stream, t, a, plan->nbra, plan->d_hoff, work));
  else if (plan->pairs)
    HIP_TRY(plan->f32 ? plan_launch_f32p(grid, plan->lds_bytes, stream, t, a)
                      : plan_launch_f64p(grid, plan->lds_bytes, stream, t, a));
  else
    HIP_TRY(plan->f32 ? plan_launch_f32(grid, plan->lds_bytes, stream, t, a)
                      : plan_launch_f64(grid, plan->lds_bytes, stream, t, a));
  return ERI4_SUCCESS;
}

eri4_status eri4_plan_execute(eri4_plan plan, const double* centers, const double* exponents, const double* coeffs,
                              double* out, hipStream_t stream) {
  g_err.clear();
  if (!plan) return fail(ERI4_ERROR_INVALID_ARGUMENT, "NULL plan");
  if (plan->pairs)
    return fail(ERI4_ERROR_INVALID_ARGUMENT, "plan made from pair lists: use eri4_plan_execute_pairs");
  if (plan->solid) return fail(ERI4_ERROR_INVALID_ARGUMENT, "solid-harmonic plan: use eri4_plan_execute_solid");
  return plan_launch(plan, Shells{centers, exponents, coeffs, nullptr, nullptr, nullptr, 0}, nullptr, 0, out, stream);
}

// Workspace layout of a solid plan's H matrices: entry e (l and contraction
// lengths pl[2e..2e+1], pn[2e..2e+1]; a ket pair if e >= nbra, or for nbra < 0
// if e is odd) holds K1 * K2 slots from hoff[e] (solid_hpairs_kernel); uploads
// pl, pn and hoff into the plan and sets its workspace size.  Frees the plan
// and clears *plan on error.
static eri4_status solid_entries(eri4_plan* plan, int64_t ne, int64_t nbra, const int32_t* pl, const int32_t* pn) {
  eri4_plan_s* p = *plan;
  std::vector<int64_t> hoff(ne);
  int64_t off = 0;
  for (int64_t e = 0; e < ne; ++e) {
    hoff[e] = off;
    const int l1 = pl[2 * e], l2 = pl[2 * e + 1];
    const int nk4 = (nherm(l1 + l2) + 3) & ~3;
    off += (int64_t)pn[2 * e] * pn[2 * e + 1] * solid_pair_units(l1, l2, nbra < 0 ? (e & 1) != 0 : e >= nbra) * 16 *
           nk4;
    p->hlds = std::max(p->hlds, solid_h_lds(l1, l2, nk4));
  }
  p->work = off;
  p->nentries = ne;
  const bool ok = hipMalloc(&p->d_pl, std::max<int64_t>(1, 2 * ne) * sizeof(int32_t)) == hipSuccess &&
                  hipMalloc(&p->d_pn, std::max<int64_t>(1, 2 * ne) * sizeof(int32_t)) == hipSuccess &&
                  hipMalloc(&p->d_hoff, std::max<int64_t>(1, ne) * sizeof(int64_t)) == hipSuccess;
  hipError_t e = ok ? hipSuccess : hipErrorOutOfMemory;
  if (e == hipSuccess && ne > 0) e = hipMemcpy(p->d_pl, pl, 2 * ne * sizeof(int32_t), hipMemcpyHostToDevice);
  if (e == hipSuccess && ne > 0) e = hipMemcpy(p->d_pn, pn, 2 * ne * sizeof(int32_t), hipMemcpyHostToDevice);
  if (e == hipSuccess && ne > 0) e = hipMemcpy(p->d_hoff, hoff.data(), ne * sizeof(int64_t), hipMemcpyHostToDevice);
  if (e != hipSuccess) {
    plan_free(p);
    *plan = nullptr;
    return ok ? fail(ERI4_ERROR_HIP, "plan upload: %s", hipGetErrorString(e))
              : fail(ERI4_ERROR_OUT_OF_MEMORY, "device allocation for the plan failed");
  }
  return ERI4_SUCCESS;
}

eri4_status eri4_plan_create_solid(eri4_plan* plan, int64_t nquartets, const int32_t* l, const int32_t* nprim,
                                   int kmax, const char* tune_file) {
  g_err.clear();
  if (!plan) return fail(ERI4_ERROR_INVALID_ARGUMENT, "NULL plan pointer");
  *plan = nullptr;
  std::vector<eri4_tile_choice> choices;
  if (tune_file) {
    const eri4_status st = read_tile_table(tune_file, &choices);
    if (st != ERI4_SUCCESS) return st;
  }
  eri4_status st = plan_create(plan, nquartets, l, nprim, kmax, ERI4_PREC_FP64, choices.data(), (int)choices.size(),
                               false, 0, 0, true);
  if (st != ERI4_SUCCESS) return st;
  // entries 2q (bra pair) and 2q + 1 (ket pair): the quartet arrays as they are
  return solid_entries(plan, 2 * nquartets, -1, l, nprim);
}

eri4_status eri4_plan_execute_solid(eri4_plan plan, const double* centers, const double* exponents,
                                    const double* coeffs, double* work, int64_t work_size, double* out,
                                    hipStream_t stream) {
  g_err.clear();
  if (!plan) return fail(ERI4_ERROR_INVALID_ARGUMENT, "NULL plan");
  if (plan->pairs) return fail(ERI4_ERROR_INVALID_ARGUMENT, "plan made from pair lists: use eri4_plan_execute_pairs");
  if (!plan->solid) return fail(ERI4_ERROR_INVALID_ARGUMENT, "Cartesian plan: use eri4_plan_execute");
  return plan_launch(plan, Shells{centers, exponents, coeffs, nullptr, nullptr, nullptr, 0}, work, work_size, out,
                     stream);
}

eri4_status eri4_plan_create_pairs(eri4_plan* plan, int64_t nbra, const int32_t* bra_l, const int32_t* bra_nprim,
                                   int64_t nket, const int32_t* ket_l, const int32_t* ket_nprim, int kmax,
                                   eri4_precision precision, eri4_functions functions,
                                   const eri4_tile_choice* choices, int nchoices) {
  g_err.clear();
  if (!plan) return fail(ERI4_ERROR_INVALID_ARGUMENT, "NULL plan pointer");
  *plan = nullptr;
  if (functions != ERI4_CARTESIAN && functions != ERI4_SOLID)
    return fail(ERI4_ERROR_INVALID_ARGUMENT, "unknown functions %d", (int)functions);
  const bool solid = functions == ERI4_SOLID;
  if (solid && precision != ERI4_PREC_FP64)
    return fail(ERI4_ERROR_INVALID_ARGUMENT, "solid-harmonic output runs FP64 transforms only");
  if (nbra < 0 || nket < 0) return fail(ERI4_ERROR_INVALID_ARGUMENT, "negative list length");
  if (nbra > 0 && nket > (((int64_t)1 << 31) - 1) / nbra)
    return fail(ERI4_ERROR_INVALID_ARGUMENT, "nbra * nket must be below 2^31");
  if ((nbra > 0 && (!bra_l || !bra_nprim)) || (nket > 0 && (!ket_l || !ket_nprim)))
    return fail(ERI4_ERROR_INVALID_ARGUMENT, "NULL host array");
  // quartet (i, j) = bra pair i with ket pair j, at q = i * nket + j
  const int64_t nq = nbra * nket;
  std::vector<int32_t> l(4 * nq), np(4 * nq);
  for (int64_t i = 0; i < nbra; ++i)
    for (int64_t j = 0; j < nket; ++j) {
      const int64_t q = i * nket + j;
      l[4 * q] = bra_l[2 * i], l[4 * q + 1] = bra_l[2 * i + 1];
      l[4 * q + 2] = ket_l[2 * j], l[4 * q + 3] = ket_l[2 * j + 1];
      np[4 * q] = bra_nprim[2 * i], np[4 * q + 1] = bra_nprim[2 * i + 1];
      np[4 * q + 2] = ket_nprim[2 * j], np[4 * q + 3] = ket_nprim[2 * j + 1];
    }
  eri4_status st = plan_create(plan, nq, l.data(), np.data(), kmax, precision, choices, nchoices, true, nbra, nket, solid);
  if (st != ERI4_SUCCESS || !solid) return st;
  // H matrices of every list entry, bra entries first
  const int64_t ne = nbra + nket;
  std::vector<int32_t> pl(2 * ne), pn(2 * ne);
  for (int64_t e = 0; e < ne; ++e) {
    const bool ket = e >= nbra;
    const int64_t i = ket ? e - nbra : e;
    const int32_t* lsrc = ket ? ket_l : bra_l;
    const int32_t* nsrc = ket ? ket_nprim : bra_nprim;
    pl[2 * e] = lsrc[2 * i], pl[2 * e + 1] = lsrc[2 * i + 1];
    pn[2 * e] = nsrc[2 * i], pn[2 * e + 1] = nsrc[2 * i + 1];
  }
  return solid_entries(plan, ne, nbra, pl.data(), pn.data());
}

int64_t eri4_plan_work_size(eri4_plan plan) { return plan ? plan->work : -1; }

eri4_status eri4_plan_create_coulomb(eri4_plan* plan, int64_t nbra, const int32_t* bra_l, const int32_t* bra_nprim,
                                     int64_t nket, const int32_t* ket_l, const int32_t* ket_nprim, int kmax) {
  g_err.clear();
  if (!plan) return fail(ERI4_ERROR_INVALID_ARGUMENT, "NULL plan pointer");
  *plan = nullptr;
  if (nbra < 0 || nket < 0) return fail(ERI4_ERROR_INVALID_ARGUMENT, "negative list length");
  if (nbra > 0 && nket > (((int64_t)1 << 31) - 1) / nbra)
    return fail(ERI4_ERROR_INVALID_ARGUMENT, "nbra * nket must be below 2^31");
  if ((nbra > 0 && (!bra_l || !bra_nprim)) || (nket > 0 && (!ket_l || !ket_nprim)))
    return fail(ERI4_ERROR_INVALID_ARGUMENT, "NULL host array");
  const int64_t nq = nbra * nket;
  std::vector<int32_t> l(4 * nq), np(4 * nq);
  for (int64_t i = 0; i < nbra; ++i)
    for (int64_t j = 0; j < nket; ++j) {
      const int64_t q = i * nket + j;
      l[4 * q] = bra_l[2 * i], l[4 * q + 1] = bra_l[2 * i + 1];
      l[4 * q + 2] = ket_l[2 * j], l[4 * q + 3] = ket_l[2 * j + 1];
      np[4 * q] = bra_nprim[2 * i], np[4 * q + 1] = bra_nprim[2 * i + 1];
      np[4 * q + 2] = ket_nprim[2 * j], np[4 * q + 3] = ket_nprim[2 * j + 1];
    }
  eri4_status st = plan_create(plan, nq, l.data(), np.data(), kmax, ERI4_PREC_FP64, nullptr, 0, true, nbra, nket,
                               false, true);
  if (st != ERI4_SUCCESS) return st;
  eri4_plan_s* p = *plan;
  // workspace: dket of every ket entry (kmax^2 slots), then the quartets' J rows
  const int64_t ne = nbra + nket;
  std::vector<int32_t> pl(2 * ne), pn(2 * ne);
  std::vector<int64_t> doff(std::max<int64_t>(1, nket)), dkoff(std::max<int64_t>(1, nket)), joff(nbra);
  for (int64_t e = 0; e < ne; ++e) {
    const bool ket = e >= nbra;
    const int64_t i = ket ? e - nbra : e;
    pl[2 * e] = (ket ? ket_l : bra_l)[2 * i], pl[2 * e + 1] = (ket ? ket_l : bra_l)[2 * i + 1];
    pn[2 * e] = (ket ? ket_nprim : bra_nprim)[2 * i], pn[2 * e + 1] = (ket ? ket_nprim : bra_nprim)[2 * i + 1];
  }
  int64_t od = 0, ok_ = 0, oj = 0;
  for (int64_t j = 0; j < nket; ++j) {
    const int lc = ket_l[2 * j], ld = ket_l[2 * j + 1];
    doff[j] = od;
    od += (int64_t)ncart(lc) * ncart(ld);
    dkoff[j] = ok_;
    ok_ += (int64_t)kmax * kmax * 16 * ((nherm(lc + ld) + 15) / 16);
  }
  for (int64_t i = 0; i < nbra; ++i) {
    joff[i] = oj;
    oj += (int64_t)ncart(bra_l[2 * i]) * ncart(bra_l[2 * i + 1]);
  }
  p->dket_size = ok_;
  p->work = ok_ + p->out_size;  // out_size so far: the quartets' J rows
  p->out_size = oj;
  p->ooff = joff;
  p->ket_dens_size = od;
  const bool ok = hipMalloc(&p->d_pl, std::max<int64_t>(1, 2 * ne) * sizeof(int32_t)) == hipSuccess &&
                  hipMalloc(&p->d_pn, std::max<int64_t>(1, 2 * ne) * sizeof(int32_t)) == hipSuccess &&
                  hipMalloc(&p->d_doff, doff.size() * sizeof(int64_t)) == hipSuccess &&
                  hipMalloc(&p->d_dkoff, dkoff.size() * sizeof(int64_t)) == hipSuccess &&
                  hipMalloc(&p->d_joff, std::max<int64_t>(1, nbra) * sizeof(int64_t)) == hipSuccess;
  hipError_t e = ok ? hipSuccess : hipErrorOutOfMemory;
  if (e == hipSuccess && ne > 0) e = hipMemcpy(p->d_pl, pl.data(), 2 * ne * sizeof(int32_t), hipMemcpyHostToDevice);
  if (e == hipSuccess && ne > 0) e = hipMemcpy(p->d_pn, pn.data(), 2 * ne * sizeof(int32_t), hipMemcpyHostToDevice);
  if (e == hipSuccess) e = hipMemcpy(p->d_doff, doff.data(), doff.size() * sizeof(int64_t), hipMemcpyHostToDevice);
  if (e == hipSuccess) e = hipMemcpy(p->d_dkoff, dkoff.data(), dkoff.size() * sizeof(int64_t), hipMemcpyHostToDevice);
  if (e == hipSuccess && nbra > 0) e = hipMemcpy(p->d_joff, joff.data(), nbra * sizeof(int64_t), hipMemcpyHostToDevice);
  if (e != hipSuccess) {
    plan_free(p);
    *plan = nullptr;
    return ok ? fail(ERI4_ERROR_HIP, "plan upload: %s", hipGetErrorString(e))
              : fail(ERI4_ERROR_OUT_OF_MEMORY, "device allocation for the plan failed");
  }
  return ERI4_SUCCESS;
}

eri4_status eri4_plan_execute_coulomb(eri4_plan plan, const double* bra_centers, const double* bra_exponents,
                                      const double* bra_coeffs, const double* ket_centers,
                                      const double* ket_exponents, const double* ket_coeffs, const double* ket_dens,
                                      double* work, int64_t work_size, double* out, hipStream_t stream) {
  g_err.clear();
  if (!plan) return fail(ERI4_ERROR_INVALID_ARGUMENT, "NULL plan");
  if (!plan->coul) return fail(ERI4_ERROR_INVALID_ARGUMENT, "not a Coulomb plan (eri4_plan_create_coulomb)");
  if (plan->nitems == 0) {
    // an empty ket list: every J_i is an empty sum
    if (plan->out_size == 0) return ERI4_SUCCESS;
    if (!out) return fail(ERI4_ERROR_INVALID_ARGUMENT, "NULL buffer pointer");
    const int64_t nb = std::min<int64_t>((plan->out_size + 255) / 256, 4096);
    hipLaunchKernelGGL(zero_fill_kernel, dim3((unsigned)nb), dim3(256), 0, stream, out, plan->out_size);
    HIP_TRY(hipGetLastError());
    return ERI4_SUCCESS;
  }
  if (!bra_centers || !bra_exponents || !bra_coeffs || !ket_centers || !ket_exponents || !ket_coeffs || !ket_dens ||
      !out)
    return fail(ERI4_ERROR_INVALID_ARGUMENT, "NULL buffer pointer");
  if (!work || work_size < plan->work)
    return fail(ERI4_ERROR_INVALID_ARGUMENT, "workspace of %lld doubles is below the plan's %lld",
                (long long)(work ? work_size : 0), (long long)plan->work);
  int dev = 0;
  HIP_TRY(hipGetDevice(&dev));
  if (dev != plan->device)
    return fail(ERI4_ERROR_INVALID_ARGUMENT, "plan was made for device %d, current device is %d", plan->device, dev);
  DeviceState* d;
  eri4_status st = ensure_device(&d);
  if (st != ERI4_SUCCESS) return st;
  hipLaunchKernelGGL(reset_counter_kernel, dim3(1), dim3(64), 0, stream, plan->d_counter);
  HIP_TRY(hipGetLastError());
  const Shells shl{bra_centers, bra_exponents, bra_coeffs, ket_centers, ket_exponents, ket_coeffs, plan->nket};
  const PlanArgs a{plan->d_classes, plan->d_items, plan->nitems, plan->d_qoff, plan->d_nprim, plan->d_counter, shl,
                   nullptr};
  HIP_TRY(plan_coulomb_launch(dim3(plan->grid), plan->lds_bytes, stream, Tables{d->boys, d->rtab}, a,
                              (int)plan->nbra, plan->kmax, plan->d_pl, plan->d_pn, ket_dens, plan->d_doff,
                              plan->d_dkoff, plan->d_joff, work, work + plan->dket_size, out));
  return ERI4_SUCCESS;
}

eri4_status eri4_plan_execute_pairs(eri4_plan plan, const double* bra_centers, const double* bra_exponents,
                                    const double* bra_coeffs, const double* ket_centers,
                                    const double* ket_exponents, const double* ket_coeffs, double* work,
                                    int64_t work_size, double* out, hipStream_t stream) {
  g_err.clear();
  if (!plan) return fail(ERI4_ERROR_INVALID_ARGUMENT, "NULL plan");
  if (!plan->pairs) return fail(ERI4_ERROR_INVALID_ARGUMENT, "plan made from quartets: use eri4_plan_execute");
  if (plan->coul) return fail(ERI4_ERROR_INVALID_ARGUMENT, "Coulomb plan: use eri4_plan_execute_coulomb");
  return plan_launch(plan,
                     Shells{bra_centers, bra_exponents, bra_coeffs, ket_centers, ket_exponents, ket_coeffs,
                            plan->nket},
                     work, work_size, out, stream);
}

eri4_status eri4_plan_destroy(eri4_plan plan) {
  g_err.clear();
  plan_free(plan);
  return ERI4_SUCCESS;
}

eri4_status eri4_boys(int mmax, int64_t n, const double* T, double* F, hipStream_t stream) {
  g_err.clear();
  if (mmax < 0 || mmax > ERI4_MAX_BOYS_M)
    return fail(ERI4_ERROR_INVALID_ARGUMENT, "mmax must be in 0..%d", ERI4_MAX_BOYS_M);
  if (n < 0) return fail(ERI4_ERROR_INVALID_ARGUMENT, "n must be >= 0");
  if (n == 0) return ERI4_SUCCESS;
  if (!T || !F) return fail(ERI4_ERROR_INVALID_ARGUMENT, "NULL buffer pointer");
  DeviceState* d;
  eri4_status s = ensure_device(&d);
  if (s != ERI4_SUCCESS) return s;
  const int64_t total = n * (mmax + 1);
  const int64_t nb = (total + 255) / 256;
  if (nb > ((int64_t)1 << 31) - 1) return fail(ERI4_ERROR_INVALID_ARGUMENT, "n too large");
  hipLaunchKernelGGL(boys_kernel, dim3((unsigned)nb), dim3(256), 0, stream, mmax, n, T, F, d->boys);
  HIP_TRY(hipGetLastError());
  return ERI4_SUCCESS;
}

eri4_status eri4_hermite_r(int L, int64_t n, const double* zp, const double* zq, const double* P,
                           const double* Q, double* R, hipStream_t stream) {
  g_err.clear();
  if (L < 0 || L > 4 * ERI4_MAX_L)
    return fail(ERI4_ERROR_INVALID_ARGUMENT, "L must be in 0..%d", 4 * ERI4_MAX_L);
  if (n < 0) return fail(ERI4_ERROR_INVALID_ARGUMENT, "n must be >= 0");
  if (n == 0) return ERI4_SUCCESS;
  if (!zp || !zq || !P || !Q || !R) return fail(ERI4_ERROR_INVALID_ARGUMENT, "NULL buffer pointer");
  if (n > ((int64_t)1 << 31) - 1) return fail(ERI4_ERROR_INVALID_ARGUMENT, "n too large");
  DeviceState* d;
  eri4_status s = ensure_device(&d);
  if (s != ERI4_SUCCESS) return s;
  const bool slab = (36 + r_cells(false, L)) * 8 > kMaxLdsBytes;
  const int lds = (36 + r_cells(slab, L)) * 8;
  hipLaunchKernelGGL(hermite_r_kernel, dim3((unsigned)n), dim3(kThreads), lds, stream, L, slab, zp, zq, P, Q, R,
                     d->boys, d->rtab + d->rstart[(slab ? 1 : 0) * (kMaxL + 1) + L]);
  HIP_TRY(hipGetLastError());
  return ERI4_SUCCESS;
}

eri4_status eri4_hermite_e(int la, int lb, int64_t n, const double* za, const double* zb, const double* A,
                           const double* B, double* E, hipStream_t stream) {
  g_err.clear();
  if (la < 0 || lb < 0 || la > kTableLMax || lb > kTableLMax)
    return fail(ERI4_ERROR_INVALID_ARGUMENT, "la, lb must be in 0..%d", kTableLMax);
  if (n < 0) return fail(ERI4_ERROR_INVALID_ARGUMENT, "n must be >= 0");
  if (n == 0) return ERI4_SUCCESS;
  if (!za || !zb || !A || !B || !E) return fail(ERI4_ERROR_INVALID_ARGUMENT, "NULL buffer pointer");
  if (n > ((int64_t)1 << 31) - 1) return fail(ERI4_ERROR_INVALID_ARGUMENT, "n too large");
  DeviceState* d;
  eri4_status s = ensure_device(&d);
  if (s != ERI4_SUCCESS) return s;
  const int trow = odd_row(la + lb + 2);
  const int lds = (3 * ((la + 1) * (lb + 1) + 1) * trow + 16) * 8;
  hipLaunchKernelGGL(hermite_e_kernel, dim3((unsigned)n), dim3(64), lds, stream, la, lb, za, zb, A, B, E);
  HIP_TRY(hipGetLastError());
  return ERI4_SUCCESS;
}

}  // extern "C"
