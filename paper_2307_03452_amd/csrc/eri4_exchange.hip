// eri4_exchange.hip -- exchange-type contraction without forming (ab|cd) (FP64,
// Cartesian): K_ac = sum_bd (ab|cd) D_bd per quartet.  The density's ket index
// is first taken to Hermite space per ket primitive pair and shell-b
// component, F^b[q][c] = sum_d E_cd^q D_bd (sign of eq. (pq) included), then
// the tile code contracts the first transform's [ab|q] with F^b on the matrix
// cores instead of running the second transform (rows of a tile ordered
// (b, a), one b per 16-row block), and a last kernel sums the per-b partial
// rows y^b[a][c] = sum_d (ab|cd) D_bd over b in a fixed order.
#include "eri4_device.h"

namespace eri4 {
namespace {

// F^b of ket primitives (z1, w1) of shell lc and (z2, w2) of shell ld at
// centres c[0..5], for every row b < nb of the density block D[Nb][Nd] (device
// memory), in the operand order of exch_gemm: F^b at out + b * fbs, with
// out[(cc * nq4 / 4 + s) * 64 + l] = F^b[4 s + l / 16][16 cc + l % 16], zero
// past the nq Hermite functions and the nc components.  On the FP64 matrix
// cores: for each Hermite index q and block of 16 components c, the nb x 16
// block F[b][q][c] = sum_d D[b][d] E_cd^q is one product over d (A: D held in
// registers, B: E_cd^q formed from the three 1-d tables).  Called by all
// threads of a workgroup.
__device__ __forceinline__ void build_f(int lc, int ld, int nb, const double* __restrict__ c, double z1, double z2,
                                        double w1, double w2, const double* __restrict__ D,
                                        double* __restrict__ out, int64_t fbs, int tid) {
  constexpr int kNd = ncart(kTableLMax);
  constexpr int kSd = (kNd + 3) / 4;   // MFMA k steps over d, at most
  constexpr int kCb = (kNd + 15) / 16;  // 16-wide blocks of b, at most
  __shared__ double tabs[kMaxEtab];
  __shared__ double pair[16];
  __shared__ int2 qt[kMaxHerm + 16];
  __shared__ int cart[2][kNd];  // (x, y, z) of each component of shells c and d, packed
  const int lane = tid & 63, g = lane >> 4, n = lane & 15, wave = tid >> 6;
  const int Lk = lc + ld, nq = nherm(Lk), nq4 = (nq + 3) & ~3;
  const int tkrow = odd_row(Lk + 2), tkaxis = ((lc + 1) * (ld + 1) + 1) * tkrow;
  const int nc = ncart(lc), nd = ncart(ld), ncc = (nc + 15) / 16;
  const int ksd = (nd + 3) >> 2, ncb = (nb + 15) >> 4;
  if (tid == 0) make_pair(pair, z1, z2, w1, w2, c, c + 3);
  build_htab(qt, Lk, nq, nq4, 0, 0, false, tid);
  for (int e = tid; e < 2 * kNd; e += kThreads) {
    const int sh = e / kNd, k = e - sh * kNd, l = sh ? ld : lc;
    int x = 0, y = 0, z = 0;
    if (k < ncart(l)) cart_of(l, k, x, y, z);
    cart[sh][k] = x | (y << 8) | (z << 16);
  }
  __syncthreads();
  if (tid < 64) build_etab(tabs, lc, ld, tkrow, tkaxis, 0.5 / pair[0], pair + 5, pair + 8, true, lane);
  // A operands: lane (n, g) holds D[16 cb + n][4 s + g] (zero past nb, nd), and
  // the table row offsets of component d = 4 s + g of shell d
  double bd[kCb][kSd];
  int rdx[kSd], rdy[kSd], rdz[kSd];
#pragma unroll
  for (int st = 0; st < kSd; ++st) {
    const int d = 4 * st + g;
    const int cd = cart[1][min(d, nd - 1)];
    rdx[st] = cd & 0xff;
    rdy[st] = (cd >> 8) & 0xff;
    rdz[st] = (cd >> 16) & 0xff;
#pragma unroll
    for (int cb = 0; cb < kCb; ++cb) {
      const int b = 16 * cb + n;
      bd[cb][st] = (b < nb && d < nd) ? D[b * nd + d] : 0.0;
    }
  }
  __syncthreads();
  for (int unit = wave; unit < nq4 * ncc; unit += kWaves) {
    const int q = unit / ncc, cc = unit - (unit / ncc) * ncc;
    const int ci = 16 * cc + n;  // this lane's row: component c of shell c
    const int cw = cart[0][min(ci, nc - 1)];
    const int cx = cw & 0xff, cy = (cw >> 8) & 0xff, cz = (cw >> 16) & 0xff;
    const int hx = qt[q].x;
    const int t = hx & 0xff, u = (hx >> 8) & 0xff, w = (hx >> 16) & 0xff;
    d4 acc[kCb];
#pragma unroll
    for (int cb = 0; cb < kCb; ++cb) acc[cb] = acc_zero<false>();
#pragma unroll
    for (int st = 0; st < kSd; ++st) {
      if (st < ksd) {
        const bool ok = ci < nc && 4 * st + g < nd;
        const double e = ok ? tabs[(cx * (ld + 1) + rdx[st]) * tkrow + t] *
                                  tabs[tkaxis + (cy * (ld + 1) + rdy[st]) * tkrow + u] *
                                  tabs[2 * tkaxis + (cz * (ld + 1) + rdz[st]) * tkrow + w]
                            : 0.0;
#pragma unroll
        for (int cb = 0; cb < kCb; ++cb)
          if (cb < ncb) acc[cb] = mfma16<false>(bd[cb][st], e, acc[cb]);
      }
    }
    // acc[cb]: rows b = 16 cb + acc_row, columns c = 16 cc + n, so that each
    // store covers 16 consecutive components of four b
    const int64_t base = (int64_t)(cc * (nq4 >> 2) + (q >> 2)) * 64 + (q & 3) * 16 + n;
#pragma unroll
    for (int cb = 0; cb < kCb; ++cb) {
      if (cb < ncb) {
#pragma unroll
        for (int jj = 0; jj < 4; ++jj) {
          const int b = 16 * cb + acc_row<false>(jj, g);
          if (b < nb) out[b * fbs + base] = acc[cb][jj];
        }
      }
    }
  }
}

// One workgroup per (quartet q0 + blockIdx.x, ket pair slot blockIdx.y = k *
// kmax + l): F^b of every b at fb + ((blockIdx.x * kmax^2 + slot) * nb + b) * fbs.
__global__ __launch_bounds__(kThreads, 1) void exchange_f_kernel(
    const ClassParams cp, const double* __restrict__ centers, const double* __restrict__ exps,
    const double* __restrict__ coefs, const int32_t* __restrict__ nprim, const double* __restrict__ dens,
    double* __restrict__ fb, int64_t q0, int64_t fbs) {
  const int tid = threadIdx.x;
  const int64_t iq = blockIdx.x;
  const int64_t q = q0 + iq;
  const int slot = blockIdx.y, kmax = cp.kmax;
  const int k = slot / kmax, l = slot - (slot / kmax) * kmax;
  const int Kc = nprim[q * 4 + 2], Kd = nprim[q * 4 + 3];
  if (Kc < 1 || Kc > kmax || Kd < 1 || Kd > kmax || k >= Kc || l >= Kd) return;
  const double* e = exps + (q * 4 + 2) * kmax;
  const double* w = coefs + (q * 4 + 2) * kmax;
  build_f(cp.lc, cp.ld, cp.nb, centers + q * 12 + 6, e[k], e[kmax + l], w[k], w[kmax + l], dens + q * cp.nb * cp.nd,
          fb + (iq * kmax * kmax + slot) * cp.nb * fbs, fbs, tid);
}

// One workgroup = one quartet x one tile of RB*16 bra rows in (b, a) order
// (eri4_fused_kernel with the exchange contraction); the tile's y^b rows go to
// part + q * nb * na * nc.
template <int RB, int LAY>
__global__ __launch_bounds__(kThreads, 1) void eri4_exchange_kernel(
    const ClassParams cp, const double* __restrict__ boys_tab, const uint2* __restrict__ rtab,
    const double* __restrict__ centers, const double* __restrict__ exps, const double* __restrict__ coefs,
    const int32_t* __restrict__ nprim, double* __restrict__ part, int64_t q0, const double* __restrict__ fb,
    int64_t fss) {
  extern __shared__ __align__(16) unsigned char lds[];
  const int tid = threadIdx.x, lane = tid & 63;
  const int wave = __builtin_amdgcn_readfirstlane(tid >> 6);
  const int64_t i = blockIdx.x / cp.nrt;
  const int64_t q = q0 + i;
  const int rt = blockIdx.x % cp.nrt;
  const int64_t kk2 = (int64_t)cp.kmax * cp.kmax;
  process_tile<RB, LAY, false, false, false, true>(
      cp, lds, boys_tab, rtab + cp.rtab_off, centers, exps, coefs, nprim,
      part + i * (int64_t)cp.nb * cp.na * cp.nc, q, rt, tid, wave, lane, nullptr, nullptr, nullptr, 0, nullptr,
      fb + i * kk2 * fss, 0, fss);
}

// K[q0 + blockIdx.x][a][c] = sum over b = 0..nb-1, in that order, of the
// partial rows y^b[a][c].
__global__ void exchange_reduce_kernel(const ClassParams cp, const double* __restrict__ part,
                                       double* __restrict__ out, int64_t q0) {
  const int64_t i = blockIdx.x;
  const int nac = cp.na * cp.nc;
  const double* p = part + i * (int64_t)cp.nb * nac;
  for (int ac = threadIdx.x; ac < nac; ac += blockDim.x) {
    double a = 0.0;
    for (int b = 0; b < cp.nb; ++b) a += p[(int64_t)b * nac + ac];
    out[(q0 + i) * nac + ac] = a;
  }
}

template <int RB, int LAY>
hipError_t exchange_launch_t(const ClassParams& p, dim3 grid, hipStream_t s, const Tables& t, const double* centers,
                             const double* exps, const double* coefs, const int32_t* nprim, double* part, int64_t q0,
                             const double* fb, int64_t fss) {
  hipLaunchKernelGGL((eri4_exchange_kernel<RB, LAY>), grid, dim3(kThreads), p.lds_bytes, s, p, t.boys, t.rtab, centers,
                     exps, coefs, nprim, part, q0, fb, fss);
  return hipGetLastError();
}

}  // namespace

hipError_t exchange_set_attrs() {
  const void* k[8] = {(const void*)eri4_exchange_kernel<1, kLayBox>,  (const void*)eri4_exchange_kernel<2, kLayBox>,
                      (const void*)eri4_exchange_kernel<4, kLayBox>,  (const void*)eri4_exchange_kernel<1, kLaySlab>,
                      (const void*)eri4_exchange_kernel<2, kLaySlab>, (const void*)eri4_exchange_kernel<1, kLayBox2>,
                      (const void*)eri4_exchange_kernel<2, kLayBox2>, (const void*)eri4_exchange_kernel<4, kLayBox2>};
  for (const void* f : k) {
    const hipError_t e = hipFuncSetAttribute(f, hipFuncAttributeMaxDynamicSharedMemorySize, kMaxLdsBytes);
    if (e != hipSuccess) return e;
  }
  return hipSuccess;
}

// The three steps for quartets q0..q0+nq-1: F^b of every ket pair slot and b
// (fbs doubles each, nb per slot, kmax^2 slots per quartet), the integral
// kernels writing y^b into part (nb * na * nc doubles per quartet), and the
// sum over b into out.
hipError_t exchange_launch(const ClassParams& p, int64_t nq, hipStream_t s, const Tables& t, const double* centers,
                           const double* exps, const double* coefs, const int32_t* nprim, const double* dens,
                           double* fb, int64_t fbs, double* part, double* out, int64_t q0) {
  hipLaunchKernelGGL(exchange_f_kernel, dim3((unsigned)nq, (unsigned)(p.kmax * p.kmax)), dim3(kThreads), 0, s, p,
                     centers, exps, coefs, nprim, dens, fb, q0, fbs);
  hipError_t e = hipGetLastError();
  if (e != hipSuccess) return e;
  const dim3 grid((unsigned)(nq * p.nrt));
  const int64_t fss = fbs * p.nb;  // doubles per ket pair slot
  const bool two = p.rb == 2;
#define L(RB, LAY) exchange_launch_t<RB, LAY>(p, grid, s, t, centers, exps, coefs, nprim, part, q0, fb, fss)
  switch (p.lay) {
    case kLaySlab:
      e = two ? L(2, kLaySlab) : L(1, kLaySlab);
      break;
    case kLayBox2:
      e = p.rb == 4 ? L(4, kLayBox2) : (two ? L(2, kLayBox2) : L(1, kLayBox2));
      break;
    default:
      e = p.rb == 4 ? L(4, kLayBox) : (two ? L(2, kLayBox) : L(1, kLayBox));
  }
#undef L
  if (e != hipSuccess) return e;
  hipLaunchKernelGGL(exchange_reduce_kernel, dim3((unsigned)nq), dim3(256), 0, s, p, part, out, q0);
  return hipGetLastError();
}

}  // namespace eri4
