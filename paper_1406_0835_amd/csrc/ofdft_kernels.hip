// HIP kernels of the finite-T orbital-free DFT hot path (CDNA4, wave64).
//
// One F[n] + gradient evaluation with n = phi^2 (arXiv:1406.0835 Sec. II-IV)
// is a fixed sequence of fused passes over a real grid [N1][N2][N3] and its
// transposed half spectrum S[k3][k1][k2] (k3 = 0..N3/2 slowest):
//
//   plane_fwd_density   n = phi^2, real FFT along x3 (two rows per complex
//                       row) and FFT along x2 of one i1 plane in LDS,
//                       transposed store; sum phi^2
//   x1_density_*        FFT along x1 on column tiles, then in reciprocal space:
//                       Hartree (Eq. E2) and pseudopotential energies, the
//                       potential 4 pi n/G^2 + v_ext(G), and for gradient
//                       functionals i G_a n(G) (Eq. s_0defn), inverse x1 FFT
//   plane_inv_grad3     inverse x2 and x3 FFTs of the three components of grad n
//   pointwise_gga       ftGGA + PZ81 at every point (Eqs. FGGA..vftGGA),
//                       W = 2 df/dsigma grad n
//   plane_fwd_w3        forward x3 and x2 FFTs of W
//   x1_divergence       S = v_H + v_ext - i G.W(G) (last line of Eq. vftGGA
//                       in reciprocal space), inverse x1 FFT
//   plane_final         inverse x2 and x3 FFTs, v = df/dn + v_xc + S + alpha,
//                       sum n v
//   reduce_scalars      fixed-order sums of the per-block partials (FP64),
//                       published to host memory when asked
//
// Grids whose (i2, i3) planes are not square or exceed 128 use row passes
// (x3 only: rpass_*) with a separate x2 pass (cpass_x2) instead of the plane
// passes.
// Reciprocal-space operators act on the G set without Nyquist components
// (closed under G -> -G), so the potential is the exact gradient of the
// discrete energy.  All energy and dot-product sums are FP64 wave-shuffle +
// LDS block reductions written per block and summed in a fixed order.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <thread>
#include <cstdio>
#include <cstring>
#include <mutex>
#include <vector>

#include "ofdft_fd.h"
#include "ofdft_fft.h"
#include "ofdft_internal.h"

namespace ofdft {

constexpr int NT = 256;
// block sums of a final pass: f_s, T s_s, XC, T s_xc, sum n v and the two slope sums of a trial
constexpr int kFinalSums = 7;
constexpr double kFourPi = 12.566370614359172953850573533118;

// ---------------------------------------------------------------- helpers
struct Smem {
  char* p;
  __device__ explicit Smem(char* base) : p(base) {}
  template <typename T>
  __device__ T* take(size_t n) {
    T* r = reinterpret_cast<T*>(p);
    p += ((n * sizeof(T) + 15) / 16) * 16;
    return r;
  }
};

template <typename T>
__host__ __device__ constexpr size_t pad16(size_t n) { return ((n * sizeof(T) + 15) / 16) * 16; }

__device__ __forceinline__ double wave_sum(double v) {
#pragma unroll
  for (int off = 32; off > 0; off >>= 1) v += __shfl_xor(v, off, 64);
  return v;
}

// Block sum of K values over NTH threads; the result is valid in thread 0.
// red: LDS of K*NTH/64 doubles.
template <int K, int NTH = NT>
__device__ __forceinline__ void block_sum(double* v, double* red) {
  const int lane = threadIdx.x & 63, w = threadIdx.x >> 6;
#pragma unroll
  for (int k = 0; k < K; ++k) {
    const double s = wave_sum(v[k]);
    if (lane == 0) red[k * (NTH / 64) + w] = s;
  }
  __syncthreads();
  if (threadIdx.x == 0) {
#pragma unroll
    for (int k = 0; k < K; ++k) {
      double s = 0.0;
      for (int i = 0; i < NTH / 64; ++i) s += red[k * (NTH / 64) + i];
      v[k] = s;
    }
  }
  __syncthreads();
}

// Uniform early exit of a whole launch when its gate flag (device memory) is 0.
#define OFDFT_GATE(gp)                         \
  do {                                         \
    if ((gp) != nullptr && *(gp) == 0.0) return; \
  } while (0)

__device__ __forceinline__ int signed_freq(int k, int n) { return (2 * k <= n) ? k : k - n; }

// Cartesian G of spectrum element (k1, k2, k3) and whether it is kept.
__device__ __forceinline__ bool gvec(const GridDesc& g, int k1, int k2, int k3, double& gx, double& gy,
                                     double& gz) {
  const int m1 = signed_freq(k1, g.n1), m2 = signed_freq(k2, g.n2);
  const double m3 = k3;
  gx = m1 * g.b[0] + m2 * g.b[3] + m3 * g.b[6];
  gy = m1 * g.b[1] + m2 * g.b[4] + m3 * g.b[7];
  gz = m1 * g.b[2] + m2 * g.b[5] + m3 * g.b[8];
  return (2 * k1 != g.n1) && (2 * k2 != g.n2) && (2 * k3 != g.n3);
}

// ---------------------------------------------------------------- tile staging
// Tile loads go through registers: each thread first issues all of its global
// loads (elements e = tid + u NT, u < MAXU), then writes them to LDS, so its
// loads are in flight together instead of paying one memory latency each.
// Tile sizes are powers of two (indices by shift and mask) and a staged tile
// holds at most MAXU * NT elements (both checked on the host).
constexpr int MAXU = 8;
static_assert(MAXU * NT == kStageElems, "staged tile size and the host check disagree");

__device__ __forceinline__ int ilog2(int pow2) { return __ffs(pow2) - 1; }

// Element u of this thread in a staged tile of cnt elements, clamped into the
// tile: loads are issued for every u without branches (a clamped lane reads a
// valid element it does not use), so none of them waits for another.
__device__ __forceinline__ int tile_elem(int u, int cnt) {
  const int e = threadIdx.x + u * NT;
  return e < cnt ? e : cnt - 1;
}

// Offsets (elements, from the tile origin) of this thread's staged elements in
// an x1 tile of the transposed spectrum: row k1 = e >> tcl, column c = e & (tc - 1).
template <int U>
__device__ __forceinline__ void x1_offsets(unsigned* off, int cnt, int n2, int tc, int tcl) {
#pragma unroll
  for (int u = 0; u < U; ++u) {
    const int e = tile_elem(u, cnt);
    off[u] = (unsigned)((e >> tcl) * n2 + (e & (tc - 1)));
  }
}

// Twiddles of one transform length go to LDS once per block.  The global load
// is issued before the tile loads and stored after them, so waiting for it
// does not wait for the tile.
// Twiddle m is held by thread m mod NT (lengths above NT take two or more per thread).
template <typename R, int L>
struct TwReg {
  static constexpr int K = (L + NT - 1) / NT;
  cplx<R> v[K];
};
template <typename R, int L>
__device__ __forceinline__ TwReg<R, L> twiddle_load(const cplx<R>* tw_g) {
  TwReg<R, L> r;
#pragma unroll
  for (int m = 0; m < TwReg<R, L>::K; ++m) {
    const int i = (int)threadIdx.x + m * NT;
    r.v[m] = tw_g[i < L ? i : L - 1];
  }
  return r;
}
template <typename R, int L>
__device__ __forceinline__ void twiddle_store(cplx<R>* tw, const TwReg<R, L>& r) {
#pragma unroll
  for (int m = 0; m < TwReg<R, L>::K; ++m) {
    const int i = (int)threadIdx.x + m * NT;
    if (i < L) tw[i] = r.v[m];
  }
}

// ---------------------------------------------------------------- contiguous-axis helpers
// Separate two real rows packed as z = x_a + i x_b (after a forward FFT) into
// their half spectra and store them transposed: S[k3][i1][i2_0 + r] for
// k3 < L/2.  The k3 = L/2 plane holds only Nyquist modes, which every
// reciprocal-space operator drops, so it is neither stored nor read.
template <typename R, int L>
__device__ __forceinline__ void store_half_spectra(const cplx<R>* res, cplx<R>* out, const GridDesc& g,
                                                   int i1, int i2_0, int tr) {
  const int trl = ilog2(tr);
  const int plane = g.n1 * g.n2;
  cplx<R>* ob = out + (size_t)i1 * g.n2 + i2_0;
  const int cnt = (L / 2) * tr;
  cplx<R> X[MAXU];
#pragma unroll
  for (int u = 0; u < MAXU; ++u) {
    const int e = tile_elem(u, cnt);
    const int k3 = e >> trl, r = e & (tr - 1), p = r >> 1;
    const cplx<R> z = res[Lay<L>::at(p, k3)];
    const cplx<R> zc = cconj(res[Lay<L>::at(p, (L - k3) % L)]);
    if ((r & 1) == 0) {
      X[u] = {R(0.5) * (z.x + zc.x), R(0.5) * (z.y + zc.y)};
    } else {
      X[u] = {R(0.5) * (z.y - zc.y), R(-0.5) * (z.x - zc.x)};
    }
  }
#pragma unroll
  for (int u = 0; u < MAXU; ++u) {
    const int e = threadIdx.x + u * NT;
    if (e < cnt) ob[(e >> trl) * plane + (e & (tr - 1))] = X[u];
  }
}

// Load a transposed half-spectrum tile S[k3][i1][i2_0 + r], k3 < L/2
// (staging in LDS), and build z_p[k] = X_{2p}[k] + i X_{2p+1}[k] over the
// full k range using Hermitian symmetry, with the Nyquist term k = L/2 zero.
// stage must hold (L/2)*tr elements; z holds tr/2 rows in the padded row
// layout.  Also stores the twiddles twv (see twiddle_load).
template <typename R, int L>
__device__ __forceinline__ void load_pack_half_spectra(const cplx<R>* in, cplx<R>* stage, cplx<R>* z,
                                                       const GridDesc& g, int i1, int i2_0, int tr,
                                                       cplx<R>* tw, const TwReg<R, L>& twv) {
  const int trl = ilog2(tr);
  const int plane = g.n1 * g.n2;
  const int cnt = (L / 2) * tr;
  const cplx<R>* ib = in + (size_t)i1 * g.n2 + i2_0;
  cplx<R> v[MAXU];
#pragma unroll
  for (int u = 0; u < MAXU; ++u) {
    const int e = tile_elem(u, cnt);
    v[u] = ib[(e >> trl) * plane + (e & (tr - 1))];
  }
  twiddle_store<R, L>(tw, twv);
#pragma unroll
  for (int u = 0; u < MAXU; ++u) {
    const int e = threadIdx.x + u * NT;
    if (e < cnt) stage[e] = v[u];
  }
  __syncthreads();
  const int hp = tr >> 1, hpl = trl - 1;
  for (int e = threadIdx.x; e < hp * L; e += NT) {
    const int k = e >> hpl, p = e & (hp - 1);
    cplx<R> xa = {R(0), R(0)}, xb = {R(0), R(0)};
    if (2 * k < L) {
      xa = stage[k * tr + 2 * p];
      xb = stage[k * tr + 2 * p + 1];
    } else if (2 * k > L) {
      xa = cconj(stage[(L - k) * tr + 2 * p]);
      xb = cconj(stage[(L - k) * tr + 2 * p + 1]);
    }
    z[Lay<L>::at(p, k)] = {xa.x - xb.y, xa.y + xb.x};
  }
  __syncthreads();
}

// LDS elements of the second row buffer of the contiguous-axis passes: it
// also stages a transposed half-spectrum tile of (L/2+1)*tr elements.
template <int L>
__host__ __device__ constexpr int zb_elems(int tr) {
  return ((tr / 2) * Lay<L>::RS > (L / 2 + 1) * tr) ? (tr / 2) * Lay<L>::RS : (L / 2 + 1) * tr;
}

// ---------------------------------------------------------------- K1: density, x3 forward
// A line-search trial on the sphere (ROT) forms its amplitude here:
// phi_t = ca phi + sb dir, stored to phi_out, and n = phi_t^2.
struct Rotation {
  const double* dir;
  double ca, sb;
  double* phi_out;
  const double* coef;   // if set, ca and sb are coef[0], coef[1] (device values)
  __device__ double cos_part() const { return coef ? coef[0] : ca; }
  __device__ double sin_part() const { return coef ? coef[1] : sb; }
};

template <typename R, int L, bool ROT>
__global__ void __launch_bounds__(NT) k_rpass_fwd_density(const double* __restrict__ phi, cplx<R>* __restrict__ out,
                                                          const cplx<R>* __restrict__ tw_g, GridDesc g,
                                                          double* __restrict__ partials, int maxb, Rotation rot) {
  OFDFT_GATE(g.gate);
  extern __shared__ __align__(16) char smem_raw[];
  const int tr = g.tr;
  Smem sm(smem_raw);
  cplx<R>* za = sm.take<cplx<R>>((tr / 2) * Lay<L>::RS);
  cplx<R>* zb = sm.take<cplx<R>>((tr / 2) * Lay<L>::RS);
  cplx<R>* tw = sm.take<cplx<R>>(L);
  double* red = sm.take<double>(NT / 64);
  const int i1 = blockIdx.y, i2_0 = blockIdx.x * tr;
  const double* src = phi + ((size_t)i1 * g.n2 + i2_0) * L;
  const int cnt = tr * L;
  const auto twv = twiddle_load<R, L>(tw_g);
  double pv[MAXU];
#pragma unroll
  for (int u = 0; u < MAXU; ++u) pv[u] = src[tile_elem(u, cnt)];
  if constexpr (ROT) {
    const size_t off = ((size_t)i1 * g.n2 + i2_0) * L;
    double dv_[MAXU];
    const double ca = rot.cos_part(), sb = rot.sin_part();
#pragma unroll
    for (int u = 0; u < MAXU; ++u) dv_[u] = rot.dir[off + tile_elem(u, cnt)];
#pragma unroll
    for (int u = 0; u < MAXU; ++u) {
      pv[u] = ca * pv[u] + sb * dv_[u];
      const int e = threadIdx.x + u * NT;
      if (e < cnt) rot.phi_out[off + e] = pv[u];
    }
  }
  twiddle_store<R, L>(tw, twv);
  R* zr = reinterpret_cast<R*>(za);
  double acc = 0.0;
#pragma unroll
  for (int u = 0; u < MAXU; ++u) {
    const int e = threadIdx.x + u * NT;
    if (e < cnt) {
      const int r = e / L, i3 = e - r * L;
      const double n = pv[u] * pv[u];
      acc += n;
      zr[2 * Lay<L>::at(r >> 1, i3) + (r & 1)] = R(n);
    }
  }
  __syncthreads();
  const cplx<R>* res = lds_fft<R, -1, L, NT>(za, zb, tw, tr / 2, threadIdx.x);
  store_half_spectra<R, L>(res, out, g, i1, i2_0, tr);
  double v[1] = {acc};
  block_sum<1>(v, red);
  if (threadIdx.x == 0) partials[SL_PHI2 * maxb + blockIdx.y * gridDim.x + blockIdx.x] = v[0];
}

// ---------------------------------------------------------------- K2: x2 pass (contiguous rows)
struct Arr3 {
  void* p[3];
};

// One tile of rb rows per block; U staged elements per thread (U * NT >= rb * L).
template <typename R, int L, int SIGN, int U>
__global__ void __launch_bounds__(NT) k_cpass_x2(Arr3 arrs, const cplx<R>* __restrict__ tw_g, int nrows, int rb,
                                                  const double* __restrict__ gate) {
  OFDFT_GATE(gate);
  extern __shared__ __align__(16) char smem_raw[];
  Smem sm(smem_raw);
  cplx<R>* a = sm.take<cplx<R>>(rb * Lay<L>::RS);
  cplx<R>* b = sm.take<cplx<R>>(rb * Lay<L>::RS);
  cplx<R>* tw = sm.take<cplx<R>>(L);
  const int row0 = blockIdx.x * rb;
  const int nr = min(rb, nrows - row0);
  const int cnt = nr * L;
  cplx<R>* x = reinterpret_cast<cplx<R>*>(arrs.p[blockIdx.y]) + (size_t)row0 * L;
  const auto twv = twiddle_load<R, L>(tw_g);
  cplx<R> v[U];
#pragma unroll
  for (int u = 0; u < U; ++u) v[u] = x[tile_elem(u, cnt)];
  twiddle_store<R, L>(tw, twv);
#pragma unroll
  for (int u = 0; u < U; ++u) {
    const int e = threadIdx.x + u * NT;
    if (e < rb * L) {
      const int row = e / L, col = e - row * L;
      a[Lay<L>::at(row, col)] = (e < cnt) ? v[u] : cplx<R>{R(0), R(0)};
    }
  }
  __syncthreads();
  const cplx<R>* res = lds_fft<R, SIGN, L, NT>(a, b, tw, rb, threadIdx.x);
#pragma unroll
  for (int u = 0; u < U; ++u) {
    const int e = tile_elem(u, cnt);
    const int row = e / L, col = e - row * L;
    v[u] = res[Lay<L>::at(row, col)];
  }
#pragma unroll
  for (int u = 0; u < U; ++u) {
    const int e = threadIdx.x + u * NT;
    if (e < cnt) x[e] = v[u];
  }
}

// ---------------------------------------------------------------- K3: x1 pass + density ops
// Store an x1 tile from LDS (row k1 = e >> tcl, column c = e & (tc - 1)): all
// LDS reads first, then the global stores.
template <typename R, int L, int U>
__device__ __forceinline__ void store_x1_tile(const cplx<R>* o, cplx<R>* dst, const unsigned* off, int tc,
                                              int tcl, int cnt) {
  cplx<R> t[U];
#pragma unroll
  for (int u = 0; u < U; ++u) {
    const int e = tile_elem(u, cnt);
    t[u] = o[Lay<L>::at(e & (tc - 1), e >> tcl)];
  }
#pragma unroll
  for (int u = 0; u < U; ++u) {
    const int e = threadIdx.x + u * NT;
    if (e < cnt) dst[off[u]] = t[u];
  }
}

// X1_TF: 4 pi n/G^2 + v_ext and energies, inverse x1 (ftTF); X1_GGA: also i G_a n(G) x 3;
// X1_NHAT: n(G) only (forces); X1_PREC: (P(G) - 1) g(G) with the minimiser's filter
// P = 1/(1 + G^2/k0^2), inverse x1 (modes the passes do not carry keep P = 1).
enum { X1_TF = 0, X1_GGA = 1, X1_NHAT = 2, X1_PREC = 3 };

// U: staged elements per thread, U * NT >= L * tc.
template <typename R, int L, int MODE, int U>
__global__ void __launch_bounds__(NT) k_x1_density(const cplx<R>* __restrict__ A, const cplx<R>* __restrict__ vext,
                                                   cplx<R>* __restrict__ out0, cplx<R>* __restrict__ out1,
                                                   cplx<R>* __restrict__ out2, cplx<R>* __restrict__ s0,
                                                   const cplx<R>* __restrict__ tw_g, GridDesc g,
                                                   double* __restrict__ partials, int maxb) {
  OFDFT_GATE(g.gate);
  extern __shared__ __align__(16) char smem_raw[];
  const int tc = g.tc, tcl = ilog2(tc);
  Smem sm(smem_raw);
  // two tile buffers and in-place transforms: at 128 points and 16 columns a block takes 38 KB,
  // so four blocks share a CU
  cplx<R>* b0 = sm.take<cplx<R>>(tc * Lay<L>::RS);
  cplx<R>* b1 = sm.take<cplx<R>>(tc * Lay<L>::RS);
  cplx<R>* tw = sm.take<cplx<R>>(L);
  double* red = sm.take<double>(2 * NT / 64);
  const int k3 = blockIdx.y, i2_0 = blockIdx.x * tc;
  // element e of the tile: row k1 = e >> tcl (x1 index), column c = e & (tc - 1)
  const size_t tile0 = (size_t)k3 * g.n1 * g.n2 + i2_0;
  const int cnt = L * tc;
  const auto twv = twiddle_load<R, L>(tw_g);
  unsigned off[U];
  x1_offsets<U>(off, cnt, g.n2, tc, tcl);
  cplx<R> av[U], ve[U];
  const cplx<R>* At = A + tile0;
#pragma unroll
  for (int u = 0; u < U; ++u) av[u] = At[off[u]];
  if constexpr (MODE == X1_TF || MODE == X1_GGA) {
    // v_ext(G) of the tile: needed after the forward FFT, in flight meanwhile
    const cplx<R>* Vt = vext + tile0;
#pragma unroll
    for (int u = 0; u < U; ++u) ve[u] = Vt[off[u]];
  }
#pragma unroll
  for (int u = 0; u < U; ++u) {
    const int e = threadIdx.x + u * NT;
    if (e < cnt) b0[Lay<L>::at(e & (tc - 1), e >> tcl)] = av[u];
  }
  twiddle_store<R, L>(tw, twv);
  __syncthreads();
  lds_fft_inplace<R, -1, L, NT, U>(b0, tw, tc, threadIdx.x);
  cplx<R>* res = b0;
  cplx<R>* fa = b1;   // work buffer of the gradient components
  const R inv_n = R(g.inv_n);
  const double wk = (k3 == 0) ? 1.0 : 2.0;
  double eh = 0.0, ee = 0.0;
#pragma unroll
  for (int u = 0; u < U; ++u) {
    const int e = threadIdx.x + u * NT;
    if (e < cnt) {
      const int k1 = e >> tcl, c = e & (tc - 1);
      const int idx = Lay<L>::at(c, k1);
      const size_t gi = tile0 + off[u];
      double gx, gy, gz;
      const bool keep = gvec(g, k1, i2_0 + c, k3, gx, gy, gz);
      const double G2 = gx * gx + gy * gy + gz * gz;
      cplx<R> nh = cscale(res[idx], inv_n);
      cplx<R> S = {R(0), R(0)};
      if (keep && G2 > 0.0) {
        const double nx = nh.x, ny = nh.y;
        const double kern = kFourPi / G2;
        if constexpr (MODE == X1_TF || MODE == X1_GGA) {
          const cplx<R> v = ve[u];
          eh += wk * kern * (nx * nx + ny * ny);
          ee += wk * (nx * double(v.x) + ny * double(v.y));
          S = {R(kern * nx + double(v.x)), R(kern * ny + double(v.y))};
        }
      }
      if (!keep) nh = {R(0), R(0)};
      if constexpr (MODE == X1_PREC) {
        res[idx] = cscale(nh, R(-G2 / (G2 + g.prec_k2)));   // P(G) - 1
      } else if constexpr (MODE == X1_TF) {
        res[idx] = S;
      } else if constexpr (MODE == X1_GGA) {
        s0[gi] = S;
        res[idx] = nh;
      } else {
        out0[gi] = nh;
      }
    }
  }
  if constexpr (MODE == X1_TF || MODE == X1_GGA) {
    double v[2] = {eh, ee};
    block_sum<2>(v, red);
    if (threadIdx.x == 0) {
      const int blk = blockIdx.y * gridDim.x + blockIdx.x;
      partials[SL_EH * maxb + blk] = v[0];
      partials[SL_EEXT * maxb + blk] = v[1];
    }
  } else {
    __syncthreads();
  }
  if constexpr (MODE == X1_TF || MODE == X1_PREC) {
    lds_fft_inplace<R, +1, L, NT, U>(res, tw, tc, threadIdx.x);
    store_x1_tile<R, L, U>(res, out0 + tile0, off, tc, tcl, cnt);
  } else if constexpr (MODE == X1_GGA) {
    cplx<R>* outs[3] = {out0, out1, out2};
#pragma unroll 1
    for (int a = 0; a < 3; ++a) {
      // i G_a n(G) in the transposed order (column c, row k1)
      for (int e = threadIdx.x; e < cnt; e += NT) {
        const int c = e / L, k1 = e - c * L;
        const int m1 = signed_freq(k1, g.n1), m2 = signed_freq(i2_0 + c, g.n2);
        const R ga = R(m1 * g.b[a] + m2 * g.b[3 + a] + double(k3) * g.b[6 + a]);
        const int idx = Lay<L>::at(c, k1);
        const cplx<R> z = res[idx];
        fa[idx] = {-ga * z.y, ga * z.x};
      }
      __syncthreads();
      lds_fft_inplace<R, +1, L, NT, U>(fa, tw, tc, threadIdx.x);
      store_x1_tile<R, L, U>(fa, outs[a] + tile0, off, tc, tcl, cnt);
      __syncthreads();
    }
  }
}

// ---------------------------------------------------------------- K4 split form
// (a) inverse x3 FFT of one gradient component per block (blockIdx.z) into a
// real array; (b) streaming pointwise functional; (c) forward x3 FFT of W.
struct RealArr3 {
  void* p[3];
};

template <typename R, int L>
__global__ void __launch_bounds__(NT) k_rpass_inv_real(Arr3 in, RealArr3 out, const cplx<R>* __restrict__ tw_g,
                                                       GridDesc g) {
  OFDFT_GATE(g.gate);
  extern __shared__ __align__(16) char smem_raw[];
  const int tr = g.tr;
  Smem sm(smem_raw);
  cplx<R>* za = sm.take<cplx<R>>((tr / 2) * Lay<L>::RS);
  cplx<R>* zb = sm.take<cplx<R>>(zb_elems<L>(tr));
  cplx<R>* tw = sm.take<cplx<R>>(L);
  const int i1 = blockIdx.y, i2_0 = blockIdx.x * tr;
  const cplx<R>* src = reinterpret_cast<const cplx<R>*>(in.p[blockIdx.z]);
  R* dst = reinterpret_cast<R*>(out.p[blockIdx.z]) + ((size_t)i1 * g.n2 + i2_0) * L;
  load_pack_half_spectra<R, L>(src, zb, za, g, i1, i2_0, tr, tw, twiddle_load<R, L>(tw_g));
  const cplx<R>* res = lds_fft<R, +1, L, NT>(za, zb, tw, tr / 2, threadIdx.x);
  const int cnt = tr * L;
  R t[MAXU];
#pragma unroll
  for (int u = 0; u < MAXU; ++u) {
    const int e = tile_elem(u, cnt);
    const int r = e / L, i3 = e - r * L;
    const cplx<R> z = res[Lay<L>::at(r >> 1, i3)];
    t[u] = (r & 1) ? z.y : z.x;
  }
#pragma unroll
  for (int u = 0; u < MAXU; ++u) {
    const int e = threadIdx.x + u * NT;
    if (e < cnt) dst[e] = t[u];
  }
}

constexpr int PW_BLOCKS = 2048;   // at most; four points per thread at 128^3

// Blocks of the pointwise kernel: PW_BLOCKS, or one point per thread on grids
// too small to give every thread of PW_BLOCKS blocks a point.
static inline int pw_blocks(const GridDesc& g) {
  const long long b = (g.N + NT - 1) / NT;
  const int cap = g.pwb > 0 ? std::min(g.pwb, PW_BLOCKS) : PW_BLOCKS;
  return (int)std::max(1LL, std::min<long long>(cap, b));
}

// Waves per SIMD the register allocation of k_pointwise_gga must allow: 5 for the FP32 point
// with PZ81 or no XC (96 VGPRs, no spills), fewer where the FP64 point or the KSDT fit need
// more registers.  With NT = 256 a block is one wave per SIMD, so this is also the number of
// resident blocks per CU.
constexpr int pointwise_waves_of(int rsize, int xc) {
  return rsize == 4 ? (xc == 2 ? 3 : 5) : (xc == 2 ? 2 : 3);
}
template <typename R, int XC>
constexpr int pointwise_waves() {
  return pointwise_waves_of((int)sizeof(R), XC);
}

// The gradient functional and XC at one point of amplitude p with density gradient (gx, gy, gz):
// returns v_loc = df/dn + v_xc, replaces the gradient by W = 2 (df/dsigma) grad n and adds the
// point's f, T s, n eps_xc and n T s_xc to the running sums.
template <typename R, int XC>
__device__ __forceinline__ R gga_xc_at(double p, R& gx, R& gy, R& gz, double lt0, const EnhParams& enh,
                                       double& fs, double& ts, double& exc, double& tsxc) {
  const double n = p * p;
  const double nf = n > kDensityFloor ? n : kDensityFloor;
  const R sigma = gx * gx + gy * gy + gz * gz;
  double f, tsl;
  R dfdn, dfds;
  const double ln_n = ln_pos(nf);
  gga_point<R>(nf, ln_n, sigma, lt0, enh, f, dfdn, dfds, tsl);
  R vl = dfdn;
  xc_point<R>(XC, n, ln_n, lt0, vl, exc, tsxc);   // XC fixed at compile time: no registers for the others
  fs += f;
  ts += tsl;
  const R w2 = R(2) * dfds;
  gx *= w2;
  gy *= w2;
  gz *= w2;
  return vl;
}

// Finite-T GGA + PZ81 at every point: v_loc = df/dn + v_xc, W = 2 df/dsigma grad n
// (written over grad n), energy partial sums per block.
template <typename R, int XC>
__global__ void __launch_bounds__(NT, (pointwise_waves<R, XC>()))
    k_pointwise_gga(const double* __restrict__ phi, R* __restrict__ g0, R* __restrict__ g1, R* __restrict__ g2,
                    R* __restrict__ vloc, long long npts, EvalParams ep, double* __restrict__ partials, int maxb) {
  OFDFT_GATE(ep.gate);
  __shared__ double red[4 * NT / 64];
  EnhParams enh{(int)ep.enh_kind, ep.enh_c1, ep.enh_a1};
  double fs = 0.0, ts = 0.0, exc = 0.0, tsxc = 0.0;
  for (long long i = (long long)blockIdx.x * NT + threadIdx.x; i < npts; i += (long long)gridDim.x * NT) {
    R gx = g0[i], gy = g1[i], gz = g2[i];
    vloc[i] = gga_xc_at<R, XC>(phi[i], gx, gy, gz, ep.lt0, enh, fs, ts, exc, tsxc);
    g0[i] = gx;
    g1[i] = gy;
    g2[i] = gz;
  }
  double v[4] = {fs, ts, exc, tsxc};
  block_sum<4>(v, red);
  if (threadIdx.x == 0) {
    partials[SL_FS * maxb + blockIdx.x] = v[0];
    partials[SL_TS * maxb + blockIdx.x] = v[1];
    partials[SL_EXC * maxb + blockIdx.x] = v[2];
    partials[SL_TSXC * maxb + blockIdx.x] = v[3];
  }
}

template <typename R, int L>
__global__ void __launch_bounds__(NT) k_rpass_fwd_real(RealArr3 in, Arr3 out, const cplx<R>* __restrict__ tw_g,
                                                       GridDesc g) {
  OFDFT_GATE(g.gate);
  extern __shared__ __align__(16) char smem_raw[];
  const int tr = g.tr;
  Smem sm(smem_raw);
  cplx<R>* za = sm.take<cplx<R>>((tr / 2) * Lay<L>::RS);
  cplx<R>* zb = sm.take<cplx<R>>((tr / 2) * Lay<L>::RS);
  cplx<R>* tw = sm.take<cplx<R>>(L);
  const int i1 = blockIdx.y, i2_0 = blockIdx.x * tr;
  const R* src = reinterpret_cast<const R*>(in.p[blockIdx.z]) + ((size_t)i1 * g.n2 + i2_0) * L;
  cplx<R>* dst = reinterpret_cast<cplx<R>*>(out.p[blockIdx.z]);
  const int cnt = tr * L;
  const auto twv = twiddle_load<R, L>(tw_g);
  R xv[MAXU];
#pragma unroll
  for (int u = 0; u < MAXU; ++u) xv[u] = src[tile_elem(u, cnt)];
  twiddle_store<R, L>(tw, twv);
  R* zr = reinterpret_cast<R*>(za);
#pragma unroll
  for (int u = 0; u < MAXU; ++u) {
    const int e = threadIdx.x + u * NT;
    if (e < cnt) {
      const int r = e / L, i3 = e - r * L;
      zr[2 * Lay<L>::at(r >> 1, i3) + (r & 1)] = xv[u];
    }
  }
  __syncthreads();
  const cplx<R>* res = lds_fft<R, -1, L, NT>(za, zb, tw, tr / 2, threadIdx.x);
  store_half_spectra<R, L>(res, dst, g, i1, i2_0, tr);
}

// Forward x3 FFT of the minimiser's projected gradient g = 2 dv phi (v - mu),
// formed on the fly (the first pass of the preconditioner P g).
template <typename R, int L>
__global__ void __launch_bounds__(NT) k_rpass_fwd_grad(const double* __restrict__ phi, const R* __restrict__ v,
                                                       const double* __restrict__ sc, double two_dv,
                                                       cplx<R>* __restrict__ out, const cplx<R>* __restrict__ tw_g,
                                                       GridDesc g) {
  OFDFT_GATE(g.gate);
  extern __shared__ __align__(16) char smem_raw[];
  const int tr = g.tr;
  Smem sm(smem_raw);
  cplx<R>* za = sm.take<cplx<R>>((tr / 2) * Lay<L>::RS);
  cplx<R>* zb = sm.take<cplx<R>>((tr / 2) * Lay<L>::RS);
  cplx<R>* tw = sm.take<cplx<R>>(L);
  const int i1 = blockIdx.y, i2_0 = blockIdx.x * tr;
  const size_t base = ((size_t)i1 * g.n2 + i2_0) * L;
  const int cnt = tr * L;
  const auto twv = twiddle_load<R, L>(tw_g);
  double pv[MAXU];
  R vv[MAXU];
#pragma unroll
  for (int u = 0; u < MAXU; ++u) {
    const int e = tile_elem(u, cnt);
    pv[u] = phi[base + e];
    vv[u] = v[base + e];
  }
  twiddle_store<R, L>(tw, twv);
  const double mu = sc[SC_MU];
  R* zr = reinterpret_cast<R*>(za);
#pragma unroll
  for (int u = 0; u < MAXU; ++u) {
    const int e = threadIdx.x + u * NT;
    if (e < cnt) {
      const int r = e / L, i3 = e - r * L;
      zr[2 * Lay<L>::at(r >> 1, i3) + (r & 1)] = R(two_dv * pv[u] * (double(vv[u]) - mu));
    }
  }
  __syncthreads();
  const cplx<R>* res = lds_fft<R, -1, L, NT>(za, zb, tw, tr / 2, threadIdx.x);
  store_half_spectra<R, L>(res, out, g, i1, i2_0, tr);
}

// ---------------------------------------------------------------- K5: x1 pass + divergence term
template <typename R, int L, int U>
__global__ void __launch_bounds__(NT) k_x1_divergence(const cplx<R>* __restrict__ C0, const cplx<R>* __restrict__ C1,
                                                      const cplx<R>* __restrict__ C2, const cplx<R>* __restrict__ s0,
                                                      cplx<R>* __restrict__ out, const cplx<R>* __restrict__ tw_g,
                                                      GridDesc g) {
  OFDFT_GATE(g.gate);
  extern __shared__ __align__(16) char smem_raw[];
  const int tc = g.tc, tcl = ilog2(tc);
  Smem sm(smem_raw);
  cplx<R>* acc = sm.take<cplx<R>>(tc * Lay<L>::RS);
  cplx<R>* b0 = sm.take<cplx<R>>(tc * Lay<L>::RS);
  cplx<R>* tw = sm.take<cplx<R>>(L);
  const int k3 = blockIdx.y, i2_0 = blockIdx.x * tc;
  const size_t tile0 = (size_t)k3 * g.n1 * g.n2 + i2_0;
  const int cnt = L * tc;
  const cplx<R>* Cs[3] = {C0, C1, C2};
  const auto twv = twiddle_load<R, L>(tw_g);
  // S0 and the first component are loaded together; each later component is
  // loaded into registers while the previous one is transformed
  unsigned off[U];
  x1_offsets<U>(off, cnt, g.n2, tc, tcl);
  cplx<R> sv[U], cv[U];
  {
    const cplx<R>* St = s0 + tile0;
    const cplx<R>* Ct = C0 + tile0;
#pragma unroll
    for (int u = 0; u < U; ++u) {
      sv[u] = St[off[u]];
      cv[u] = Ct[off[u]];
    }
  }
#pragma unroll
  for (int u = 0; u < U; ++u) {
    const int e = threadIdx.x + u * NT;
    if (e < cnt) acc[Lay<L>::at(e & (tc - 1), e >> tcl)] = sv[u];
  }
  twiddle_store<R, L>(tw, twv);
  const R inv_n = R(g.inv_n);
#pragma unroll 1
  for (int a = 0; a < 3; ++a) {
#pragma unroll
    for (int u = 0; u < U; ++u) {
      const int e = threadIdx.x + u * NT;
      if (e < cnt) b0[Lay<L>::at(e & (tc - 1), e >> tcl)] = cv[u];
    }
    if (a < 2) {
      const cplx<R>* nxt = Cs[a + 1] + tile0;
#pragma unroll
      for (int u = 0; u < U; ++u) cv[u] = nxt[off[u]];
    }
    __syncthreads();
    lds_fft_inplace<R, -1, L, NT, U>(b0, tw, tc, threadIdx.x);
    const cplx<R>* res = b0;
    for (int e = threadIdx.x; e < cnt; e += NT) {
      const int c = e / L, k1 = e - c * L;
      const int k2 = i2_0 + c;
      if ((2 * k1 != g.n1) && (2 * k2 != g.n2) && (2 * k3 != g.n3)) {
        const int m1 = signed_freq(k1, g.n1), m2 = signed_freq(k2, g.n2);
        const R ga = R(m1 * g.b[a] + m2 * g.b[3 + a] + double(k3) * g.b[6 + a]) * inv_n;
        const int idx = Lay<L>::at(c, k1);
        const cplx<R> z = res[idx];
        // acc -= i G_a W_a(G)
        acc[idx].x += ga * z.y;
        acc[idx].y -= ga * z.x;
      }
    }
    __syncthreads();
  }
  lds_fft_inplace<R, +1, L, NT, U>(acc, tw, tc, threadIdx.x);
  store_x1_tile<R, L, U>(acc, out + tile0, off, tc, tcl, cnt);
}

// ---------------------------------------------------------------- scalar reduction
struct ReduceParams {
  int nb_r, nb_x1;   // partial counts of the density/final passes and the x1 pass
  int nb_fs;         // partial count of the free-energy slots (pointwise kernel or final pass)
  int trial;         // 1: also dF/dtheta of a line-search trial into SC_DOT0
  double dv, volume, alpha_sum;
  const double* gate;
  int nb_fin;        // partial count of the final pass's slots (n v, dF/dtheta)
};

// Destination of a device-written readback: dst[0..n) and then the sequence
// word flag = seq, both in fine-grained host memory (dst == nullptr: none).
struct Publish {
  double* dst;
  unsigned long long* flag;
  unsigned long long seq;
  const double* extra;   // also extra[0..n_extra) after the kernel's own values
  int n_extra;
};

// Store vals[0..n) into the host buffer and raise its sequence word.  Called by
// lanes of one wavefront only; the system-scope release on the flag orders it
// after the wavefront's data stores.
__device__ __forceinline__ void publish(const Publish& pub, const double* vals, int n, int lane) {
  for (int k = lane; k < n; k += 64) pub.dst[k] = vals[k];
  for (int k = lane; k < pub.n_extra; k += 64) pub.dst[n + k] = pub.extra[k];
  __threadfence_system();
  if (lane == 0) __hip_atomic_store(pub.flag, pub.seq, __ATOMIC_RELEASE, __HIP_MEMORY_SCOPE_SYSTEM);
}

// The evaluation's scalars from the per-block partials: each wavefront of the
// NTH-thread block sums whole slots in a fixed order (eight accumulators per
// lane, then the wave sum), thread 0 forms the energies, mu and dF/dtheta.
// raw: LDS of SL_COUNT doubles, out: LDS of SC_COUNT doubles.
template <int NTH>
__device__ __forceinline__ void reduce_scalars(const double* __restrict__ partials, int maxb, const ReduceParams& rp,
                                               double* __restrict__ sc, const Publish& pub, double* raw,
                                               double* out) {
  const int w = threadIdx.x >> 6, lane = threadIdx.x & 63;
  for (int s = w; s < SL_COUNT; s += NTH / 64) {
    const int cnt = (s == SL_EH || s == SL_EEXT) ? rp.nb_x1
                    : (s == SL_FS || s == SL_TS || s == SL_EXC || s == SL_TSXC) ? rp.nb_fs
                    : (s == SL_DT1 || s == SL_DT2) ? (rp.trial ? rp.nb_fin : 0)
                    : (s == SL_NV) ? rp.nb_fin : rp.nb_r;
    const double* ps = partials + (size_t)s * maxb;
    double a[8] = {0, 0, 0, 0, 0, 0, 0, 0};
    int i = lane;
    for (; i + 7 * 64 < cnt; i += 8 * 64) {
#pragma unroll
      for (int u = 0; u < 8; ++u) a[u] += ps[i + u * 64];
    }
    for (; i < cnt; i += 64) a[0] += ps[i];
    double acc = ((a[0] + a[1]) + (a[2] + a[3])) + ((a[4] + a[5]) + (a[6] + a[7]));
    acc = wave_sum(acc);
    if (lane == 0) raw[s] = acc;
  }
  __syncthreads();
  if (threadIdx.x == 0) {
    const double Ne = rp.dv * raw[SL_PHI2];
    out[SC_NE] = Ne;
    out[SC_FS] = rp.dv * raw[SL_FS];
    out[SC_TS] = rp.dv * raw[SL_TS];
    out[SC_EXC] = rp.dv * raw[SL_EXC];
    out[SC_EH] = 0.5 * rp.volume * raw[SL_EH];
    out[SC_EEXT] = rp.volume * raw[SL_EEXT];
    out[SC_NV] = rp.dv * raw[SL_NV];
    out[SC_MU] = raw[SL_NV] / raw[SL_PHI2];
    out[SC_EAZ] = Ne * rp.alpha_sum;
    out[SC_EION] = 0.0;
    out[SC_FTOT] = out[SC_FS] + out[SC_EXC] + out[SC_EH] + out[SC_EEXT] + out[SC_EAZ];
    for (int k = SC_FTOT + 1; k < SC_COUNT; ++k) out[k] = 0.0;   // dot slots cleared
    if (rp.trial) out[SC_DOT0] = 2.0 * rp.dv * (raw[SL_DT1] - out[SC_MU] * raw[SL_DT2]);
    out[SC_TSXC] = rp.dv * raw[SL_TSXC];
  }
  __syncthreads();
  if (threadIdx.x < SC_COUNT) sc[threadIdx.x] = out[threadIdx.x];
  if (pub.dst && threadIdx.x < 64) publish(pub, out, SC_COUNT, threadIdx.x);
}

// ---------------------------------------------------------------- K6: final potential
// DT: a line-search trial also accumulates sum phi_t v_t q and sum phi_t q with
// q = ms phi0 + mc dir (phi0 the point the trial rotates from), the two pieces of
// dF/dtheta = 2 dv (sum phi_t v_t q - mu sum phi_t q).
struct Slope {
  const double* phi0;
  const double* dir;
  double ms, mc;
  const double* coef;   // if set, ms and mc are coef[2], coef[3] (device values)
  __device__ double ms_part() const { return coef ? coef[2] : ms; }
  __device__ double mc_part() const { return coef ? coef[3] : mc; }
};

template <typename R, int L, bool TF, bool DT>
__global__ void __launch_bounds__(NT) k_rpass_final(const cplx<R>* __restrict__ D, const double* __restrict__ phi,
                                                    const R* __restrict__ vloc, R* __restrict__ vout,
                                                    const cplx<R>* __restrict__ tw_g, GridDesc g, EvalParams ep,
                                                    double* __restrict__ partials, int maxb, Slope sl) {
  OFDFT_GATE(g.gate);
  extern __shared__ __align__(16) char smem_raw[];
  const int tr = g.tr;
  Smem sm(smem_raw);
  cplx<R>* za = sm.take<cplx<R>>((tr / 2) * Lay<L>::RS);
  cplx<R>* zb = sm.take<cplx<R>>(zb_elems<L>(tr));
  cplx<R>* tw = sm.take<cplx<R>>(L);
  double* red = sm.take<double>(kFinalSums * NT / 64);
  const int i1 = blockIdx.y, i2_0 = blockIdx.x * tr;
  const size_t base = ((size_t)i1 * g.n2 + i2_0) * L;
  const int cnt = tr * L;
  load_pack_half_spectra<R, L>(D, zb, za, g, i1, i2_0, tr, tw, twiddle_load<R, L>(tw_g));
  // phi and v_loc of the tile, in flight during the inverse FFT
  double pv[MAXU], q[MAXU];
  R lv[MAXU];
#pragma unroll
  for (int u = 0; u < MAXU; ++u) {
    const int e = tile_elem(u, cnt);
    pv[u] = phi[base + e];
    if constexpr (!TF) lv[u] = vloc[base + e];
  }
  if constexpr (DT) {
    double p0[MAXU], dd[MAXU];
#pragma unroll
    for (int u = 0; u < MAXU; ++u) {
      const int e = tile_elem(u, cnt);
      p0[u] = sl.phi0[base + e];
      dd[u] = sl.dir[base + e];
    }
    const double ms = sl.ms_part(), mc = sl.mc_part();
#pragma unroll
    for (int u = 0; u < MAXU; ++u) q[u] = ms * p0[u] + mc * dd[u];
  }
  const cplx<R>* res = lds_fft<R, +1, L, NT>(za, zb, tw, tr / 2, threadIdx.x);
  double fs = 0.0, ts = 0.0, exc = 0.0, tsxc = 0.0, nv = 0.0, dt1 = 0.0, dt2 = 0.0;
#pragma unroll
  for (int u = 0; u < MAXU; ++u) {
    const int e = threadIdx.x + u * NT;
    if (e >= cnt) continue;
    const int r = e / L, i3 = e - r * L;
    const cplx<R> z = res[Lay<L>::at(r >> 1, i3)];
    const double S = (r & 1) ? double(z.y) : double(z.x);
    const double p = pv[u];
    const double n = p * p;
    double vl;
    if constexpr (TF) {
      const double nf = n > kDensityFloor ? n : kDensityFloor;
      double f, vt, tsl;
      const double ln_n = ln_pos(nf);
      tf_point(nf, ln_n, ep.lt0, f, vt, tsl);
      vl = vt;
      fs += f;
      ts += tsl;
      xc_point<R>(ep.xc, n, ln_n, ep.lt0, vl, exc, tsxc);
    } else {
      vl = double(lv[u]);
    }
    const R vv = R(vl + S + ep.alpha_sum);
    vout[base + e] = vv;
    nv += n * double(vv);
    if constexpr (DT) {
      dt1 += p * double(vv) * q[u];
      dt2 += p * q[u];
    }
  }
  constexpr int K = (TF ? 5 : 1) + (DT ? 2 : 0);
  double v[K];
  int slot[K];
  int k = 0;
  if constexpr (TF) {
    v[k] = fs; slot[k++] = SL_FS;
    v[k] = ts; slot[k++] = SL_TS;
    v[k] = exc; slot[k++] = SL_EXC;
    v[k] = tsxc; slot[k++] = SL_TSXC;
  }
  v[k] = nv; slot[k++] = SL_NV;
  if constexpr (DT) {
    v[k] = dt1; slot[k++] = SL_DT1;
    v[k] = dt2; slot[k++] = SL_DT2;
  }
  block_sum<K>(v, red);
  if (threadIdx.x == 0) {
    const int blk = blockIdx.y * gridDim.x + blockIdx.x;
#pragma unroll
    for (int m = 0; m < K; ++m) partials[slot[m] * maxb + blk] = v[m];
  }
}

// ---------------------------------------------------------------- plane passes
// Grids with n2 == n3 = L <= 128: the x3 and x2 transforms of one i1 plane run
// in one block of NTP threads, and the plane's half spectrum stays in LDS
// between the two axes, so the x2 transform costs no HBM round trip (the
// separate x2 pass and the row passes above serve the other grids).  One LDS
// buffer of L/2 padded rows holds both layouts: packed rows P[p][i3] with
// z_p = x_{2p} + i x_{2p+1} for the x3 transform, and T[k3][k2], k3 < L/2, for
// the x2 transform.  Changes of layout go through registers, every read
// before a barrier and every write after it.
constexpr int NTP = 1024;   // threads of a plane block

// Elements per thread of the in-place transforms of a half plane ((L/2) L points).
template <int L, int NTH>
__host__ __device__ constexpr int plane_maxe() { return ((L / 2) * L + NTH - 1) / NTH; }
// The same for a quarter of the rows (the half-plane transforms of the split passes).
template <int L, int NTH>
__host__ __device__ constexpr int plane_maxe_q() { return ((L / 4) * L + NTH - 1) / NTH; }

template <typename R, int L>
__host__ __device__ constexpr size_t lds_plane(int nred) {
  return pad16<cplx<R>>((size_t)(L / 2) * Lay<L>::RS) + pad16<cplx<R>>(L) + pad16<double>((size_t)nred * NTP / 64);
}

// x3 forward transform of the packed rows, then the half spectra of rows 2p
// and 2p+1 (k3 < L/2) written transposed into T[k3][2p], T[k3][2p+1].
template <typename R, int L, int NTH>
__device__ __forceinline__ void plane_x3_fwd_to_T(cplx<R>* buf, const cplx<R>* tw) {
  lds_fft_inplace<R, -1, L, NTH, plane_maxe<L, NTH>()>(buf, tw, L / 2, threadIdx.x);
  constexpr int H = L / 2, ITEMS = H * H, MI = (ITEMS + NTH - 1) / NTH;
  cplx<R> xa[MI], xb[MI];
#pragma unroll
  for (int m = 0; m < MI; ++m) {
    const int it = threadIdx.x + m * NTH;
    if (it < ITEMS) {
      const int p = it / H, k3 = it - p * H;
      const cplx<R> z = buf[Lay<L>::at(p, k3)];
      const cplx<R> zc = cconj(buf[Lay<L>::at(p, (L - k3) % L)]);
      xa[m] = {R(0.5) * (z.x + zc.x), R(0.5) * (z.y + zc.y)};
      xb[m] = {R(0.5) * (z.y - zc.y), R(-0.5) * (z.x - zc.x)};
    }
  }
  __syncthreads();
#pragma unroll
  for (int m = 0; m < MI; ++m) {
    const int it = threadIdx.x + m * NTH;
    if (it < ITEMS) {
      const int p = it / H, k3 = it - p * H;
      buf[Lay<L>::at(k3, 2 * p)] = xa[m];
      buf[Lay<L>::at(k3, 2 * p + 1)] = xb[m];
    }
  }
  __syncthreads();
}

// x2 forward transform of the T rows, stored as S[k3][i1][k2].
template <typename R, int L, int NTH>
__device__ __forceinline__ void plane_x2_fwd_store(cplx<R>* buf, const cplx<R>* tw, cplx<R>* out,
                                                   const GridDesc& g, int i1) {
  lds_fft_inplace<R, -1, L, NTH, plane_maxe<L, NTH>()>(buf, tw, L / 2, threadIdx.x);
  const size_t plane = (size_t)g.n1 * L;
  constexpr int CNT = (L / 2) * L;
  for (int e = threadIdx.x; e < CNT; e += NTH) {
    const int k3 = e / L, k2 = e - k3 * L;
    out[k3 * plane + (size_t)i1 * L + k2] = buf[Lay<L>::at(k3, k2)];
  }
}

// T[k3][k2] = S[k3][i1][k2] (k3 < L/2) and the twiddles; ends with a barrier.
template <typename R, int L, int NTH>
__device__ __forceinline__ void plane_load_T(cplx<R>* buf, cplx<R>* tw, const cplx<R>* in,
                                             const cplx<R>* tw_g, const GridDesc& g, int i1) {
  const size_t plane = (size_t)g.n1 * L;
  constexpr int CNT = (L / 2) * L, MU = (CNT + NTH - 1) / NTH;
  const auto twv = twiddle_load<R, L>(tw_g);
  cplx<R> v[MU];
#pragma unroll
  for (int m = 0; m < MU; ++m) {
    const int e = min((int)threadIdx.x + m * NTH, CNT - 1);
    const int k3 = e / L, k2 = e - k3 * L;
    v[m] = in[k3 * plane + (size_t)i1 * L + k2];
  }
  twiddle_store<R, L>(tw, twv);
#pragma unroll
  for (int m = 0; m < MU; ++m) {
    const int e = threadIdx.x + m * NTH;
    if (e < CNT) {
      const int k3 = e / L, k2 = e - k3 * L;
      buf[Lay<L>::at(k3, k2)] = v[m];
    }
  }
  __syncthreads();
}

// x2 inverse transform of the T rows, the packed rows z_p[k] = X_{2p}[k] +
// i X_{2p+1}[k] over all k (Hermitian symmetry, Nyquist term zero), and the x3
// inverse transform: real element (i2, i3) is then Re or Im of P[i2/2][i3].
template <typename R, int L, int NTH>
__device__ __forceinline__ void plane_inv(cplx<R>* buf, const cplx<R>* tw) {
  lds_fft_inplace<R, +1, L, NTH, plane_maxe<L, NTH>()>(buf, tw, L / 2, threadIdx.x);
  constexpr int H = L / 2, ITEMS = H * L, MI = (ITEMS + NTH - 1) / NTH;
  cplx<R> z[MI];
#pragma unroll
  for (int m = 0; m < MI; ++m) {
    const int it = threadIdx.x + m * NTH;
    if (it < ITEMS) {
      const int p = it / L, k = it - p * L;
      cplx<R> xa = {R(0), R(0)}, xb = {R(0), R(0)};
      if (2 * k < L) {
        xa = buf[Lay<L>::at(k, 2 * p)];
        xb = buf[Lay<L>::at(k, 2 * p + 1)];
      } else if (2 * k > L) {
        xa = cconj(buf[Lay<L>::at(L - k, 2 * p)]);
        xb = cconj(buf[Lay<L>::at(L - k, 2 * p + 1)]);
      }
      z[m] = {xa.x - xb.y, xa.y + xb.x};
    }
  }
  __syncthreads();
#pragma unroll
  for (int m = 0; m < MI; ++m) {
    const int it = threadIdx.x + m * NTH;
    if (it < ITEMS) {
      const int p = it / L, k = it - p * L;
      buf[Lay<L>::at(p, k)] = z[m];
    }
  }
  __syncthreads();
  // an opaque copy of the thread index, so that the second transform recomputes its LDS
  // addresses instead of keeping the first transform's live (which spilled them)
  int tid = threadIdx.x;
  asm volatile("" : "+v"(tid));
  lds_fft_inplace<R, +1, L, NTH, plane_maxe<L, NTH>()>(buf, tw, L / 2, tid);
}

template <typename R, int L>
__device__ __forceinline__ R plane_real(const cplx<R>* buf, int e) {
  const int i2 = e / L, i3 = e - i2 * L;
  const cplx<R> z = buf[Lay<L>::at(i2 >> 1, i3)];
  return (i2 & 1) ? z.y : z.x;
}

// Chunk of the plane's real elements per thread in the load and store loops.
constexpr int PCH = 8;

// The density and final passes split each i1 plane over two blocks (at 128^3 one block per
// plane gives 128 workgroups for 256 CUs).  Block b takes plane i1 and half h; the two halves
// of a plane are 8 block indices apart, so the round-robin dispatch of workgroups over the
// 8 XCDs places them on the same XCD, whose L2 then serves the second read of the plane.
__device__ __forceinline__ void plane_half(int b, int n1, int& i1, int& h) {
  if ((n1 & 7) == 0) {
    i1 = (b >> 4) * 8 + (b & 7);
    h = (b >> 3) & 1;
  } else {
    i1 = b >> 1;
    h = b & 1;
  }
}

// x3 forward transform of the packed rows, then the half spectra written transposed into
// T[k3][i2] for k3 in [k0, k0 + L/4) only (the rows this block's x2 transform takes).
template <typename R, int L, int NTH>
__device__ __forceinline__ void plane_x3_fwd_to_T_half(cplx<R>* buf, const cplx<R>* tw, int k0) {
  lds_fft_inplace<R, -1, L, NTH, plane_maxe<L, NTH>()>(buf, tw, L / 2, threadIdx.x);
  constexpr int H = L / 2, Q = L / 4, ITEMS = H * Q, MI = (ITEMS + NTH - 1) / NTH;
  cplx<R> xa[MI], xb[MI];
#pragma unroll
  for (int m = 0; m < MI; ++m) {
    const int it = threadIdx.x + m * NTH;
    if (it < ITEMS) {
      const int p = it / Q, k3 = k0 + (it - p * Q);
      const cplx<R> z = buf[Lay<L>::at(p, k3)];
      const cplx<R> zc = cconj(buf[Lay<L>::at(p, (L - k3) % L)]);
      xa[m] = {R(0.5) * (z.x + zc.x), R(0.5) * (z.y + zc.y)};
      xb[m] = {R(0.5) * (z.y - zc.y), R(-0.5) * (z.x - zc.x)};
    }
  }
  __syncthreads();
#pragma unroll
  for (int m = 0; m < MI; ++m) {
    const int it = threadIdx.x + m * NTH;
    if (it < ITEMS) {
      const int p = it / Q, k3 = k0 + (it - p * Q);
      buf[Lay<L>::at(k3, 2 * p)] = xa[m];
      buf[Lay<L>::at(k3, 2 * p + 1)] = xb[m];
    }
  }
  __syncthreads();
}

// x2 forward transform of the T rows k3 in [k0, k0 + L/4), stored as S[k3][i1][k2].
template <typename R, int L, int NTH>
__device__ __forceinline__ void plane_x2_fwd_store_half(cplx<R>* buf, const cplx<R>* tw, cplx<R>* out,
                                                        const GridDesc& g, int i1, int k0) {
  cplx<R>* rows = buf + k0 * Lay<L>::RS;
  lds_fft_inplace<R, -1, L, NTH, plane_maxe_q<L, NTH>()>(rows, tw, L / 4, threadIdx.x);
  const size_t plane = (size_t)g.n1 * L;
  constexpr int CNT = (L / 4) * L;
  for (int e = threadIdx.x; e < CNT; e += NTH) {
    const int r = e / L, k2 = e - r * L;
    out[(k0 + r) * plane + (size_t)i1 * L + k2] = rows[Lay<L>::at(r, k2)];
  }
}

// Inverse of a half plane: x2 inverse of all T rows, the packed rows z_p (p in [p0, p0 + L/4))
// and their x3 inverse; real element (i2, i3) with i2 in [2 p0, 2 p0 + L/2) is then Re or Im of
// P[i2/2][i3].
template <typename R, int L, int NTH>
__device__ __forceinline__ void plane_inv_half(cplx<R>* buf, const cplx<R>* tw, int p0) {
  lds_fft_inplace<R, +1, L, NTH, plane_maxe<L, NTH>()>(buf, tw, L / 2, threadIdx.x);
  constexpr int Q = L / 4, ITEMS = Q * L, MI = (ITEMS + NTH - 1) / NTH;
  cplx<R> z[MI];
#pragma unroll
  for (int m = 0; m < MI; ++m) {
    const int it = threadIdx.x + m * NTH;
    if (it < ITEMS) {
      const int p = p0 + it / L, k = it % L;
      cplx<R> xa = {R(0), R(0)}, xb = {R(0), R(0)};
      if (2 * k < L) {
        xa = buf[Lay<L>::at(k, 2 * p)];
        xb = buf[Lay<L>::at(k, 2 * p + 1)];
      } else if (2 * k > L) {
        xa = cconj(buf[Lay<L>::at(L - k, 2 * p)]);
        xb = cconj(buf[Lay<L>::at(L - k, 2 * p + 1)]);
      }
      z[m] = {xa.x - xb.y, xa.y + xb.x};
    }
  }
  __syncthreads();
#pragma unroll
  for (int m = 0; m < MI; ++m) {
    const int it = threadIdx.x + m * NTH;
    if (it < ITEMS) {
      const int p = p0 + it / L, k = it % L;
      buf[Lay<L>::at(p, k)] = z[m];
    }
  }
  __syncthreads();
  int tid = threadIdx.x;
  asm volatile("" : "+v"(tid));
  lds_fft_inplace<R, +1, L, NTH, plane_maxe_q<L, NTH>()>(buf + p0 * Lay<L>::RS, tw, L / 4, tid);
}

// F1: n = phi^2 (phi_t = ca phi + sb dir for a line-search trial), x3 and x2
// forward; sum phi^2 per plane.
template <typename R, int L, bool ROT>
__global__ void __launch_bounds__(NTP) k_plane_fwd_density(const double* __restrict__ phi, cplx<R>* __restrict__ out,
                                                           const cplx<R>* __restrict__ tw_g, GridDesc g,
                                                           double* __restrict__ partials, int maxb, Rotation rot) {
  OFDFT_GATE(g.gate);
  static_assert(plane_maxe<L, NTP>() <= 16, "plane too large for the in-place FFT registers");
  extern __shared__ __align__(16) char smem_raw[];
  Smem sm(smem_raw);
  cplx<R>* buf = sm.take<cplx<R>>((L / 2) * Lay<L>::RS);
  cplx<R>* tw = sm.take<cplx<R>>(L);
  double* red = sm.take<double>(NTP / 64);
  int i1, h;
  plane_half(blockIdx.x, g.n1, i1, h);
  const size_t base = (size_t)i1 * L * L;
  constexpr int CNT = L * L;
  const int e_lo = h * (CNT / 2), e_hi = e_lo + CNT / 2;   // this block's half of the plane's points
  const auto twv = twiddle_load<R, L>(tw_g);
  R* zr = reinterpret_cast<R*>(buf);
  double acc = 0.0;
  for (int c0 = 0; c0 < CNT; c0 += PCH * NTP) {
    double pv[PCH];
#pragma unroll
    for (int u = 0; u < PCH; ++u) pv[u] = phi[base + min(c0 + (int)threadIdx.x + u * NTP, CNT - 1)];
    if constexpr (ROT) {
      double dv_[PCH];
      const double ca = rot.cos_part(), sb = rot.sin_part();
#pragma unroll
      for (int u = 0; u < PCH; ++u) dv_[u] = rot.dir[base + min(c0 + (int)threadIdx.x + u * NTP, CNT - 1)];
#pragma unroll
      for (int u = 0; u < PCH; ++u) {
        pv[u] = ca * pv[u] + sb * dv_[u];
        const int e = c0 + threadIdx.x + u * NTP;
        if (e >= e_lo && e < e_hi) rot.phi_out[base + e] = pv[u];   // each half stores its points
      }
    }
#pragma unroll
    for (int u = 0; u < PCH; ++u) {
      const int e = c0 + threadIdx.x + u * NTP;
      if (e < CNT) {
        const int i2 = e / L, i3 = e - i2 * L;
        const double n = pv[u] * pv[u];
        if (e >= e_lo && e < e_hi) acc += n;
        zr[2 * Lay<L>::at(i2 >> 1, i3) + (i2 & 1)] = R(n);
      }
    }
  }
  twiddle_store<R, L>(tw, twv);
  __syncthreads();
  // the x3 transform needs every row; the x2 transform and the store take this half's k3 rows
  plane_x3_fwd_to_T_half<R, L, NTP>(buf, tw, h * (L / 4));
  plane_x2_fwd_store_half<R, L, NTP>(buf, tw, out, g, i1, h * (L / 4));
  double v[1] = {acc};
  block_sum<1, NTP>(v, red);
  if (threadIdx.x == 0) partials[SL_PHI2 * maxb + 2 * i1 + h] = v[0];
}

// F3: forward x3 and x2 transforms of real arrays (component blockIdx.y).
template <typename R, int L, int NTH>
__global__ void __launch_bounds__(NTH, sizeof(R) == 4 ? 8 : 4) k_plane_fwd_real(RealArr3 in, Arr3 out, const cplx<R>* __restrict__ tw_g,
                                                        GridDesc g) {
  OFDFT_GATE(g.gate);
  static_assert(plane_maxe<L, NTH>() <= 16, "plane too large for the in-place FFT registers");
  extern __shared__ __align__(16) char smem_raw[];
  Smem sm(smem_raw);
  cplx<R>* buf = sm.take<cplx<R>>((L / 2) * Lay<L>::RS);
  cplx<R>* tw = sm.take<cplx<R>>(L);
  const int i1 = blockIdx.x;
  constexpr int CNT = L * L;
  const R* src = reinterpret_cast<const R*>(in.p[blockIdx.y]) + (size_t)i1 * CNT;
  const auto twv = twiddle_load<R, L>(tw_g);
  R* zr = reinterpret_cast<R*>(buf);
  for (int c0 = 0; c0 < CNT; c0 += PCH * NTH) {
    R xv[PCH];
#pragma unroll
    for (int u = 0; u < PCH; ++u) xv[u] = src[min(c0 + (int)threadIdx.x + u * NTH, CNT - 1)];
#pragma unroll
    for (int u = 0; u < PCH; ++u) {
      const int e = c0 + threadIdx.x + u * NTH;
      if (e < CNT) {
        const int i2 = e / L, i3 = e - i2 * L;
        zr[2 * Lay<L>::at(i2 >> 1, i3) + (i2 & 1)] = xv[u];
      }
    }
  }
  twiddle_store<R, L>(tw, twv);
  __syncthreads();
  plane_x3_fwd_to_T<R, L, NTH>(buf, tw);
  plane_x2_fwd_store<R, L, NTH>(buf, tw, reinterpret_cast<cplx<R>*>(out.p[blockIdx.y]), g, i1);
}

// The minimiser's projected gradient g = 2 dv phi (v - mu), formed on the fly,
// forward x3 and x2 (the first half of the preconditioner P g).
template <typename R, int L>
__global__ void __launch_bounds__(NTP) k_plane_fwd_grad(const double* __restrict__ phi, const R* __restrict__ v,
                                                        const double* __restrict__ sc, double two_dv,
                                                        cplx<R>* __restrict__ out, const cplx<R>* __restrict__ tw_g,
                                                        GridDesc g) {
  OFDFT_GATE(g.gate);
  static_assert(plane_maxe<L, NTP>() <= 16, "plane too large for the in-place FFT registers");
  extern __shared__ __align__(16) char smem_raw[];
  Smem sm(smem_raw);
  cplx<R>* buf = sm.take<cplx<R>>((L / 2) * Lay<L>::RS);
  cplx<R>* tw = sm.take<cplx<R>>(L);
  const int i1 = blockIdx.x;
  const size_t base = (size_t)i1 * L * L;
  constexpr int CNT = L * L;
  const auto twv = twiddle_load<R, L>(tw_g);
  const double mu = sc[SC_MU];
  R* zr = reinterpret_cast<R*>(buf);
  for (int c0 = 0; c0 < CNT; c0 += PCH * NTP) {
    double pv[PCH];
    R vv[PCH];
#pragma unroll
    for (int u = 0; u < PCH; ++u) {
      const int e = min(c0 + (int)threadIdx.x + u * NTP, CNT - 1);
      pv[u] = phi[base + e];
      vv[u] = v[base + e];
    }
#pragma unroll
    for (int u = 0; u < PCH; ++u) {
      const int e = c0 + threadIdx.x + u * NTP;
      if (e < CNT) {
        const int i2 = e / L, i3 = e - i2 * L;
        zr[2 * Lay<L>::at(i2 >> 1, i3) + (i2 & 1)] = R(two_dv * pv[u] * (double(vv[u]) - mu));
      }
    }
  }
  twiddle_store<R, L>(tw, twv);
  __syncthreads();
  plane_x3_fwd_to_T<R, L, NTP>(buf, tw);
  plane_x2_fwd_store<R, L, NTP>(buf, tw, out, g, i1);
}

// I3: inverse x2 and x3 transforms into real arrays (component blockIdx.y).
template <typename R, int L, int NTH>
__global__ void __launch_bounds__(NTH, sizeof(R) == 4 ? 8 : 4) k_plane_inv_real(Arr3 in, RealArr3 out, const cplx<R>* __restrict__ tw_g,
                                                        GridDesc g) {
  OFDFT_GATE(g.gate);
  static_assert(plane_maxe<L, NTH>() <= 16, "plane too large for the in-place FFT registers");
  extern __shared__ __align__(16) char smem_raw[];
  Smem sm(smem_raw);
  cplx<R>* buf = sm.take<cplx<R>>((L / 2) * Lay<L>::RS);
  cplx<R>* tw = sm.take<cplx<R>>(L);
  const int i1 = blockIdx.x;
  constexpr int CNT = L * L;
  plane_load_T<R, L, NTH>(buf, tw, reinterpret_cast<const cplx<R>*>(in.p[blockIdx.y]), tw_g, g, i1);
  plane_inv<R, L, NTH>(buf, tw);
  R* dst = reinterpret_cast<R*>(out.p[blockIdx.y]) + (size_t)i1 * CNT;
  for (int e = threadIdx.x; e < CNT; e += NTH) dst[e] = plane_real<R, L>(buf, e);
}

// FI: inverse x2 and x3 transforms of the reciprocal-space potential, then
// v = v_loc + S + alpha (ftTF: the pointwise ftTF and XC here), sum n v and the
// per-plane partials (as k_rpass_final).
template <typename R, int L, bool TF, bool DT>
__global__ void __launch_bounds__(NTP) k_plane_final(const cplx<R>* __restrict__ D, const double* __restrict__ phi,
                                                     const R* __restrict__ vloc, R* __restrict__ vout,
                                                     const cplx<R>* __restrict__ tw_g, GridDesc g, EvalParams ep,
                                                     double* __restrict__ partials, int maxb, Slope sl) {
  OFDFT_GATE(g.gate);
  static_assert(plane_maxe<L, NTP>() <= 16, "plane too large for the in-place FFT registers");
  extern __shared__ __align__(16) char smem_raw[];
  Smem sm(smem_raw);
  cplx<R>* buf = sm.take<cplx<R>>((L / 2) * Lay<L>::RS);
  cplx<R>* tw = sm.take<cplx<R>>(L);
  double* red = sm.take<double>(kFinalSums * NTP / 64);
  int i1, h;
  plane_half(blockIdx.x, g.n1, i1, h);
  // this block's half: real rows i2 in [h L/2, (h + 1) L/2), i.e. points [h CNT/2, (h + 1) CNT/2)
  const size_t base = (size_t)i1 * L * L + (size_t)h * (L * L / 2);
  constexpr int CNT = L * L / 2;
  plane_load_T<R, L, NTP>(buf, tw, D, tw_g, g, i1);
  plane_inv_half<R, L, NTP>(buf, tw, h * (L / 4));
  const cplx<R>* hbuf = buf + h * (L / 4) * Lay<L>::RS;   // packed rows of this half
  double fs = 0.0, ts = 0.0, exc = 0.0, tsxc = 0.0, nv = 0.0, dt1 = 0.0, dt2 = 0.0;
  constexpr int CH = TF ? 2 : PCH;   // the inlined ftTF point is register-heavy
  for (int c0 = 0; c0 < CNT; c0 += CH * NTP) {
    double pv[CH], q[CH];
    R lv[CH];
#pragma unroll
    for (int u = 0; u < CH; ++u) {
      const int e = min(c0 + (int)threadIdx.x + u * NTP, CNT - 1);
      pv[u] = phi[base + e];
      if constexpr (!TF) lv[u] = vloc[base + e];
    }
    if constexpr (DT) {
      double p0[CH], dd[CH];
#pragma unroll
      for (int u = 0; u < CH; ++u) {
        const int e = min(c0 + (int)threadIdx.x + u * NTP, CNT - 1);
        p0[u] = sl.phi0[base + e];
        dd[u] = sl.dir[base + e];
      }
      const double ms = sl.ms_part(), mc = sl.mc_part();
#pragma unroll
      for (int u = 0; u < CH; ++u) q[u] = ms * p0[u] + mc * dd[u];
    }
#pragma unroll
    for (int u = 0; u < CH; ++u) {
      const int e = c0 + threadIdx.x + u * NTP;
      if (e >= CNT) continue;
      const double S = double(plane_real<R, L>(hbuf, e));
      const double p = pv[u];
      const double n = p * p;
      double vl;
      if constexpr (TF) {
        const double nf = n > kDensityFloor ? n : kDensityFloor;
        double f, vt, tsl;
        const double ln_n = ln_pos(nf);
        tf_point(nf, ln_n, ep.lt0, f, vt, tsl);
        vl = vt;
        fs += f;
        ts += tsl;
        xc_point<R>(ep.xc, n, ln_n, ep.lt0, vl, exc, tsxc);
      } else {
        vl = double(lv[u]);
      }
      const R vv = R(vl + S + ep.alpha_sum);
      vout[base + e] = vv;
      nv += n * double(vv);
      if constexpr (DT) {
        dt1 += p * double(vv) * q[u];
        dt2 += p * q[u];
      }
    }
  }
  constexpr int K = (TF ? 5 : 1) + (DT ? 2 : 0);
  double v[K];
  int slot[K];
  int k = 0;
  if constexpr (TF) {
    v[k] = fs; slot[k++] = SL_FS;
    v[k] = ts; slot[k++] = SL_TS;
    v[k] = exc; slot[k++] = SL_EXC;
    v[k] = tsxc; slot[k++] = SL_TSXC;
  }
  v[k] = nv; slot[k++] = SL_NV;
  if constexpr (DT) {
    v[k] = dt1; slot[k++] = SL_DT1;
    v[k] = dt2; slot[k++] = SL_DT2;
  }
  block_sum<K, NTP>(v, red);
  if (threadIdx.x == 0) {
#pragma unroll
    for (int m = 0; m < K; ++m) partials[slot[m] * maxb + 2 * i1 + h] = v[m];
  }
}

// ---------------------------------------------------------------- K4 plane form, fused
// Gradient functional on the plane passes, FP32 assembly: the inverse x2 and x3 transforms of
// the three grad n spectra of one i1 plane, then the pointwise functional and XC on the real
// rows they give, with W and v_loc stored; grad n itself stays on the CU.  The x2 inverse
// is split four ways by decimation in time over i2 mod 4 = q: with Q = L/4 and w = e^{-2 pi i/L},
//   y[4m + q] = sum_{k < Q} Y_q[k] e^{+2 pi i k m/Q},  Y_q[k] = conj(w)^{k q} sum_{s < 4} i^{s q} X[k + s Q],
// so each of the plane's four blocks runs Q-point transforms over its own rows and together
// they do the arithmetic of one full-plane pass (each reads the plane's spectrum; the four sit
// on one XCD, whose L2 serves all but the first read).  Blocks of IGG_NT threads, two per CU
// (the point functional's registers allow no more).
constexpr int IGG_NT = 512;

// Block b takes plane i1 and row class q; the four blocks of a plane are 8 block indices
// apart, so the round-robin dispatch over the 8 XCDs puts them on the same XCD.
__device__ __forceinline__ void plane_quarter(int b, int n1, int& i1, int& q) {
  if ((n1 & 7) == 0) {
    i1 = (b >> 5) * 8 + (b & 7);
    q = (b >> 3) & 3;
  } else {
    i1 = b >> 2;
    q = b & 3;
  }
}

// z multiplied by i^p
template <typename R>
__device__ __forceinline__ cplx<R> mul_ipow(cplx<R> z, int p) {
  switch (p & 3) {
    case 0: return z;
    case 1: return {-z.y, z.x};
    case 2: return {-z.x, -z.y};
    default: return {z.y, -z.x};
  }
}

template <int L>
struct InvGgaLds {
  static constexpr int H = L / 2, Q = L / 4, NP = Q / 2;
  static constexpr int ELEMS = (H * Lay<Q>::RS > NP * Lay<L>::RS) ? H * Lay<Q>::RS : NP * Lay<L>::RS;
};

// The four-way split inverse of one plane's half spectrum S (component rows S[k3][i1][.]) for
// row class q: on return buf holds the block's Q real rows packed in pairs (Lay<L> rows p),
// real row m (i2 = 4m + q) being Re (m even) or Im (m odd) of packed row m/2.  tw (L entries)
// and twq (Q entries) are written by the caller before the call; the first barrier here
// publishes them, and also orders this call's writes of buf after earlier reads of it.
template <typename R, int L, int NTH>
__device__ __forceinline__ void plane_inv_quarter(const cplx<R>* __restrict__ S, cplx<R>* buf, const cplx<R>* tw,
                                                  const cplx<R>* twq, size_t slab, size_t row0, int q, int tid) {
  constexpr int H = L / 2, Q = L / 4, NP = Q / 2;
  constexpr int NY = H * Q, MY = (NY + NTH - 1) / NTH;   // Y_q elements (k3 < H, k < Q), per thread
  constexpr int NZ = NP * L, MZ = (NZ + NTH - 1) / NTH;  // packed x3 rows' elements, per thread
  static_assert(L % 8 == 0 && MY <= 4 && MZ <= 4, "plane too large for the split inverse");
  // X[k + s Q] (s < 4) of this thread's Y_q elements: rows of the spectrum are read whole
  cplx<R> x[MY][4];
#pragma unroll
  for (int m = 0; m < MY; ++m) {
    const int e = min(tid + m * NTH, NY - 1);
    const int k3 = e / Q, k = e - k3 * Q;
    const cplx<R>* r = S + k3 * slab + row0 + k;
#pragma unroll
    for (int s = 0; s < 4; ++s) x[m][s] = r[s * Q];
  }
  __syncthreads();
#pragma unroll
  for (int m = 0; m < MY; ++m) {
    const int e = tid + m * NTH;
    if (e < NY) {
      const int k3 = e / Q, k = e - k3 * Q;
      cplx<R> y = x[m][0];
#pragma unroll
      for (int s = 1; s < 4; ++s) y = y + mul_ipow(x[m][s], s * q);
      buf[Lay<Q>::at(k3, k)] = q == 0 ? y : cmul(y, cconj(tw[k * q]));
    }
  }
  __syncthreads();
  // x2 inverse: Q-point transforms along k of the rows k3 (y_q[k3][m] in place)
  lds_fft_inplace<R, +1, Q, NTH, MY>(buf, twq, H, tid);
  // packed rows z_p[k] = A[k] + i B[k] of the block's real rows 2p and 2p + 1, over the
  // whole k range by Hermitian symmetry (Nyquist term zero)
  cplx<R> z[MZ];
#pragma unroll
  for (int m = 0; m < MZ; ++m) {
    const int it = tid + m * NTH;
    if (it < NZ) {
      const int p = it / L, k = it - p * L;
      cplx<R> A = {R(0), R(0)}, B = {R(0), R(0)};
      if (2 * k < L) {
        A = buf[Lay<Q>::at(k, 2 * p)];
        B = buf[Lay<Q>::at(k, 2 * p + 1)];
      } else if (2 * k > L) {
        A = cconj(buf[Lay<Q>::at(L - k, 2 * p)]);
        B = cconj(buf[Lay<Q>::at(L - k, 2 * p + 1)]);
      }
      z[m] = {A.x - B.y, A.y + B.x};
    }
  }
  __syncthreads();
#pragma unroll
  for (int m = 0; m < MZ; ++m) {
    const int it = tid + m * NTH;
    if (it < NZ) {
      const int p = it / L, k = it - p * L;
      buf[Lay<L>::at(p, k)] = z[m];
    }
  }
  __syncthreads();
  // x3 inverse of the packed rows
  int tid2 = tid;
  asm volatile("" : "+v"(tid2));
  lds_fft_inplace<R, +1, L, NTH, MZ>(buf, tw, NP, tid2);
}

template <typename R, int L, int XC>
__global__ void __launch_bounds__(IGG_NT, 4) k_plane_inv_gga(Arr3 in, const double* __restrict__ phi,
                                                             R* __restrict__ g0, R* __restrict__ g1,
                                                             R* __restrict__ g2, R* __restrict__ vloc,
                                                             const cplx<R>* __restrict__ tw_g, GridDesc g,
                                                             EvalParams ep, double* __restrict__ partials,
                                                             int maxb) {
  OFDFT_GATE(g.gate);
  constexpr int NTH = IGG_NT;
  constexpr int Q = L / 4;
  constexpr int NR = Q * L, MR = (NR + NTH - 1) / NTH;   // real points of the block, per thread
  static_assert(MR <= 8, "plane too large for the fused pass");
  __shared__ cplx<R> buf[InvGgaLds<L>::ELEMS];
  __shared__ cplx<R> tw[L];
  __shared__ cplx<R> twq[Q];
  __shared__ double red[4 * NTH / 64];
  // grad n of the block's points: components 0 and 1 here, component 2 read from buf, which
  // holds the last transform's real rows (registers would cap the kernel below its two blocks
  // per CU)
  __shared__ R greal[2][NR];
  int i1, q;
  plane_quarter(blockIdx.x, g.n1, i1, q);
  const int tid = threadIdx.x;
  const size_t slab = (size_t)g.n1 * L;   // elements per k3 of the spectrum S[k3][i1][k2]
  const size_t row0 = (size_t)i1 * L;
  const size_t base = (size_t)i1 * L * L;
  if (tid < L) tw[tid] = tw_g[tid];
  if (tid < Q) twq[tid] = tw_g[4 * tid];
  double pv[MR];
#pragma unroll
  for (int a = 0; a < 3; ++a) {
    if (a == 2) {
#pragma unroll
      for (int u = 0; u < MR; ++u) {
        const int e = min(tid + u * NTH, NR - 1);
        const int m = e / L, i3 = e - m * L;
        pv[u] = phi[base + (size_t)(4 * m + q) * L + i3];
      }
    }
    // (its first barrier: the twiddles are in place, every thread has read the previous rows)
    plane_inv_quarter<R, L, NTH>(reinterpret_cast<const cplx<R>*>(in.p[a]), buf, tw, twq, slab, row0, q, tid);
    if (a < 2) {
      // each thread keeps the points it takes in the pointwise loop: no barrier needed
#pragma unroll
      for (int u = 0; u < MR; ++u) {
        const int e = tid + u * NTH;
        if (e < NR) {
          const int m = e / L, i3 = e - m * L;
          const cplx<R> v = buf[Lay<L>::at(m >> 1, i3)];
          greal[a][e] = (m & 1) ? v.y : v.x;
        }
      }
    }
  }
  const EnhParams enh{(int)ep.enh_kind, ep.enh_c1, ep.enh_a1};
  double fs = 0.0, ts = 0.0, exc = 0.0, tsxc = 0.0;
#pragma unroll
  for (int u = 0; u < MR; ++u) {
    const int e = tid + u * NTH;
    if (e < NR) {
      const int m = e / L, i3 = e - m * L;
      const size_t i = base + (size_t)(4 * m + q) * L + i3;
      const cplx<R> v = buf[Lay<L>::at(m >> 1, i3)];
      R gx = greal[0][e], gy = greal[1][e], gz = (m & 1) ? v.y : v.x;
      vloc[i] = gga_xc_at<R, XC>(pv[u], gx, gy, gz, ep.lt0, enh, fs, ts, exc, tsxc);
      g0[i] = gx;
      g1[i] = gy;
      g2[i] = gz;
    }
  }
  double v[4] = {fs, ts, exc, tsxc};
  block_sum<4, NTH>(v, red);
  if (tid == 0) {
    partials[SL_FS * maxb + blockIdx.x] = v[0];
    partials[SL_TS * maxb + blockIdx.x] = v[1];
    partials[SL_EXC * maxb + blockIdx.x] = v[2];
    partials[SL_TSXC * maxb + blockIdx.x] = v[3];
  }
}

// Final pass of the gradient functionals on the same four-way split (mixed precision, planes of
// 32, 64 or 128): the inverse x2 and x3 of D for the block's rows i2 = 4m + q, then
// v = v_loc + S + alpha_sum and the sums of k_plane_final (n v; a trial's phi_t v_t q and
// phi_t q).  One slot of partial sums per block.
template <typename R, int L, bool DT>
__global__ void __launch_bounds__(IGG_NT, 4) k_plane_final_q(const cplx<R>* __restrict__ D,
                                                             const double* __restrict__ phi,
                                                             const R* __restrict__ vloc, R* __restrict__ vout,
                                                             const cplx<R>* __restrict__ tw_g, GridDesc g,
                                                             EvalParams ep, double* __restrict__ partials,
                                                             int maxb, Slope sl) {
  OFDFT_GATE(g.gate);
  constexpr int NTH = IGG_NT;
  constexpr int Q = L / 4;
  constexpr int NR = Q * L, MR = (NR + NTH - 1) / NTH;   // real points of the block, per thread
  static_assert(MR <= 8, "plane too large for the split final pass");
  __shared__ cplx<R> buf[InvGgaLds<L>::ELEMS];
  __shared__ cplx<R> tw[L];
  __shared__ cplx<R> twq[Q];
  constexpr int K = DT ? 3 : 1;
  __shared__ double red[K * NTH / 64];
  int i1, q;
  plane_quarter(blockIdx.x, g.n1, i1, q);
  const int tid = threadIdx.x;
  const size_t base = (size_t)i1 * L * L;
  if (tid < L) tw[tid] = tw_g[tid];
  if (tid < Q) twq[tid] = tw_g[4 * tid];
  plane_inv_quarter<R, L, NTH>(D, buf, tw, twq, (size_t)g.n1 * L, (size_t)i1 * L, q, tid);
  double pv[MR], qv[MR];
  R lv[MR];
#pragma unroll
  for (int u = 0; u < MR; ++u) {
    const int e = min(tid + u * NTH, NR - 1);
    const int m = e / L, i3 = e - m * L;
    const size_t i = base + (size_t)(4 * m + q) * L + i3;
    pv[u] = phi[i];
    lv[u] = vloc[i];
    if constexpr (DT) qv[u] = sl.ms_part() * sl.phi0[i] + sl.mc_part() * sl.dir[i];
  }
  double nv = 0.0, dt1 = 0.0, dt2 = 0.0;
#pragma unroll
  for (int u = 0; u < MR; ++u) {
    const int e = tid + u * NTH;
    if (e < NR) {
      const int m = e / L, i3 = e - m * L;
      const size_t i = base + (size_t)(4 * m + q) * L + i3;
      const cplx<R> z = buf[Lay<L>::at(m >> 1, i3)];
      const double S = double((m & 1) ? z.y : z.x);
      const double p = pv[u];
      const double n = p * p;
      const R vv = R(double(lv[u]) + S + ep.alpha_sum);
      vout[i] = vv;
      nv += n * double(vv);
      if constexpr (DT) {
        dt1 += p * double(vv) * qv[u];
        dt2 += p * qv[u];
      }
    }
  }
  double v[K];
  v[0] = nv;
  if constexpr (DT) {
    v[1] = dt1;
    v[2] = dt2;
  }
  block_sum<K, NTH>(v, red);
  if (tid == 0) {
    partials[SL_NV * maxb + blockIdx.x] = v[0];
    if constexpr (DT) {
      partials[SL_DT1 * maxb + blockIdx.x] = v[1];
      partials[SL_DT2 * maxb + blockIdx.x] = v[2];
    }
  }
}

// Density pass split by the parity r of k3 (mixed precision, planes of 32, 64 or 128): both
// blocks of a plane form the packed rows z_p = n_{2p} + i n_{2p+1} of the whole plane, and block
// r keeps the x3 outputs k3 = 2j + r by decimation in frequency,
//   Z_p[2j + r] = sum_{m < H} (z_p[m] + (-1)^r z_p[m + H]) w^{r m} e^{-2 pi i j m/H},  H = L/2,
// so each block runs H-point transforms on its own half of the frequencies.  The Hermitian
// partner L - k3 of k3 has the same parity, so the half spectra of the two real rows separate
// within the block; the x2 transform of its L/4 k3 rows follows.  Together the two blocks do the
// butterflies of one full-plane pass (the split density pass above repeats the x3 transform).
// Block r sums phi^2 (and stores a trial's phi_t) on the points i3 in [r H, (r + 1) H).
template <int L>
struct FwdParLds {
  static constexpr int H = L / 2;
  static constexpr int ELEMS = (H * Lay<H>::RS > (L / 4) * Lay<L>::RS) ? H * Lay<H>::RS : (L / 4) * Lay<L>::RS;
};

template <typename R, int L, bool ROT>
__global__ void __launch_bounds__(NTP) k_plane_fwd_density_par(const double* __restrict__ phi,
                                                               cplx<R>* __restrict__ out,
                                                               const cplx<R>* __restrict__ tw_g, GridDesc g,
                                                               double* __restrict__ partials, int maxb,
                                                               Rotation rot) {
  OFDFT_GATE(g.gate);
  constexpr int H = L / 2, QK = L / 4;                   // x3 outputs per block: k3 = 2j + r, j < QK
  constexpr int NE = H * H, ME = (NE + NTP - 1) / NTP;   // (p, m) elements, per thread
  constexpr int NU = H * QK, MU = (NU + NTP - 1) / NTP;  // (p, j) unpack items, per thread
  constexpr int NT2 = QK * L, MT = (NT2 + NTP - 1) / NTP;
  static_assert(L % 8 == 0 && ME <= 4 && MU <= 2 && MT <= 4, "plane too large for the parity-split pass");
  __shared__ cplx<R> buf[FwdParLds<L>::ELEMS];
  __shared__ cplx<R> tw[L];
  __shared__ cplx<R> twh[H];
  __shared__ double red[NTP / 64];
  int i1, r;
  plane_half(blockIdx.x, g.n1, i1, r);
  const int tid = threadIdx.x;
  const size_t base = (size_t)i1 * L * L;
  // amplitudes of rows 2p, 2p + 1 at columns m and m + H
  double pa[ME][4];
#pragma unroll
  for (int u = 0; u < ME; ++u) {
    const int e = min(tid + u * NTP, NE - 1);
    const int pp = e / H, m = e - pp * H;
    const size_t i0 = base + (size_t)(2 * pp) * L + m;
    pa[u][0] = phi[i0];
    pa[u][1] = phi[i0 + H];
    pa[u][2] = phi[i0 + L];
    pa[u][3] = phi[i0 + L + H];
  }
  if constexpr (ROT) {
    const double ca = rot.cos_part(), sb = rot.sin_part();
#pragma unroll
    for (int u = 0; u < ME; ++u) {
      const int e = min(tid + u * NTP, NE - 1);
      const int pp = e / H, m = e - pp * H;
      const size_t i0 = base + (size_t)(2 * pp) * L + m;
      double dv[4] = {rot.dir[i0], rot.dir[i0 + H], rot.dir[i0 + L], rot.dir[i0 + L + H]};
#pragma unroll
      for (int t = 0; t < 4; ++t) pa[u][t] = ca * pa[u][t] + sb * dv[t];
      if (tid + u * NTP < NE) {   // each block stores the points of its column half
        const size_t j0 = i0 + (size_t)r * H;
        rot.phi_out[j0] = pa[u][r];
        rot.phi_out[j0 + L] = pa[u][2 + r];
      }
    }
  }
  if (tid < L) tw[tid] = tw_g[tid];
  if (tid < H) twh[tid] = tw_g[2 * tid];
  __syncthreads();
  double acc = 0.0;
#pragma unroll
  for (int u = 0; u < ME; ++u) {
    const int e = tid + u * NTP;
    if (e < NE) {
      const int pp = e / H, m = e - pp * H;
      double n[4];
#pragma unroll
      for (int t = 0; t < 4; ++t) n[t] = pa[u][t] * pa[u][t];
      acc += n[r] + n[2 + r];
      // z_p[m] = n(2p, m) + i n(2p + 1, m), z_p[m + H] likewise
      const cplx<R> zl = {R(n[0]), R(n[2])}, zh = {R(n[1]), R(n[3])};
      const cplx<R> zc = r == 0 ? zl + zh : cmul(zl - zh, tw[m]);
      buf[Lay<H>::at(pp, m)] = zc;
    }
  }
  __syncthreads();
  // x3: H-point forward transforms of the packed rows, Zr[p][j] = Z_p[2j + r]
  lds_fft_inplace<R, -1, H, NTP, ME>(buf, twh, H, tid);
  // separate the two real rows of each packed row: X_{2p}[k] = (Z[k] + conj Z[L - k]) / 2,
  // X_{2p+1}[k] = (Z[k] - conj Z[L - k]) / (2i), with L - k = 2 j' + r, j' = (H - j - r) mod H
  cplx<R> xa[MU], xb[MU];
#pragma unroll
  for (int u = 0; u < MU; ++u) {
    const int it = tid + u * NTP;
    if (it < NU) {
      const int pp = it / QK, j = it - pp * QK;
      const int jc = (H - j - r) & (H - 1);
      const cplx<R> z = buf[Lay<H>::at(pp, j)];
      const cplx<R> zc = cconj(buf[Lay<H>::at(pp, jc)]);
      xa[u] = {R(0.5) * (z.x + zc.x), R(0.5) * (z.y + zc.y)};
      xb[u] = {R(0.5) * (z.y - zc.y), R(-0.5) * (z.x - zc.x)};
    }
  }
  __syncthreads();
#pragma unroll
  for (int u = 0; u < MU; ++u) {
    const int it = tid + u * NTP;
    if (it < NU) {
      const int pp = it / QK, j = it - pp * QK;
      buf[Lay<L>::at(j, 2 * pp)] = xa[u];
      buf[Lay<L>::at(j, 2 * pp + 1)] = xb[u];
    }
  }
  __syncthreads();
  // x2 forward of the block's QK k3 rows, stored as S[k3][i1][k2]
  int tid2 = tid;
  asm volatile("" : "+v"(tid2));
  lds_fft_inplace<R, -1, L, NTP, MT>(buf, tw, QK, tid2);
  const size_t plane = (size_t)g.n1 * L;
#pragma unroll
  for (int u = 0; u < MT; ++u) {
    const int e = tid + u * NTP;
    if (e < NT2) {
      const int j = e / L, k2 = e - j * L;
      out[(size_t)(2 * j + r) * plane + (size_t)i1 * L + k2] = buf[Lay<L>::at(j, k2)];
    }
  }
  double v[1] = {acc};
  block_sum<1, NTP>(v, red);
  if (tid == 0) partials[SL_PHI2 * maxb + 2 * i1 + r] = v[0];
}

// ---------------------------------------------------------------- K7: scalar reduction
constexpr int RED_NT = 64 * SL_COUNT;   // one wavefront per slot

__global__ void __launch_bounds__(RED_NT) k_reduce_scalars(const double* __restrict__ partials, int maxb,
                                                           ReduceParams rp, double* __restrict__ sc, Publish pub) {
  OFDFT_GATE(rp.gate);
  __shared__ double raw[SL_COUNT];
  __shared__ double out[SC_COUNT];
  reduce_scalars<RED_NT>(partials, maxb, rp, sc, pub, raw, out);
}

// Generic small readback (dev_read): one wavefront.
__global__ void __launch_bounds__(64) k_publish(const double* __restrict__ src, int n, Publish pub) {
  __shared__ double v[kMapDoubles];
  if ((int)threadIdx.x < n) v[threadIdx.x] = src[threadIdx.x];
  __syncthreads();
  publish(pub, v, n, threadIdx.x);
}

// ---------------------------------------------------------------- vector reductions
constexpr int VEC_BLOCKS = 512;

template <int K, class Op>
__global__ void __launch_bounds__(NT) k_vec(long long n, Op op, double* __restrict__ part,
                                             const double* __restrict__ gate) {
  OFDFT_GATE(gate);
  __shared__ double red[(K > 0 ? K : 1) * NT / 64];
  double acc[K > 0 ? K : 1];
#pragma unroll
  for (int k = 0; k < (K > 0 ? K : 1); ++k) acc[k] = 0.0;
  for (long long i = (long long)blockIdx.x * NT + threadIdx.x; i < n; i += (long long)gridDim.x * NT) op(i, acc);
  if constexpr (K > 0) {
    block_sum<K>(acc, red);
    if (threadIdx.x == 0) {
#pragma unroll
      for (int k = 0; k < K; ++k) part[k * gridDim.x + blockIdx.x] = acc[k];
    }
  }
}

template <int K>
__global__ void __launch_bounds__(NT) k_vec_final(const double* __restrict__ part, int nb, double* __restrict__ out) {
  __shared__ double red[NT / 64];
  for (int k = 0; k < K; ++k) {
    double a = 0.0;
    for (int i = threadIdx.x; i < nb; i += NT) a += part[k * nb + i];
    double v[1] = {a};
    block_sum<1>(v, red);
    if (threadIdx.x == 0) out[k] = v[0];
  }
}

// The gradient dots of a CG step reduced into sc[SC_DOT0..], then the step's
// coefficients: c_z = z.phi / phi.phi (preconditioned) and
// beta = max(0, (z.g - (z.g_old - c_z phi.g_old)) / gg_prev) (Polak-Ribiere+).
struct CgCoef {
  int pcg, have_prev;
  double gg_prev, dv;
  const double* st;   // graph mode: have_prev and gg_prev come from the device CG state
  const double* gate;
};

template <int K>
__global__ void __launch_bounds__(NT) k_cg_dots_final(const double* __restrict__ part, int nb,
                                                      double* __restrict__ sc, CgCoef cf) {
  OFDFT_GATE(cf.gate);
  if (cf.st) {
    cf.have_prev = cf.st[CG_HAVE_PREV] != 0.0;
    cf.gg_prev = cf.st[CG_GG_PREV];
  }
  __shared__ double red[NT / 64];
  double dots[K];
  for (int k = 0; k < K; ++k) {
    double a = 0.0;
    for (int i = threadIdx.x; i < nb; i += NT) a += part[k * nb + i];
    double v[1] = {a};
    block_sum<1>(v, red);
    dots[k] = v[0];
  }
  if (threadIdx.x == 0) {
    for (int k = 0; k < K; ++k) sc[SC_DOT0 + k] = dots[k];
    const double cz = (cf.pcg && K >= 5) ? dots[2] / (sc[SC_NE] / cf.dv) : 0.0;
    double beta = 0.0;
    if (cf.have_prev) {
      const double cross = (cf.pcg && K >= 5) ? dots[1] - cz * dots[K >= 5 ? 4 : 0] : dots[1];
      beta = fmax(0.0, (dots[0] - cross) / cf.gg_prev);
    }
    sc[SC_BETA] = beta;
    sc[SC_CZ] = cz;
  }
}

// Direction dots d.d, d.g of a CG step, then the first line-search angle along d
// and its rotation/slope coefficients (dF0 = r d.g / |d|): theta = -dF0 / kappa with
// kappa the curvature d2F/dtheta2 measured by the previous line search, else
// 2 (F_prev - F) / (-dF0) when a previous step decreased F, clamped to [1e-6, 0.3];
// 0.05 without either.
struct TrialCoef {
  double F_prev;
  int have_prev;
  double r, dv, kappa;
  const double* st;   // graph mode: F_prev, have_prev and kappa come from the device CG state
  const double* gate;
};

__global__ void __launch_bounds__(NT) k_dir_final(const double* __restrict__ part, int nb, double* __restrict__ sc,
                                                  TrialCoef tc) {
  OFDFT_GATE(tc.gate);
  if (tc.st) {
    tc.F_prev = tc.st[CG_F_PREV];
    tc.have_prev = tc.st[CG_HAVE_PREV] != 0.0;
    tc.kappa = tc.st[CG_KAPPA];
  }
  __shared__ double red[NT / 64];
  double dots[2];
  for (int k = 0; k < 2; ++k) {
    double a = 0.0;
    for (int i = threadIdx.x; i < nb; i += NT) a += part[k * nb + i];
    double v[1] = {a};
    block_sum<1>(v, red);
    dots[k] = v[0];
  }
  if (threadIdx.x == 0) {
    sc[SC_DD] = dots[0];
    sc[SC_DG] = dots[1];
    const double dn = sqrt(dots[0]);
    const double dF0 = tc.r * dots[1] / dn;
    const double F = sc[SC_FTOT];
    double th = 0.05;
    if (tc.kappa > 0.0 && dF0 < 0.0) th = fmin(fmax(-dF0 / tc.kappa, 1e-6), 0.3);
    else if (tc.have_prev && dF0 < 0.0 && tc.F_prev > F) th = fmin(fmax(2.0 * (tc.F_prev - F) / (-dF0), 1e-6), 0.3);
    if (tc.st && tc.st[CG_THCAP] > 0.0) th = fmin(th, tc.st[CG_THCAP]);   // after a failed line search
    const double ratio = tc.r / sqrt(sc[SC_NE] / tc.dv);
    const double ct = cos(th), st = sin(th);
    sc[SC_TH1] = th;
    sc[SC_CA] = ct * ratio;
    sc[SC_SB] = st * tc.r / dn;
    sc[SC_MS] = -st * ratio;
    sc[SC_MC] = ct * tc.r / dn;
  }
}

// g = 2 dv phi (v - mu): dots g.g, g.gprev, g.d and sum n (v - mu)^2
// st (graph mode): gprev and d count only while the device CG state has a previous step.
template <typename R>
struct OpGradDots {
  const double* phi; const R* v; const double* sc; const double* gprev; const double* d; double two_dv;
  const double* st;
  __device__ void operator()(long long i, double* acc) const {
    const bool prev = !st || st[CG_HAVE_PREV] != 0.0;
    const double mu = sc[SC_MU];
    const double p = phi[i];
    const double dvm = double(v[i]) - mu;
    const double gi = two_dv * p * dvm;
    acc[0] += gi * gi;
    acc[1] += (gprev && prev) ? gi * gprev[i] : 0.0;
    acc[2] += (d && prev) ? gi * d[i] : 0.0;
    acc[3] += p * p * dvm * dvm;
  }
};

// Preconditioned dots: z = P g = g + w with w = ((P - 1) g) from the FFT passes
// (held in R); g.g is not needed, z.g takes its place.
template <typename R>
struct OpPrecDots {
  const double* phi; const R* v; const R* w; const double* sc; const double* gprev; double two_dv;
  const double* st;
  __device__ void operator()(long long i, double* acc) const {
    const bool prev = gprev && (!st || st[CG_HAVE_PREV] != 0.0);
    const double mu = sc[SC_MU];
    const double p = phi[i];
    const double dvm = double(v[i]) - mu;
    const double gi = two_dv * p * dvm;
    const double zi = gi + double(w[i]);
    acc[0] += zi * gi;
    acc[1] += prev ? zi * gprev[i] : 0.0;
    acc[2] += zi * p;
    acc[3] += p * p * dvm * dvm;
    acc[4] += prev ? p * gprev[i] : 0.0;
  }
};

// d = -(z - cz phi) + beta (d - cproj phi), z = g + w; gprev = g; dots d.d and d.g.
// beta and cz are the device values sc[SC_BETA], sc[SC_CZ] (beta = 0 on a restart).
template <typename R>
struct OpPrecDirection {
  const double* phi; const R* v; const R* w; const double* sc; double* gprev; double* d;
  double two_dv, cproj; int restart;
  const double* st;   // graph mode: cproj from the device CG state
  __device__ void operator()(long long i, double* acc) const {
    const double beta = restart ? 0.0 : sc[SC_BETA], cz = sc[SC_CZ];
    const double cproj = st ? st[CG_CPROJ] : this->cproj;
    const double p = phi[i];
    const double gi = two_dv * p * (double(v[i]) - sc[SC_MU]);
    // with beta = 0 the previous direction is not read: before the first step it has never
    // been written (a fresh allocation may hold non-finite bit patterns, and 0 * NaN = NaN)
    const double di = -(gi + double(w[i]) - cz * p) + (beta != 0.0 ? beta * (d[i] - cproj * p) : 0.0);
    d[i] = di;
    gprev[i] = gi;
    acc[0] += di * di;
    acc[1] += di * gi;
  }
};

// d = -g + beta (d - c phi); gprev = g; dots d.d and d.g.  beta from the host, or
// the device value sc[SC_BETA] when dev_beta is set.
template <typename R>
struct OpDirection {
  const double* phi; const R* v; const double* sc; double* gprev; double* d; double two_dv, beta_host, cproj;
  int dev_beta;
  const double* st;   // graph mode: cproj from the device CG state
  __device__ void operator()(long long i, double* acc) const {
    const double beta = dev_beta ? sc[SC_BETA] : beta_host;
    const double cproj = st ? st[CG_CPROJ] : this->cproj;
    const double p = phi[i];
    const double gi = two_dv * p * (double(v[i]) - sc[SC_MU]);
    // with beta = 0 the previous direction is not read (see OpPrecDirection)
    const double di = -gi + (beta != 0.0 ? beta * (d[i] - cproj * p) : 0.0);
    d[i] = di;
    gprev[i] = gi;
    acc[0] += di * di;
    acc[1] += di * gi;
  }
};

struct OpRotate {
  double* dst; const double* phi; const double* dir; double ca, sb;
  __device__ void operator()(long long i, double*) const { dst[i] = ca * phi[i] + sb * dir[i]; }
};

// dF/dtheta = g_t . (ms phi + mc d)
template <typename R>
struct OpDtheta {
  const double* phi_t; const R* v_t; const double* sc_t; const double* phi; const double* d;
  double two_dv, ms, mc;
  __device__ void operator()(long long i, double* acc) const {
    const double gt = two_dv * phi_t[i] * (double(v_t[i]) - sc_t[SC_MU]);
    acc[0] += gt * (ms * phi[i] + mc * d[i]);
  }
};

// out += sign * 2 dv phi_t v_t  (unconstrained gradient)
template <typename R>
struct OpFullGradAcc {
  double* out; const double* phi_t; const R* v_t; double two_dv, sign; int init;
  __device__ void operator()(long long i, double*) const {
    const double gfull = sign * two_dv * phi_t[i] * double(v_t[i]);
    out[i] = init ? gfull : out[i] + gfull;
  }
};

struct OpDot {
  const double* a; const double* b;
  __device__ void operator()(long long i, double* acc) const { acc[0] += a[i] * b[i]; }
};

struct OpAxpby {
  double* y; const double* x; double a, b;
  __device__ void operator()(long long i, double*) const { y[i] = (a == 0.0 ? 0.0 : a * y[i]) + b * x[i]; }
};

// dst = c0 x0 + c1 x1 + c2 x2; dot dst.dst
struct OpCombine3 {
  double* dst; const double* x0; const double* x1; const double* x2; double c0, c1, c2;
  __device__ void operator()(long long i, double* acc) const {
    double y = c0 * x0[i] + c1 * x1[i];
    if (x2) y += c2 * x2[i];
    dst[i] = y;
    acc[0] += y * y;
  }
};

// hs = hs * inv2e - c phi - mu_term s, with c chosen later; first pass: hs *= inv2e; dot hs.phi
struct OpHessScale {
  double* hs; const double* phi; double inv2e;
  __device__ void operator()(long long i, double* acc) const {
    const double h = hs[i] * inv2e;
    hs[i] = h;
    acc[0] += h * phi[i];
  }
};

// ---------------------------------------------------------------- ions: phase tables, structure factor, forces
__global__ void __launch_bounds__(NT) k_phase_tables(int nat, const double* __restrict__ frac, GridDesc g,
                                                     double2* __restrict__ tab) {
  const int M = g.n1 + g.n2 + g.n3h;
  const long long total = (long long)nat * M;
  for (long long idx = (long long)blockIdx.x * NT + threadIdx.x; idx < total; idx += (long long)gridDim.x * NT) {
    const int I = (int)(idx / M), j = (int)(idx - (long long)I * M);
    int axis, m;
    if (j < g.n1) { axis = 0; m = signed_freq(j, g.n1); }
    else if (j < g.n1 + g.n2) { axis = 1; m = signed_freq(j - g.n1, g.n2); }
    else { axis = 2; m = j - g.n1 - g.n2; }
    double s, c;
    sincospi(-2.0 * m * frac[3 * I + axis], &s, &c);
    tab[idx] = make_double2(c, s);
  }
}

__device__ __forceinline__ double2 zmul(double2 a, double2 b) {
  return make_double2(a.x * b.x - a.y * b.y, a.x * b.y + a.y * b.x);
}

// form factor v_I(q) = Z_I a(q) + b(q) of the local pseudopotential (q > 0)
__device__ __forceinline__ void form_ab(const LppParams& lp, double q, double volume, double& a, double& b) {
  const double pre = -kFourPi / (volume * q * q);
  if (lp.kind == 0) {
    a = pre * exp(-0.25 * q * q * lp.rc * lp.rc);
    b = 0.0;
  } else {
    double s, c;
    sincos(q * lp.rc, &s, &c);
    const double x = q / lp.qc;
    const double x2 = x * x;
    const double f = exp(-x2 * x2 * x2);
    a = pre * c * f;
    b = pre * (-lp.A * lp.rc * c + lp.A / q * s) * f;
  }
}

template <typename R>
__global__ void __launch_bounds__(NT) k_structure_factor(int nat, const double* __restrict__ Z,
                                                         const double2* __restrict__ tab, GridDesc g, LppParams lp,
                                                         cplx<R>* __restrict__ vext, double2* __restrict__ sfac) {
  const int M = g.n1 + g.n2 + g.n3h;
  const long long plane = (long long)g.n1 * g.n2;
  for (long long gi = (long long)blockIdx.x * NT + threadIdx.x; gi < g.NS; gi += (long long)gridDim.x * NT) {
    const int k3 = (int)(gi / plane);
    const long long rem = gi - k3 * plane;
    const int k1 = (int)(rem / g.n2), k2 = (int)(rem - (long long)k1 * g.n2);
    double gx, gy, gz;
    const bool keep = gvec(g, k1, k2, k3, gx, gy, gz);
    const double G2 = gx * gx + gy * gy + gz * gz;
    double2 out = make_double2(0.0, 0.0);
    double2 sz = make_double2(0.0, 0.0), s1 = make_double2(0.0, 0.0);
    if (keep && G2 > 0.0) {
      double a, b;
      form_ab(lp, sqrt(G2), g.volume, a, b);
      for (int I = 0; I < nat; ++I) {
        const double2* t = tab + (size_t)I * M;
        const double2 e = zmul(zmul(t[k1], t[g.n1 + k2]), t[g.n1 + g.n2 + k3]);
        sz.x += Z[I] * e.x;
        sz.y += Z[I] * e.y;
        s1.x += e.x;
        s1.y += e.y;
      }
      out = make_double2(a * sz.x + b * s1.x, a * sz.y + b * s1.y);
    }
    vext[gi] = cplx<R>{R(out.x), R(out.y)};
    sfac[gi] = sz;
    sfac[g.NS + gi] = s1;
  }
}

// Reciprocal-space Ewald energy from the stored structure factor S_Z, per block:
// sum over the half spectrum of w exp(-G^2/4a^2)/G^2 |S_Z|^2 (times 2 pi/V on the host).
__global__ void __launch_bounds__(NT) k_ewald_recip(const double2* __restrict__ sfac, GridDesc g, double split,
                                                    double* __restrict__ part) {
  __shared__ double red[NT / 64];
  const long long plane = (long long)g.n1 * g.n2;
  const double q4 = 0.25 / (split * split);
  double acc[1] = {0.0};
  for (long long gi = (long long)blockIdx.x * NT + threadIdx.x; gi < g.NS; gi += (long long)gridDim.x * NT) {
    const int k3 = (int)(gi / plane);
    const long long rem = gi - k3 * plane;
    const int k1 = (int)(rem / g.n2), k2 = (int)(rem - (long long)k1 * g.n2);
    double gx, gy, gz;
    const bool keep = gvec(g, k1, k2, k3, gx, gy, gz);
    const double G2 = gx * gx + gy * gy + gz * gz;
    if (!keep || G2 == 0.0) continue;
    const double2 sz = sfac[gi];
    acc[0] += ((k3 == 0) ? 1.0 : 2.0) * exp(-G2 * q4) / G2 * (sz.x * sz.x + sz.y * sz.y);
  }
  block_sum<1>(acc, red);
  if (threadIdx.x == 0) part[blockIdx.x] = acc[0];
}

// Coefficient of conj(S_Z) that adds the reciprocal Ewald force to the
// electron-ion force sums: w (4 pi / V^2) exp(-G^2/4a^2)/G^2.
__device__ __forceinline__ double ewald_force_coef(double wk, double G2, double volume, double split) {
  return wk * kFourPi / (volume * volume) * exp(-G2 * 0.25 / (split * split)) / G2;
}

constexpr int FORCE_IONS = 8;

// F_I partial sums: sum_G w G Im[conj(n(G)) e^{-iG.R_I}] (Z_I a + b)
template <typename R>
__global__ void __launch_bounds__(NT) k_forces(int nat, const double* __restrict__ Z, const double2* __restrict__ tab,
                                               const cplx<R>* __restrict__ nhat, const double2* __restrict__ sfac,
                                               double split, GridDesc g, LppParams lp, double* __restrict__ part) {
  __shared__ double red[3 * FORCE_IONS * NT / 64];
  const int M = g.n1 + g.n2 + g.n3h;
  const long long plane = (long long)g.n1 * g.n2;
  const int I0 = blockIdx.y * FORCE_IONS;
  double acc[3 * FORCE_IONS];
#pragma unroll
  for (int k = 0; k < 3 * FORCE_IONS; ++k) acc[k] = 0.0;
  for (long long gi = (long long)blockIdx.x * NT + threadIdx.x; gi < g.NS; gi += (long long)gridDim.x * NT) {
    const int k3 = (int)(gi / plane);
    const long long rem = gi - k3 * plane;
    const int k1 = (int)(rem / g.n2), k2 = (int)(rem - (long long)k1 * g.n2);
    double gx, gy, gz;
    const bool keep = gvec(g, k1, k2, k3, gx, gy, gz);
    const double G2 = gx * gx + gy * gy + gz * gz;
    if (!keep || G2 == 0.0) continue;
    double a, b;
    form_ab(lp, sqrt(G2), g.volume, a, b);
    const double wk = (k3 == 0) ? 1.0 : 2.0;
    const cplx<R> nh = nhat[gi];
    const double cx = wk * double(nh.x), cy = -wk * double(nh.y);   // w conj(n)
    // Z-proportional part: w conj(n) a plus the Ewald term; the rest: w conj(n) b
    const double ke = ewald_force_coef(wk, G2, g.volume, split);
    const double2 sz = sfac[gi];
    const double pzx = cx * a + ke * sz.x, pzy = cy * a - ke * sz.y, pbx = cx * b, pby = cy * b;
#pragma unroll
    for (int j = 0; j < FORCE_IONS; ++j) {
      const int I = I0 + j;
      if (I < nat) {
        const double2* t = tab + (size_t)I * M;
        const double2 e = zmul(zmul(t[k1], t[g.n1 + k2]), t[g.n1 + g.n2 + k3]);
        const double im = Z[I] * (pzx * e.y + pzy * e.x) + (pbx * e.y + pby * e.x);
        acc[3 * j + 0] += gx * im;
        acc[3 * j + 1] += gy * im;
        acc[3 * j + 2] += gz * im;
      }
    }
  }
  block_sum<3 * FORCE_IONS>(acc, red);
  if (threadIdx.x == 0) {
    for (int j = 0; j < FORCE_IONS; ++j) {
      const int I = I0 + j;
      if (I < nat)
        for (int c = 0; c < 3; ++c) part[((size_t)I * 3 + c) * gridDim.x + blockIdx.x] = acc[3 * j + c];
    }
  }
}

// The same force sums with one thread per ion, for cells with many ions.  A block
// takes a tile of NT ions and a chunk of rows (k3, k1) of the half spectrum; the
// G-dependent factors of a row (G, and w conj(n) times the two form-factor parts)
// are computed once into LDS and read by every ion of the tile, and each ion
// advances its phase e^{-iG.R} along k2 by one complex multiply, re-seeded from
// the phase tables every FRC_RESEED steps and where the signed frequency wraps
// (k2 = n2/2 + 1).
constexpr int FRC_RESEED = 32;
constexpr int FRC_MAX_N2 = 512;

template <typename R>
__global__ void __launch_bounds__(NT) k_forces_ions(int nat, const double* __restrict__ Z,
                                                    const double2* __restrict__ tab,
                                                    const cplx<R>* __restrict__ nhat,
                                                    const double2* __restrict__ sfac, double split, GridDesc g,
                                                    LppParams lp, int rows_per_chunk, double* __restrict__ part) {
  __shared__ double4 sg[FRC_MAX_N2];   // G
  __shared__ double4 sp[FRC_MAX_N2];   // w conj(n) a + Ewald term, w conj(n) b as (re, im, re, im)
  const int M = g.n1 + g.n2 + g.n3h;
  const int I = blockIdx.y * NT + threadIdx.x;
  const bool have = I < nat;
  const double2* t = tab + (size_t)(have ? I : 0) * M;
  const double zI = have ? Z[I] : 0.0;
  const double2 step = t[g.n1 + 1];   // m2 = +1
  const int wrap2 = g.n2 / 2 + 1;   // m2 jumps from +n2/2 to 1 - n2/2 here
  double ax = 0.0, ay = 0.0, az = 0.0;
  const int nrows = g.n1 * g.n3h;
  const int r0 = blockIdx.x * rows_per_chunk;
  const int r1 = min(nrows, r0 + rows_per_chunk);
  for (int r = r0; r < r1; ++r) {
    const int k3 = r / g.n1, k1 = r - k3 * g.n1;
    __syncthreads();   // every ion is done with the previous row
    for (int k2 = threadIdx.x; k2 < g.n2; k2 += NT) {
      double gx, gy, gz;
      const bool keep = gvec(g, k1, k2, k3, gx, gy, gz);
      const double G2 = gx * gx + gy * gy + gz * gz;
      double4 fg = make_double4(0.0, 0.0, 0.0, 0.0), fp = make_double4(0.0, 0.0, 0.0, 0.0);
      if (keep && G2 > 0.0) {
        double a, b;
        form_ab(lp, sqrt(G2), g.volume, a, b);
        const double wk = (k3 == 0) ? 1.0 : 2.0;
        const size_t gi = (size_t)r * g.n2 + k2;
        const cplx<R> nh = nhat[gi];
        const double cx = wk * double(nh.x), cy = -wk * double(nh.y);
        const double ke = ewald_force_coef(wk, G2, g.volume, split);
        const double2 sz = sfac[gi];
        fg = make_double4(gx, gy, gz, 0.0);
        fp = make_double4(cx * a + ke * sz.x, cy * a - ke * sz.y, cx * b, cy * b);
      }
      sg[k2] = fg;
      sp[k2] = fp;
    }
    __syncthreads();
    const double2 base = zmul(t[k1], t[g.n1 + g.n2 + k3]);
    double2 e = base;
    for (int k2 = 0; k2 < g.n2; ++k2) {
      if ((k2 & (FRC_RESEED - 1)) == 0 || k2 == wrap2) e = zmul(base, t[g.n1 + k2]);
      else e = zmul(e, step);
      const double4 fg = sg[k2], fp = sp[k2];
      // Im[w conj(n) e] (Z a + b)
      const double ia = fp.x * e.y + fp.y * e.x;
      const double ib = fp.z * e.y + fp.w * e.x;
      const double im = zI * ia + ib;
      ax += fg.x * im;
      ay += fg.y * im;
      az += fg.z * im;
    }
  }
  if (have) {
    part[((size_t)I * 3 + 0) * gridDim.x + blockIdx.x] = ax;
    part[((size_t)I * 3 + 1) * gridDim.x + blockIdx.x] = ay;
    part[((size_t)I * 3 + 2) * gridDim.x + blockIdx.x] = az;
  }
}

// One wavefront per force component: lanes stride over its block partials, then
// a fixed-order wave sum (k is uniform across a wavefront, so whole waves exit).
__global__ void __launch_bounds__(NT) k_forces_final(int nat, const double* __restrict__ part, int nb, double scale,
                                                     double* __restrict__ out) {
  const int k = blockIdx.x * (NT / 64) + (threadIdx.x >> 6), lane = threadIdx.x & 63;
  if (k >= 3 * nat) return;
  double s = 0.0;
  for (int i = lane; i < nb; i += 64) s += part[(size_t)k * nb + i];
  s = wave_sum(s);
  if (lane == 0) out[k] = scale * s;
}

// ---------------------------------------------------------------- stress (Eqs. StressTensor, stressTF_a/b)
// d/dq of the volume-free form factor V v_I(q) = Z_I ua(q) + ub(q).
__device__ __forceinline__ void form_ab_dq(const LppParams& lp, double q, double& dua, double& dub) {
  const double P = -kFourPi / (q * q), dP = 2.0 * kFourPi / (q * q * q);
  if (lp.kind == 0) {
    const double e = exp(-0.25 * q * q * lp.rc * lp.rc);
    dua = dP * e + P * e * (-0.5 * q * lp.rc * lp.rc);
    dub = 0.0;
  } else {
    double sn, cs;
    sincos(q * lp.rc, &sn, &cs);
    const double x = q / lp.qc;
    const double x2 = x * x;
    const double f = exp(-x2 * x2 * x2);
    const double df = -6.0 * x2 * x2 * x / lp.qc * f;
    dua = dP * cs * f - P * lp.rc * sn * f + P * cs * df;
    const double h = -lp.A * lp.rc * cs + lp.A / q * sn;
    const double dh = lp.A * lp.rc * lp.rc * sn + lp.A * (lp.rc * cs / q - sn / (q * q));
    dub = dP * h * f + P * dh * f + P * h * df;
  }
}

// Reciprocal-space stress sums over the kept G != 0 (w = 1 on the k3 = 0 plane,
// 2 elsewhere), in the order xx, yy, zz, xy, yz, xz:
//   part[0..5]:  w 4 pi |n(G)|^2 G_a G_b / G^4                  (Hartree)
//   part[6..11]: w Re[conj(n(G)) sum_I u_I'(|G|) e^{-iG.R_I}] G_a G_b / |G|   (pseudopotential)
template <typename R>
__global__ void __launch_bounds__(NT) k_stress_recip(const double2* __restrict__ sfac,
                                                     const cplx<R>* __restrict__ nhat, GridDesc g, LppParams lp,
                                                     double split, double* __restrict__ part) {
  __shared__ double red[12 * NT / 64];
  const long long plane = (long long)g.n1 * g.n2;
  double acc[12];
#pragma unroll
  for (int k = 0; k < 12; ++k) acc[k] = 0.0;
  for (long long gi = (long long)blockIdx.x * NT + threadIdx.x; gi < g.NS; gi += (long long)gridDim.x * NT) {
    const int k3 = (int)(gi / plane);
    const long long rem = gi - k3 * plane;
    const int k1 = (int)(rem / g.n2), k2 = (int)(rem - (long long)k1 * g.n2);
    double gx, gy, gz;
    const bool keep = gvec(g, k1, k2, k3, gx, gy, gz);
    const double G2 = gx * gx + gy * gy + gz * gz;
    if (!keep || G2 == 0.0) continue;
    const double q = sqrt(G2);
    const double wk = (k3 == 0) ? 1.0 : 2.0;
    const cplx<R> nh = nhat[gi];
    const double nx = double(nh.x), ny = double(nh.y);
    const double gg[6] = {gx * gx, gy * gy, gz * gz, gx * gy, gy * gz, gx * gz};
    const double2 szf = sfac[gi];
    // Hartree, V 4 pi |n|^2 / G^4, plus the reciprocal Ewald term (1/V of it here, the
    // sum is scaled by V): (2 pi / V^2) exp(-G^2/4a^2)/G^2 |S_Z|^2 2 (1/G^2 + 1/(4 a^2))
    const double q4 = 0.25 / (split * split);
    const double h = wk * (kFourPi * (nx * nx + ny * ny) / (G2 * G2) +
                           0.5 * kFourPi / (g.volume * g.volume) * exp(-G2 * q4) / G2 * (szf.x * szf.x + szf.y * szf.y) *
                               2.0 * (1.0 / G2 + q4));
    double dua, dub;
    form_ab_dq(lp, q, dua, dub);
    // sum_I (Z_I u_a' + u_b') e^{-iG.R_I} from the stored structure factors
    const double2 sz = sfac[gi], s1 = sfac[g.NS + gi];
    const double sx = dua * sz.x + dub * s1.x;
    const double sy = dua * sz.y + dub * s1.y;
    const double x = wk * (nx * sx + ny * sy) / q;   // w Re[conj(n) S']/|G|
#pragma unroll
    for (int k = 0; k < 6; ++k) {
      acc[k] += h * gg[k];
      acc[6 + k] += x * gg[k];
    }
  }
  block_sum<12>(acc, red);
  if (threadIdx.x == 0) {
#pragma unroll
    for (int k = 0; k < 12; ++k) part[k * gridDim.x + blockIdx.x] = acc[k];
  }
}

// Local stress sums at every point (FP64), in part[k * gridDim.x + block]:
//   0: f - n df/dn (ftTF: f - n T eta), 1: n (eps_xc - v_xc),
//   2..7: W_a d_b n with W = 2 df/dsigma grad n (xx, yy, zz, xy, yz, xz; zero for ftTF).
template <typename R, bool TF>
__global__ void __launch_bounds__(NT) k_stress_local(const double* __restrict__ phi, const R* __restrict__ g0,
                                                     const R* __restrict__ g1, const R* __restrict__ g2,
                                                     long long npts, EvalParams ep, double* __restrict__ part) {
  __shared__ double red[8 * NT / 64];
  EnhParams enh{(int)ep.enh_kind, ep.enh_c1, ep.enh_a1};
  double acc[8];
#pragma unroll
  for (int k = 0; k < 8; ++k) acc[k] = 0.0;
  for (long long i = (long long)blockIdx.x * NT + threadIdx.x; i < npts; i += (long long)gridDim.x * NT) {
    const double p = phi[i];
    const double n = p * p;
    const double nf = n > kDensityFloor ? n : kDensityFloor;
    const double ln_n = ln_pos(nf);
    if constexpr (TF) {
      double f, vt, tsl;
      tf_point(nf, ln_n, ep.lt0, f, vt, tsl);
      acc[0] += f - n * vt;
    } else {
      const R gx = g0[i], gy = g1[i], gz = g2[i];
      const R sigma = gx * gx + gy * gy + gz * gz;
      double f, tsl;
      R dfdn, dfds;
      gga_point<R>(nf, ln_n, sigma, ep.lt0, enh, f, dfdn, dfds, tsl);
      acc[0] += f - n * double(dfdn);
      const double w2 = 2.0 * double(dfds);
      const double dx = double(gx), dy = double(gy), dz = double(gz);
      acc[2] += w2 * dx * dx;
      acc[3] += w2 * dy * dy;
      acc[4] += w2 * dz * dz;
      acc[5] += w2 * dx * dy;
      acc[6] += w2 * dy * dz;
      acc[7] += w2 * dx * dz;
    }
    // LDA XC term delta_ab int n (f_xc - v_xc) (PZ81, or KSDT by Eq. stressLSDAxc)
    double vx = 0.0, ex = 0.0, tx = 0.0;
    xc_point<R>(ep.xc, n, ln_n, ep.lt0, vx, ex, tx);
    acc[1] += ex - n * vx;
  }
  block_sum<8>(acc, red);
  if (threadIdx.x == 0) {
#pragma unroll
    for (int k = 0; k < 8; ++k) part[k * gridDim.x + blockIdx.x] = acc[k];
  }
}

// ---------------------------------------------------------------- host side
#define OFDFT_LENGTHS(X) \
  X(8) X(12) X(16) X(20) X(24) X(32) X(40) X(48) X(64) X(80) X(96) X(128) X(160) X(192) X(256) X(320) X(400)
#define OFDFT_PLANE_LENGTHS(X) X(8) X(12) X(16) X(20) X(24) X(32) X(40) X(48) X(64) X(80) X(96) X(128)

static inline bool hip_ok(ofdft_ctx* c, hipError_t e, const char* what) {
  if (e == hipSuccess) return true;
  c->err = std::string(what) + ": " + hipGetErrorString(e);
  return false;
}

static inline int dev_fail(ofdft_ctx* c, int code, const char* what) {
  c->err = what;
  return code;
}

// ---------------------------------------------------------------- static scratch
// Evaluation scratch of ofdft_eval_noalloc: the spectra, real work arrays, partial
// sums and scalars of one evaluation, carved out of this array instead of the
// context's own buffers.  Each device holds its own copy for the life of the process.
// Host code never uses the name: its device address is taken once per device, with
// that device current, by hipGetSymbolAddress (dev_upload_tables) and kept in
// g_scratch_addr.
static __device__ __align__(256) char scratch[kNoAllocScratchBytes];

static std::mutex g_dev_mtx;
static std::vector<char> g_tables_uploaded;
static std::vector<void*> g_scratch_addr;

// The t-factor tables live in __constant__ memory, one copy per device: upload
// once per device (the caller has made it current).  The same first call per
// device records the device address of the static scratch array.
int dev_upload_tables(int device) {
  std::lock_guard<std::mutex> lock(g_dev_mtx);
  if (device < 0) return OFDFT_E_ARG;
  if ((int)g_tables_uploaded.size() <= device) {
    g_tables_uploaded.resize(device + 1, 0);
    g_scratch_addr.resize(device + 1, nullptr);
  }
  if (g_tables_uploaded[device]) return OFDFT_OK;
  // function-major (as generated) -> coefficient-major within each piece
  auto k_major = [](const double* src, int nf) {
    std::vector<double> out((size_t)OFDFT_T_NP * nf * OFDFT_T_NC);
    for (int p = 0; p < OFDFT_T_NP; ++p)
      for (int f = 0; f < nf; ++f)
        for (int k = 0; k < OFDFT_T_NC; ++k)
          out[((size_t)p * OFDFT_T_NC + k) * nf + f] = src[((size_t)p * nf + f) * OFDFT_T_NC + k];
    return out;
  };
  const std::vector<double> gga = k_major(kTGga, 8), tf = k_major(kTTf, 3);
  if (hipMemcpyToSymbol(HIP_SYMBOL(c_t_gga), gga.data(), sizeof(kTGga)) != hipSuccess) return OFDFT_E_DEVICE;
  if (hipMemcpyToSymbol(HIP_SYMBOL(c_t_tf), tf.data(), sizeof(kTTf)) != hipSuccess) return OFDFT_E_DEVICE;
  void* addr = nullptr;
  if (hipGetSymbolAddress(&addr, HIP_SYMBOL(scratch)) != hipSuccess || addr == nullptr) return OFDFT_E_DEVICE;
  g_scratch_addr[device] = addr;
  g_tables_uploaded[device] = 1;
  return OFDFT_OK;
}

// Bytes of the scratch one evaluation of the context needs (spectra A, S0, D, B0..B2;
// real arrays gr0..gr2, vloc, v; partial sums, scalars and vector-reduction partials).
static size_t noalloc_layout(const ofdft_ctx* c, size_t* off) {
  const size_t rs = c->rsize, N = (size_t)c->g.N, NS = (size_t)c->g.NS;
  auto up = [](size_t b) { return (b + 255) & ~size_t(255); };
  size_t o = 0;
  for (int k = 0; k < 6; ++k) { off[k] = o; o += up(NS * 2 * rs); }      // A S0 D B0 B1 B2
  for (int k = 6; k < 11; ++k) { off[k] = o; o += up(N * rs); }          // gr0..gr2 vloc v
  off[11] = o; o += up((size_t)SL_COUNT * c->max_blocks * sizeof(double));  // partials
  off[12] = o; o += up(SC_COUNT * sizeof(double));                      // scalars
  off[13] = o; o += up(8 * VEC_BLOCKS * sizeof(double));                 // vpart
  off[14] = o; o += up(32 * sizeof(double));                             // vout
  return o;
}

size_t dev_noalloc_bytes(const ofdft_ctx* c) {
  size_t off[15];
  return noalloc_layout(c, off);
}

int dev_scratch_bind(ofdft_ctx* c, ScratchSave* sv) {
  size_t off[15];
  const size_t need = noalloc_layout(c, off);
  if (need > kNoAllocScratchBytes)
    return dev_fail(c, OFDFT_E_ARG, "the evaluation needs more scratch than the static scratch array holds "
                                    "(see OFDFT_NOALLOC_SCRATCH_BYTES)");
  const int dev = c->opt.device;
  char* base = nullptr;
  {
    std::lock_guard<std::mutex> lock(g_dev_mtx);
    if (dev < (int)g_scratch_addr.size()) base = static_cast<char*>(g_scratch_addr[dev]);
  }
  if (!base) return dev_fail(c, OFDFT_E_DEVICE, "static scratch address not resolved for this device");
  sv->A = c->A; sv->S0 = c->S0; sv->D = c->D;
  for (int k = 0; k < 3; ++k) { sv->B[k] = c->B[k]; sv->gr[k] = c->gr[k]; }
  sv->vloc = c->vloc; sv->v = c->v; sv->partials = c->partials; sv->scalars = c->scalars;
  sv->vpart = c->vpart; sv->vout = c->vout;
  void* spec[6];
  for (int k = 0; k < 6; ++k) spec[k] = base + off[k];
  c->A = spec[0]; c->S0 = spec[1]; c->D = spec[2];
  for (int k = 0; k < 3; ++k) { c->B[k] = spec[3 + k]; c->gr[k] = base + off[6 + k]; }
  c->vloc = base + off[9];
  c->v = base + off[10];
  c->partials = reinterpret_cast<double*>(base + off[11]);
  c->scalars = reinterpret_cast<double*>(base + off[12]);
  c->vpart = reinterpret_cast<double*>(base + off[13]);
  c->vout = reinterpret_cast<double*>(base + off[14]);
  return OFDFT_OK;
}

void dev_scratch_restore(ofdft_ctx* c, const ScratchSave* sv) {
  c->A = sv->A; c->S0 = sv->S0; c->D = sv->D;
  for (int k = 0; k < 3; ++k) { c->B[k] = sv->B[k]; c->gr[k] = sv->gr[k]; }
  c->vloc = sv->vloc; c->v = sv->v; c->partials = sv->partials; c->scalars = sv->scalars;
  c->vpart = sv->vpart; c->vout = sv->vout;
}

// out[i] = double(v[i]) for the N points of the grid (v in the context's precision).
__global__ void __launch_bounds__(NT) k_to_double(const void* __restrict__ v, int rsize, long long n,
                                                  double* __restrict__ out) {
  for (long long i = (long long)blockIdx.x * NT + threadIdx.x; i < n; i += (long long)gridDim.x * NT)
    out[i] = rsize == 4 ? double(static_cast<const float*>(v)[i]) : static_cast<const double*>(v)[i];
}

int dev_to_double(ofdft_ctx* c, const void* v, double* out) {
  const int nb = (int)std::min<long long>(2048, (c->g.N + NT - 1) / NT);
  hipLaunchKernelGGL(k_to_double, dim3(nb), dim3(NT), 0, c->stream, v, (int)c->rsize, c->g.N, out);
  return hip_ok(c, hipGetLastError(), "conversion launch") ? OFDFT_OK : OFDFT_E_DEVICE;
}

template <typename R, int L>
static size_t lds_rpass_fwd(int tr) {
  return 2 * pad16<cplx<R>>((tr / 2) * Lay<L>::RS) + pad16<cplx<R>>(L) + pad16<double>(NT / 64);
}
template <typename R, int L>
static size_t lds_rpass_inv(int tr, int extra_real, int nred) {
  return pad16<cplx<R>>((tr / 2) * Lay<L>::RS) + pad16<cplx<R>>(zb_elems<L>(tr)) + pad16<cplx<R>>(L) +
         pad16<R>((size_t)extra_real * tr * L) + pad16<double>((size_t)nred * NT / 64);
}
template <typename R, int L>
static size_t lds_x1(int tc, int nred) {
  return 2 * pad16<cplx<R>>((size_t)tc * Lay<L>::RS) + pad16<cplx<R>>(L) + pad16<double>((size_t)nred * NT / 64);
}
template <typename R, int L>
static size_t lds_x2(int rb) {
  return 2 * pad16<cplx<R>>((size_t)rb * Lay<L>::RS) + pad16<cplx<R>>(L);
}

// Timing hook: record an event before each launch when enabled.
static inline void tmark(ofdft_ctx* c, const char* name) {
  if (!c->timing.on) return;
  Timing& t = c->timing;
  if (t.used >= (int)t.events.size()) return;
  if (t.used < (int)t.names.size()) t.names[t.used] = name;
  else t.names.push_back(name);
  (void)hipEventRecord(t.events[t.used++], c->stream);
}

template <typename R>
static void set_lds_limits() {
  // allow large dynamic LDS (gfx950: 160 KB per workgroup)
}

template <typename R, int L>
static void launch_rpass_fwd(ofdft_ctx* c, const double* phi, void* out, const Rotation* rot = nullptr) {
  const GridDesc& g = c->g;
  dim3 grid(g.n2 / g.tr, g.n1);
  if (rot)
    hipLaunchKernelGGL((k_rpass_fwd_density<R, L, true>), grid, dim3(NT), (lds_rpass_fwd<R, L>(g.tr)), c->stream,
                       phi, (cplx<R>*)out, (const cplx<R>*)c->tw[2], g, c->partials, c->max_blocks, *rot);
  else
    hipLaunchKernelGGL((k_rpass_fwd_density<R, L, false>), grid, dim3(NT), (lds_rpass_fwd<R, L>(g.tr)), c->stream,
                       phi, (cplx<R>*)out, (const cplx<R>*)c->tw[2], g, c->partials, c->max_blocks, Rotation{});
}

template <typename R, int L, int SIGN, int U>
static void launch_x2_u(ofdft_ctx* c, void* a0, void* a1, void* a2, int narr) {
  const GridDesc& g = c->g;
  const int nrows = g.n3k * g.n1;   // the k3 = n3/2 plane is not used
  dim3 grid((unsigned)((nrows + g.rb - 1) / g.rb), narr);
  Arr3 arr{{a0, a1, a2}};
  hipLaunchKernelGGL((k_cpass_x2<R, L, SIGN, U>), grid, dim3(NT), (lds_x2<R, L>(g.rb)), c->stream, arr,
                     (const cplx<R>*)c->tw[1], nrows, g.rb, g.gate);
}

// Staged elements per thread of an x1 tile of L * tc elements: 1, 2, 4 or 8.
static inline int x1_stage_u(int L, int tc) {
  const int need = (L * tc + NT - 1) / NT;
  return need <= 1 ? 1 : need <= 2 ? 2 : need <= 4 ? 4 : 8;
}

#define OFDFT_DISPATCH_U(UVAL, CALL)               \
  switch (UVAL) {                                  \
    case 1: { constexpr int U_ = 1; CALL; } break; \
    case 2: { constexpr int U_ = 2; CALL; } break; \
    case 4: { constexpr int U_ = 4; CALL; } break; \
    default: { constexpr int U_ = 8; CALL; } break; \
  }

// Staged elements per thread of an x2 tile of rb rows of L: 1, 2, 4, 8 or 16.
static inline int x2_stage_u(int L, int rb) {
  const int need = (L * rb + NT - 1) / NT;
  return need <= 1 ? 1 : need <= 2 ? 2 : need <= 4 ? 4 : need <= 8 ? 8 : 16;
}

template <typename R, int L, int SIGN>
static void launch_x2(ofdft_ctx* c, void* a0, void* a1, void* a2, int narr) {
  switch (x2_stage_u(L, c->g.rb)) {
    case 1: launch_x2_u<R, L, SIGN, 1>(c, a0, a1, a2, narr); break;
    case 2: launch_x2_u<R, L, SIGN, 2>(c, a0, a1, a2, narr); break;
    case 4: launch_x2_u<R, L, SIGN, 4>(c, a0, a1, a2, narr); break;
    case 8: launch_x2_u<R, L, SIGN, 8>(c, a0, a1, a2, narr); break;
    default: launch_x2_u<R, L, SIGN, 16>(c, a0, a1, a2, narr); break;
  }
}

template <typename R, int L, int MODE, int U>
static void launch_x1_density_u(ofdft_ctx* c, const void* in, void* out0, void* out1, void* out2) {
  const GridDesc& g = c->g;
  dim3 grid(g.n2 / g.tc, g.n3k);
  hipLaunchKernelGGL((k_x1_density<R, L, MODE, U>), grid, dim3(NT), (lds_x1<R, L>(g.tc, 2)), c->stream,
                     (const cplx<R>*)in, (const cplx<R>*)c->Vext, (cplx<R>*)out0, (cplx<R>*)out1,
                     (cplx<R>*)out2, (cplx<R>*)c->S0, (const cplx<R>*)c->tw[0], g, c->partials, c->max_blocks);
}

// x1 pass over the spectrum `in` (n(G) in A, or the minimiser's gradient spectrum).
template <typename R, int L, int MODE>
static void launch_x1_density(ofdft_ctx* c, const void* in, void* out0, void* out1, void* out2) {
  OFDFT_DISPATCH_U(x1_stage_u(L, c->g.tc), (launch_x1_density_u<R, L, MODE, U_>(c, in, out0, out1, out2)));
}

template <typename R, int L>
static void launch_rpass_inv_real3(ofdft_ctx* c) {
  const GridDesc& g = c->g;
  dim3 grid(g.n2 / g.tr, g.n1, 3);
  Arr3 in{{c->B[0], c->B[1], c->B[2]}};
  RealArr3 out{{c->gr[0], c->gr[1], c->gr[2]}};
  hipLaunchKernelGGL((k_rpass_inv_real<R, L>), grid, dim3(NT), (lds_rpass_inv<R, L>(g.tr, 0, 0)), c->stream, in,
                     out, (const cplx<R>*)c->tw[2], g);
}

template <typename R, int L>
static void launch_rpass_inv_real1(ofdft_ctx* c, void* in_spec, void* out_real) {
  const GridDesc& g = c->g;
  dim3 grid(g.n2 / g.tr, g.n1, 1);
  Arr3 in{{in_spec, nullptr, nullptr}};
  RealArr3 out{{out_real, nullptr, nullptr}};
  hipLaunchKernelGGL((k_rpass_inv_real<R, L>), grid, dim3(NT), (lds_rpass_inv<R, L>(g.tr, 0, 0)), c->stream, in,
                     out, (const cplx<R>*)c->tw[2], g);
}

// ---- plane-pass launchers (n2 == n3 = L <= 128; see plane_mode)
template <typename R, int L>
static void launch_plane_fwd_density(ofdft_ctx* c, const double* phi, void* out, const Rotation* rot) {
  const GridDesc& g = c->g;
  if constexpr (sizeof(R) == 4 && (L == 32 || L == 64 || L == 128)) {
    if (c->fused_gga) {   // the parity-split form (same switch as the fused gradient pass)
      if (rot)
        hipLaunchKernelGGL((k_plane_fwd_density_par<R, L, true>), dim3(2 * g.n1), dim3(NTP), 0, c->stream, phi,
                           (cplx<R>*)out, (const cplx<R>*)c->tw[2], g, c->partials, c->max_blocks, *rot);
      else
        hipLaunchKernelGGL((k_plane_fwd_density_par<R, L, false>), dim3(2 * g.n1), dim3(NTP), 0, c->stream, phi,
                           (cplx<R>*)out, (const cplx<R>*)c->tw[2], g, c->partials, c->max_blocks, Rotation{});
      return;
    }
  }
  if (rot)
    hipLaunchKernelGGL((k_plane_fwd_density<R, L, true>), dim3(2 * g.n1), dim3(NTP), (lds_plane<R, L>(1)), c->stream,
                       phi, (cplx<R>*)out, (const cplx<R>*)c->tw[2], g, c->partials, c->max_blocks, *rot);
  else
    hipLaunchKernelGGL((k_plane_fwd_density<R, L, false>), dim3(2 * g.n1), dim3(NTP), (lds_plane<R, L>(1)), c->stream,
                       phi, (cplx<R>*)out, (const cplx<R>*)c->tw[2], g, c->partials, c->max_blocks, Rotation{});
}

template <typename R, int L>
static void launch_plane_inv_real(ofdft_ctx* c, void* in0, void* in1, void* in2, void* out0, void* out1, void* out2,
                                  int narr) {
  const GridDesc& g = c->g;
  Arr3 in{{in0, in1, in2}};
  RealArr3 out{{out0, out1, out2}};
  hipLaunchKernelGGL((k_plane_inv_real<R, L, NTP>), dim3(g.n1, narr), dim3(NTP), (lds_plane<R, L>(0)), c->stream, in,
                     out, (const cplx<R>*)c->tw[2], g);
}

template <typename R, int L>
static void launch_plane_fwd_real3(ofdft_ctx* c) {
  const GridDesc& g = c->g;
  RealArr3 in{{c->gr[0], c->gr[1], c->gr[2]}};
  Arr3 out{{c->B[0], c->B[1], c->B[2]}};
  hipLaunchKernelGGL((k_plane_fwd_real<R, L, NTP>), dim3(g.n1, 3), dim3(NTP), (lds_plane<R, L>(0)), c->stream, in,
                     out, (const cplx<R>*)c->tw[2], g);
}

template <typename R, int L>
static void launch_plane_fwd_grad(ofdft_ctx* c, const double* phi, const void* v, const double* sc, double two_dv,
                                  void* out) {
  const GridDesc& g = c->g;
  hipLaunchKernelGGL((k_plane_fwd_grad<R, L>), dim3(g.n1), dim3(NTP), (lds_plane<R, L>(0)), c->stream, phi,
                     (const R*)v, sc, two_dv, (cplx<R>*)out, (const cplx<R>*)c->tw[2], g);
}

template <int L>
static void launch_plane_final_q(ofdft_ctx* c, const double* phi, void* v_out, const EvalParams& ep, const Slope* sl) {
  const GridDesc& g = c->g;
  if (sl)
    hipLaunchKernelGGL((k_plane_final_q<float, L, true>), dim3(4 * g.n1), dim3(IGG_NT), 0, c->stream,
                       (const cplx<float>*)c->D, phi, (const float*)c->vloc, (float*)v_out,
                       (const cplx<float>*)c->tw[2], g, ep, c->partials, c->max_blocks, *sl);
  else
    hipLaunchKernelGGL((k_plane_final_q<float, L, false>), dim3(4 * g.n1), dim3(IGG_NT), 0, c->stream,
                       (const cplx<float>*)c->D, phi, (const float*)c->vloc, (float*)v_out,
                       (const cplx<float>*)c->tw[2], g, ep, c->partials, c->max_blocks, Slope{});
}

template <typename R, int L, bool TF>
static void launch_plane_final(ofdft_ctx* c, const double* phi, void* v_out, const EvalParams& ep, const Slope* sl) {
  const GridDesc& g = c->g;
  if (sl)
    hipLaunchKernelGGL((k_plane_final<R, L, TF, true>), dim3(2 * g.n1), dim3(NTP), (lds_plane<R, L>(kFinalSums)), c->stream,
                       (const cplx<R>*)c->D, phi, (const R*)c->vloc, (R*)v_out, (const cplx<R>*)c->tw[2], g, ep,
                       c->partials, c->max_blocks, *sl);
  else
    hipLaunchKernelGGL((k_plane_final<R, L, TF, false>), dim3(2 * g.n1), dim3(NTP), (lds_plane<R, L>(kFinalSums)), c->stream,
                       (const cplx<R>*)c->D, phi, (const R*)c->vloc, (R*)v_out, (const cplx<R>*)c->tw[2], g, ep,
                       c->partials, c->max_blocks, Slope{});
}

template <typename R>
static void launch_pointwise_gga(ofdft_ctx* c, const double* phi, const EvalParams& ep) {
  auto k = ep.xc == 1 ? k_pointwise_gga<R, 1> : ep.xc == 2 ? k_pointwise_gga<R, 2> : k_pointwise_gga<R, 0>;
  hipLaunchKernelGGL(k, dim3(pw_blocks(c->g)), dim3(NT), 0, c->stream, phi, (R*)c->gr[0], (R*)c->gr[1],
                     (R*)c->gr[2], (R*)c->vloc, c->g.N, ep, c->partials, c->max_blocks);
}

// The fused gradient pass (k_plane_inv_gga) serves mixed precision with PZ81 or no XC on
// square planes of 32, 64 or 128 points (the KSDT fit and the FP64 assembly need more
// registers than two of its blocks per CU leave); its four blocks per plane each write one
// slot of partial sums.
static bool fused_gga_mode(const ofdft_ctx* c, const EvalParams& ep) {
  return c->fused_gga && c->rsize == 4 && ep.xc != 2 &&
         (c->g.n3 == 32 || c->g.n3 == 64 || c->g.n3 == 128) && 4 * c->g.n1 <= c->max_blocks;
}

template <int L>
static void launch_plane_inv_gga(ofdft_ctx* c, const double* phi, const EvalParams& ep) {
  const GridDesc& g = c->g;
  Arr3 in{{c->B[0], c->B[1], c->B[2]}};
  auto k = ep.xc == 1 ? k_plane_inv_gga<float, L, 1> : k_plane_inv_gga<float, L, 0>;
  hipLaunchKernelGGL(k, dim3(4 * g.n1), dim3(IGG_NT), 0, c->stream, in, phi, (float*)c->gr[0], (float*)c->gr[1],
                     (float*)c->gr[2], (float*)c->vloc, (const cplx<float>*)c->tw[2], g, ep, c->partials,
                     c->max_blocks);
}

template <typename R, int L>
static void launch_rpass_fwd_real3(ofdft_ctx* c) {
  const GridDesc& g = c->g;
  dim3 grid(g.n2 / g.tr, g.n1, 3);
  RealArr3 in{{c->gr[0], c->gr[1], c->gr[2]}};
  Arr3 out{{c->B[0], c->B[1], c->B[2]}};
  hipLaunchKernelGGL((k_rpass_fwd_real<R, L>), grid, dim3(NT), (lds_rpass_fwd<R, L>(g.tr)), c->stream, in, out,
                     (const cplx<R>*)c->tw[2], g);
}

template <typename R, int L, int U>
static void launch_x1_div_u(ofdft_ctx* c) {
  const GridDesc& g = c->g;
  dim3 grid(g.n2 / g.tc, g.n3k);
  hipLaunchKernelGGL((k_x1_divergence<R, L, U>), grid, dim3(NT), (lds_x1<R, L>(g.tc, 0)), c->stream,
                     (const cplx<R>*)c->B[0], (const cplx<R>*)c->B[1], (const cplx<R>*)c->B[2],
                     (const cplx<R>*)c->S0, (cplx<R>*)c->D, (const cplx<R>*)c->tw[0], g);
}

template <typename R, int L>
static void launch_x1_div(ofdft_ctx* c) {
  OFDFT_DISPATCH_U(x1_stage_u(L, c->g.tc), (launch_x1_div_u<R, L, U_>(c)));
}

template <typename R, int L, bool TF>
static void launch_rpass_final(ofdft_ctx* c, const double* phi, void* v_out, const EvalParams& ep, const Slope* sl) {
  const GridDesc& g = c->g;
  dim3 grid(g.n2 / g.tr, g.n1);
  if (sl)
    hipLaunchKernelGGL((k_rpass_final<R, L, TF, true>), grid, dim3(NT), (lds_rpass_inv<R, L>(g.tr, 0, kFinalSums)),
                       c->stream, (const cplx<R>*)c->D, phi, (const R*)c->vloc, (R*)v_out, (const cplx<R>*)c->tw[2],
                       g, ep, c->partials, c->max_blocks, *sl);
  else
    hipLaunchKernelGGL((k_rpass_final<R, L, TF, false>), grid, dim3(NT), (lds_rpass_inv<R, L>(g.tr, 0, kFinalSums)),
                       c->stream, (const cplx<R>*)c->D, phi, (const R*)c->vloc, (R*)v_out, (const cplx<R>*)c->tw[2],
                       g, ep, c->partials, c->max_blocks, Slope{});
}

// Dispatch on a runtime length.
#define OFDFT_DISPATCH(LEN, CALL)              \
  switch (LEN) {                               \
    OFDFT_LENGTHS_CALL(CALL)                   \
    default: return OFDFT_E_GRID;              \
  }
#define OFDFT_LENGTHS_CALL(CALL)                                                                         \
  case 8: { constexpr int L_ = 8; CALL; } break; case 12: { constexpr int L_ = 12; CALL; } break;       \
  case 16: { constexpr int L_ = 16; CALL; } break; case 20: { constexpr int L_ = 20; CALL; } break;     \
  case 24: { constexpr int L_ = 24; CALL; } break; case 32: { constexpr int L_ = 32; CALL; } break;     \
  case 40: { constexpr int L_ = 40; CALL; } break; case 48: { constexpr int L_ = 48; CALL; } break;     \
  case 64: { constexpr int L_ = 64; CALL; } break; case 80: { constexpr int L_ = 80; CALL; } break;     \
  case 96: { constexpr int L_ = 96; CALL; } break; case 128: { constexpr int L_ = 128; CALL; } break;   \
  case 160: { constexpr int L_ = 160; CALL; } break; case 192: { constexpr int L_ = 192; CALL; } break; \
  case 256: { constexpr int L_ = 256; CALL; } break; case 320: { constexpr int L_ = 320; CALL; } break; \
  case 400: { constexpr int L_ = 400; CALL; } break;

// Dispatch of the plane passes (lengths up to 128).
#define OFDFT_DISPATCH_PLANE(LEN, CALL)                                                                  \
  switch (LEN) {                                                                                         \
    case 8: { constexpr int L_ = 8; CALL; } break; case 12: { constexpr int L_ = 12; CALL; } break;     \
    case 16: { constexpr int L_ = 16; CALL; } break; case 20: { constexpr int L_ = 20; CALL; } break;   \
    case 24: { constexpr int L_ = 24; CALL; } break; case 32: { constexpr int L_ = 32; CALL; } break;   \
    case 40: { constexpr int L_ = 40; CALL; } break; case 48: { constexpr int L_ = 48; CALL; } break;   \
    case 64: { constexpr int L_ = 64; CALL; } break; case 80: { constexpr int L_ = 80; CALL; } break;   \
    case 96: { constexpr int L_ = 96; CALL; } break; case 128: { constexpr int L_ = 128; CALL; } break; \
    default: return OFDFT_E_GRID;                                                                        \
  }

// The x3 and x2 transforms run as plane passes when the (i2, i3) planes are
// square with L <= 128 (the plane's half spectrum then fits the LDS of one
// block) and the context has not switched them off.
static bool plane_mode(const ofdft_ctx* c) {
  return c->plane_passes && c->g.n2 == c->g.n3 && c->g.n3 <= 128;
}

static EvalParams make_params(ofdft_ctx* c) {
  EvalParams ep{};
  ep.functional = c->opt.functional;
  ep.xc = c->opt.xc == OFDFT_XC_PZ81 ? 1 : c->opt.xc == OFDFT_XC_KSDT ? 2 : 0;
  ep.T = c->T_ha;
  ep.lt0 = lt_offset(c->T_ha);
  ep.alpha_sum = c->alpha_sum;
  ep.gate = c->g.gate;
  switch (c->opt.functional) {
    case OFDFT_SGA: ep.enh_kind = 0; ep.enh_c1 = c->opt.mu_sga; break;
    case OFDFT_VWTF: ep.enh_kind = 0; ep.enh_c1 = 5.0 / 3.0; break;
    case OFDFT_VT84F: ep.enh_kind = 2; break;
    case OFDFT_KST2: ep.enh_kind = 1; ep.enh_c1 = 2.03087; ep.enh_a1 = 0.29424; break;
    case OFDFT_TW: ep.enh_kind = 1; ep.enh_c1 = 0.2319; ep.enh_a1 = 0.2748; break;
    case OFDFT_APBEF: ep.enh_kind = 1; ep.enh_c1 = 0.23889; ep.enh_a1 = 0.23889 / 0.804; break;
    default: break;
  }
  return ep;
}

// One evaluation at phi, or (rot, sl non-null) a line-search trial: the density pass
// forms phi_t = rot.ca phi + rot.sb rot.dir into rot.phi_out and the evaluation runs at
// phi_t, with dF/dtheta accumulated by the final pass.
template <typename R>
static int eval_impl(ofdft_ctx* c, const double* phi, void* v_out, double* sc, const Rotation* rot,
                     const Slope* sl, const Publish& pub) {
  const GridDesc& g = c->g;
  const EvalParams ep = make_params(c);
  const bool tf = c->opt.functional == OFDFT_TF;
  const double* phi_e = rot ? rot->phi_out : phi;   // the amplitude being evaluated
  const bool plane = plane_mode(c);
  const bool fused = plane && !tf && fused_gga_mode(c, ep);
  if (plane) {
    tmark(c, "plane_fwd_density");
    OFDFT_DISPATCH_PLANE(g.n3, (launch_plane_fwd_density<R, L_>(c, phi, c->A, rot)));
  } else {
    tmark(c, "rpass_fwd_density");
    OFDFT_DISPATCH(g.n3, (launch_rpass_fwd<R, L_>(c, phi, c->A, rot)));
    tmark(c, "cpass_x2_fwd");
    OFDFT_DISPATCH(g.n2, (launch_x2<R, L_, -1>(c, c->A, nullptr, nullptr, 1)));
  }
  if (tf) {
    tmark(c, "x1_density_hartree");
    OFDFT_DISPATCH(g.n1, (launch_x1_density<R, L_, X1_TF>(c, c->A, c->D, nullptr, nullptr)));
  } else {
    tmark(c, "x1_density_gradient");
    OFDFT_DISPATCH(g.n1, (launch_x1_density<R, L_, X1_GGA>(c, c->A, c->B[0], c->B[1], c->B[2])));
    if (fused) {
      tmark(c, "plane_inv_gga");
      if (g.n3 == 128)
        launch_plane_inv_gga<128>(c, phi_e, ep);
      else if (g.n3 == 64)
        launch_plane_inv_gga<64>(c, phi_e, ep);
      else
        launch_plane_inv_gga<32>(c, phi_e, ep);
    } else {
      if (plane) {
        tmark(c, "plane_inv_grad3");
        OFDFT_DISPATCH_PLANE(g.n3, (launch_plane_inv_real<R, L_>(c, c->B[0], c->B[1], c->B[2], c->gr[0], c->gr[1],
                                                                 c->gr[2], 3)));
      } else {
        tmark(c, "cpass_x2_inv3");
        OFDFT_DISPATCH(g.n2, (launch_x2<R, L_, +1>(c, c->B[0], c->B[1], c->B[2], 3)));
        tmark(c, "rpass_inv_grad3");
        OFDFT_DISPATCH(g.n3, (launch_rpass_inv_real3<R, L_>(c)));
      }
      tmark(c, "pointwise_gga");
      launch_pointwise_gga<R>(c, phi_e, ep);
    }
    if (plane) {
      tmark(c, "plane_fwd_w3");
      OFDFT_DISPATCH_PLANE(g.n3, (launch_plane_fwd_real3<R, L_>(c)));
    } else {
      tmark(c, "rpass_fwd_w3");
      OFDFT_DISPATCH(g.n3, (launch_rpass_fwd_real3<R, L_>(c)));
      tmark(c, "cpass_x2_fwd3");
      OFDFT_DISPATCH(g.n2, (launch_x2<R, L_, -1>(c, c->B[0], c->B[1], c->B[2], 3)));
    }
    tmark(c, "x1_divergence");
    OFDFT_DISPATCH(g.n1, (launch_x1_div<R, L_>(c)));
  }
  if (plane) {
    if (tf) {
      tmark(c, "plane_tf_final");
      OFDFT_DISPATCH_PLANE(g.n3, (launch_plane_final<R, L_, true>(c, phi_e, v_out, ep, sl)));
    } else if (fused) {
      tmark(c, "plane_final");
      if (g.n3 == 128)
        launch_plane_final_q<128>(c, phi_e, v_out, ep, sl);
      else if (g.n3 == 64)
        launch_plane_final_q<64>(c, phi_e, v_out, ep, sl);
      else
        launch_plane_final_q<32>(c, phi_e, v_out, ep, sl);
    } else {
      tmark(c, "plane_final");
      OFDFT_DISPATCH_PLANE(g.n3, (launch_plane_final<R, L_, false>(c, phi_e, v_out, ep, sl)));
    }
  } else {
    tmark(c, "cpass_x2_inv");
    OFDFT_DISPATCH(g.n2, (launch_x2<R, L_, +1>(c, c->D, nullptr, nullptr, 1)));
    if (tf) {
      tmark(c, "rpass_tf_final");
      OFDFT_DISPATCH(g.n3, (launch_rpass_final<R, L_, true>(c, phi_e, v_out, ep, sl)));
    } else {
      tmark(c, "rpass_final");
      OFDFT_DISPATCH(g.n3, (launch_rpass_final<R, L_, false>(c, phi_e, v_out, ep, sl)));
    }
  }
  // partial sums of the density and final passes: one per block
  const int nb_r = plane ? 2 * g.n1 : (g.n2 / g.tr) * g.n1;   // plane passes: two blocks per i1 plane
  const ReduceParams rp{nb_r, (g.n2 / g.tc) * g.n3k, tf ? nb_r : fused ? 4 * g.n1 : pw_blocks(g), sl ? 1 : 0, g.dv, g.volume,
                        c->alpha_sum, g.gate, fused ? 4 * g.n1 : nb_r};
  tmark(c, "reduce_scalars");
  hipLaunchKernelGGL(k_reduce_scalars, dim3(1), dim3(RED_NT), 0, c->stream, c->partials, c->max_blocks, rp, sc,
                     pub);
  tmark(c, "end");
  hipError_t e = hipGetLastError();
  return hip_ok(c, e, "eval launch") ? OFDFT_OK : OFDFT_E_DEVICE;
}

template <typename R>
static size_t max_lds_impl(const ofdft_ctx* c) {
  const GridDesc& g = c->g;
  size_t m = 0;
  auto upd = [&](size_t v) { m = v > m ? v : m; };
  switch (g.n3) {
#define OFDFT_LDS3(LEN) \
    case LEN: upd(lds_rpass_fwd<R, LEN>(g.tr)); upd(lds_rpass_inv<R, LEN>(g.tr, 0, 0)); \
              upd(lds_rpass_inv<R, LEN>(g.tr, 0, kFinalSums)); break;
    OFDFT_LENGTHS(OFDFT_LDS3)
#undef OFDFT_LDS3
    default: break;
  }
  switch (g.n2) {
#define OFDFT_LDS2(LEN) case LEN: upd(lds_x2<R, LEN>(g.rb)); break;
    OFDFT_LENGTHS(OFDFT_LDS2)
#undef OFDFT_LDS2
    default: break;
  }
  switch (g.n1) {
#define OFDFT_LDS1(LEN) case LEN: upd(lds_x1<R, LEN>(g.tc, 2)); break;
    OFDFT_LENGTHS(OFDFT_LDS1)
#undef OFDFT_LDS1
    default: break;
  }
  if (plane_mode(c)) {
    switch (g.n3) {
#define OFDFT_LDSP(LEN) case LEN: upd(lds_plane<R, LEN>(kFinalSums)); break;
      OFDFT_PLANE_LENGTHS(OFDFT_LDSP)
#undef OFDFT_LDSP
      default: break;
    }
  }
  return m;
}

size_t dev_max_lds(const ofdft_ctx* c) {
  return c->rsize == 4 ? max_lds_impl<float>(c) : max_lds_impl<double>(c);
}

// Next readback slot of c->hmap.
static Publish next_publish(ofdft_ctx* c) {
  return Publish{c->dmap, reinterpret_cast<unsigned long long*>(c->dmap + kMapDoubles), ++c->read_seq};
}

// Wait until the device has raised the sequence word to seq, then copy n doubles
// out.  While waiting, the stream is polled now and then so that a failed launch
// or a drained stream without the word ends the wait with an error.  After the
// first few thousand polls the thread yields between polls, so that many
// contexts waiting at once (a batch) do not starve each other's launches.
static int wait_published(ofdft_ctx* c, unsigned long long seq, int n, double* host) {
  const volatile unsigned long long* flag = reinterpret_cast<unsigned long long*>(c->hmap + kMapDoubles);
  for (unsigned spin = 1;; ++spin) {
    if (__atomic_load_n(flag, __ATOMIC_ACQUIRE) == seq) break;
    if (spin > 4096) std::this_thread::yield();
    if ((spin & 255u) == 0) {
      const hipError_t e = hipStreamQuery(c->stream);
      if (e == hipSuccess) {
        if (__atomic_load_n(flag, __ATOMIC_ACQUIRE) == seq) break;
        return dev_fail(c, OFDFT_E_DEVICE, "readback: the stream drained without raising the sequence word");
      }
      if (e != hipErrorNotReady) {
        hip_ok(c, e, "readback");
        return OFDFT_E_DEVICE;
      }
    }
    __builtin_ia32_pause();
  }
  for (int k = 0; k < n; ++k) host[k] = c->hmap[k];
  return OFDFT_OK;
}

int dev_eval(ofdft_ctx* c, const double* phi, void* v_out, double* sc, double* host) {
  const Publish pub = host ? next_publish(c) : Publish{nullptr, nullptr, 0};
  int rc = c->rsize == 4 ? eval_impl<float>(c, phi, v_out, sc, nullptr, nullptr, pub)
                         : eval_impl<double>(c, phi, v_out, sc, nullptr, nullptr, pub);
  if (rc || !host) return rc;
  return wait_published(c, pub.seq, SC_COUNT, host);
}

int dev_eval_trial_dev(ofdft_ctx* c, const double* phi, const double* dir, const double* coef, double* phi_out,
                       void* v_out, double* sc, const double* extra, double* host) {
  const Rotation rot{dir, 0.0, 0.0, phi_out, coef};
  const Slope sl{phi, dir, 0.0, 0.0, coef};
  Publish pub = next_publish(c);
  pub.extra = extra;
  pub.n_extra = SC_COUNT;
  int rc = c->rsize == 4 ? eval_impl<float>(c, phi, v_out, sc, &rot, &sl, pub)
                         : eval_impl<double>(c, phi, v_out, sc, &rot, &sl, pub);
  if (rc) return rc;
  return wait_published(c, pub.seq, 2 * SC_COUNT, host);
}

int dev_eval_trial(ofdft_ctx* c, const double* phi, const double* dir, double ca, double sb, double* phi_out,
                   void* v_out, double* sc, double ms, double mc, double* host) {
  const Rotation rot{dir, ca, sb, phi_out};
  const Slope sl{phi, dir, ms, mc};
  const Publish pub = host ? next_publish(c) : Publish{nullptr, nullptr, 0};
  int rc = c->rsize == 4 ? eval_impl<float>(c, phi, v_out, sc, &rot, &sl, pub)
                         : eval_impl<double>(c, phi, v_out, sc, &rot, &sl, pub);
  if (rc || !host) return rc;
  return wait_published(c, pub.seq, SC_COUNT, host);
}

// ---------------------------------------------------------------- allocation
template <typename T>
static bool dalloc(ofdft_ctx* c, T** p, size_t n) {
  void* q = nullptr;
  const bool ok = hip_ok(c, ctx_malloc(c, &q, (n ? n : 1) * sizeof(T)), "device allocation");
  *p = reinterpret_cast<T*>(q);
  return ok;
}
static bool dalloc_bytes(ofdft_ctx* c, void** p, size_t bytes) {
  return hip_ok(c, ctx_malloc(c, p, bytes), "device allocation");
}

template <typename R>
static bool upload_twiddles(ofdft_ctx* c) {
  const int ns[3] = {c->g.n1, c->g.n2, c->g.n3};
  for (int a = 0; a < 3; ++a) {
    std::vector<cplx<R>> h(ns[a]);
    for (int m = 0; m < ns[a]; ++m) {
      const long double ang = -2.0L * 3.141592653589793238462643383279502884L * m / ns[a];
      h[m] = cplx<R>{R(cosl(ang)), R(sinl(ang))};
    }
    if (!dalloc_bytes(c, &c->tw[a], ns[a] * sizeof(cplx<R>))) return false;
    if (!hip_ok(c, hipMemcpy(c->tw[a], h.data(), ns[a] * sizeof(cplx<R>), hipMemcpyHostToDevice), "twiddles"))
      return false;
  }
  return true;
}

// Opt a kernel into the 160 KB of LDS a CDNA4 workgroup can hold: the dynamic
// limit is what its static LDS leaves.  A failure only keeps the default limit;
// the error is consumed here so that it cannot surface at a later launch check.
static void allow_large_lds(const void* f) {
  hipFuncAttributes a{};
  size_t stat = 0;
  if (hipFuncGetAttributes(&a, f) == hipSuccess) stat = a.sharedSizeBytes;
  (void)hipFuncSetAttribute(f, hipFuncAttributeMaxDynamicSharedMemorySize, (int)(160 * 1024 - stat));
  (void)hipGetLastError();
}

template <typename R, int L, int U>
static void allow_x1() {
  allow_large_lds((const void*)k_x1_density<R, L, X1_TF, U>);
  allow_large_lds((const void*)k_x1_density<R, L, X1_GGA, U>);
  allow_large_lds((const void*)k_x1_density<R, L, X1_NHAT, U>);
  allow_large_lds((const void*)k_x1_density<R, L, X1_PREC, U>);
  allow_large_lds((const void*)k_x1_divergence<R, L, U>);
}

template <typename R, int L>
static void allow_x2() {
  allow_large_lds((const void*)k_cpass_x2<R, L, -1, 1>);
  allow_large_lds((const void*)k_cpass_x2<R, L, -1, 2>);
  allow_large_lds((const void*)k_cpass_x2<R, L, -1, 4>);
  allow_large_lds((const void*)k_cpass_x2<R, L, -1, 8>);
  allow_large_lds((const void*)k_cpass_x2<R, L, -1, 16>);
  allow_large_lds((const void*)k_cpass_x2<R, L, +1, 1>);
  allow_large_lds((const void*)k_cpass_x2<R, L, +1, 2>);
  allow_large_lds((const void*)k_cpass_x2<R, L, +1, 4>);
  allow_large_lds((const void*)k_cpass_x2<R, L, +1, 8>);
  allow_large_lds((const void*)k_cpass_x2<R, L, +1, 16>);
}

template <typename R>
static void configure_lds() {
  // Opt every kernel into the large CDNA4 LDS.
  auto allow = [](const void* f) { allow_large_lds(f); };
#define OFDFT_ALLOW(LEN)                                                             \
  allow((const void*)k_rpass_fwd_density<R, LEN, false>);                            \
  allow((const void*)k_rpass_fwd_density<R, LEN, true>);                             \
  allow_x2<R, LEN>();                                                                \
  allow_x1<R, LEN, 1>();                                                             \
  allow_x1<R, LEN, 2>();                                                             \
  allow_x1<R, LEN, 4>();                                                             \
  allow_x1<R, LEN, 8>();                                                             \
  allow((const void*)k_rpass_final<R, LEN, true, false>);                            \
  allow((const void*)k_rpass_final<R, LEN, false, false>);                           \
  allow((const void*)k_rpass_final<R, LEN, true, true>);                             \
  allow((const void*)k_rpass_final<R, LEN, false, true>);                            \
  allow((const void*)k_rpass_inv_real<R, LEN>);                                      \
  allow((const void*)k_rpass_fwd_real<R, LEN>);                                      \
  allow((const void*)k_rpass_fwd_grad<R, LEN>);
  OFDFT_LENGTHS(OFDFT_ALLOW)
#undef OFDFT_ALLOW
#define OFDFT_ALLOW_PLANE(LEN)                                                       \
  allow((const void*)k_plane_fwd_density<R, LEN, false>);                            \
  allow((const void*)k_plane_fwd_density<R, LEN, true>);                             \
  allow((const void*)k_plane_fwd_real<R, LEN, NTP>);                                 \
  allow((const void*)k_plane_fwd_grad<R, LEN>);                                      \
  allow((const void*)k_plane_inv_real<R, LEN, NTP>);                                 \
  allow((const void*)k_plane_final<R, LEN, true, false>);                            \
  allow((const void*)k_plane_final<R, LEN, false, false>);                           \
  allow((const void*)k_plane_final<R, LEN, true, true>);                             \
  allow((const void*)k_plane_final<R, LEN, false, true>);
  OFDFT_PLANE_LENGTHS(OFDFT_ALLOW_PLANE)
#undef OFDFT_ALLOW_PLANE
}


int dev_alloc_grid(ofdft_ctx* c) {
  dev_free_grid(c);
  {
    // the pointwise kernels run one resident round of blocks over a grid-stride loop
    int cus = 0;
    if (hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, c->opt.device) != hipSuccess || cus <= 0)
      cus = 256;
    const int xc = c->opt.xc == OFDFT_XC_PZ81 ? 1 : c->opt.xc == OFDFT_XC_KSDT ? 2 : 0;
    c->g.pwb = cus * pointwise_waves_of(c->rsize, xc);
  }
  const GridDesc& g = c->g;
  const size_t rs = c->rsize;
  const size_t N = g.N, NS = g.NS;
  bool ok = dalloc(c, &c->phi, N) && dalloc(c, &c->phi_t, N) && dalloc(c, &c->d, N) && dalloc(c, &c->gprev, N);
  for (int k = 0; k < 4 && ok; ++k) ok = dalloc(c, &c->tn[k], N);
  ok = ok && dalloc_bytes(c, &c->v, N * rs) && dalloc_bytes(c, &c->v_t, N * rs) && dalloc_bytes(c, &c->vloc, N * rs);
  ok = ok && dalloc(c, &c->phi_t2, N) && dalloc_bytes(c, &c->v_t2, N * rs);
  ok = ok && dalloc_bytes(c, &c->A, NS * 2 * rs) && dalloc_bytes(c, &c->S0, NS * 2 * rs) &&
       dalloc_bytes(c, &c->D, NS * 2 * rs) && dalloc_bytes(c, &c->Vext, NS * 2 * rs);
  for (int k = 0; k < 3 && ok; ++k) ok = dalloc_bytes(c, &c->B[k], NS * 2 * rs);
  ok = ok && dalloc(c, &c->sfac, 4 * NS);
  // sized for the smallest tiles the tuner may pick (2 rows / 2 columns per block)
  const int nb_r = (g.n2 / 2) * g.n1, nb_x1 = (g.n2 / 2) * g.n3h;
  c->max_blocks = std::max(std::max(nb_r, nb_x1), PW_BLOCKS);
  for (int k = 0; k < 3 && ok; ++k) ok = dalloc_bytes(c, &c->gr[k], N * rs);
  ok = ok && dalloc(c, &c->partials, (size_t)SL_COUNT * c->max_blocks) && dalloc(c, &c->scalars, SC_COUNT) &&
       dalloc(c, &c->scalars_t, SC_COUNT) && dalloc(c, &c->scalars_t2, SC_COUNT) &&
       dalloc(c, &c->vpart, 8 * VEC_BLOCKS) && dalloc(c, &c->vout, 32) && dalloc(c, &c->cgst, CG_COUNT);
  if (ok && !c->hmap) {
    ok = hip_ok(c, hipHostMalloc((void**)&c->hmap, (kMapDoubles + 1) * sizeof(double),
                                 hipHostMallocMapped | hipHostMallocCoherent), "hipHostMalloc (mapped)");
    if (ok) ok = hip_ok(c, hipHostGetDevicePointer((void**)&c->dmap, c->hmap, 0), "hipHostGetDevicePointer");
    if (ok) {
      for (int k = 0; k < kMapDoubles; ++k) c->hmap[k] = 0.0;
      *reinterpret_cast<unsigned long long*>(c->hmap + kMapDoubles) = 0ull;
      c->read_seq = 0;
    }
  }
  ok = ok && (rs == 4 ? upload_twiddles<float>(c) : upload_twiddles<double>(c));
  if (ok) {
    static bool lds_f = false, lds_d = false;
    if (rs == 4 && !lds_f) { configure_lds<float>(); lds_f = true; }
    if (rs == 8 && !lds_d) { configure_lds<double>(); lds_d = true; }
    // the CG direction and previous gradient start at zero (they are read only with a nonzero
    // coefficient, but a fresh allocation is no valid state)
    ok = hip_ok(c, hipMemsetAsync(c->Vext, 0, NS * 2 * rs, c->stream), "memset") &&
         hip_ok(c, hipMemsetAsync(c->d, 0, N * sizeof(double), c->stream), "memset") &&
         hip_ok(c, hipMemsetAsync(c->gprev, 0, N * sizeof(double), c->stream), "memset");
  }
  if (!ok) {
    dev_free_grid(c);
    return OFDFT_E_DEVICE;
  }
  return OFDFT_OK;
}

void dev_free_grid(ofdft_ctx* c) {
  // a caller's allocator may hand the memory out again at once: let pending work finish
  // (hipFree waits by itself)
  if (c->opt.alloc && c->stream) (void)hipStreamSynchronize(c->stream);
  dev_cg_graph_release(c);   // its launches refer to the buffers freed here
  void** ps[] = {(void**)&c->phi, (void**)&c->phi_t, (void**)&c->d, (void**)&c->gprev, (void**)&c->tn[0],
                 (void**)&c->tn[1], (void**)&c->tn[2], (void**)&c->tn[3], &c->v, &c->v_t, &c->vloc, &c->A,
                 &c->S0, &c->D, &c->Vext, &c->B[0], &c->B[1], &c->B[2], &c->tw[0], &c->tw[1], &c->tw[2],
                 (void**)&c->partials, (void**)&c->scalars, (void**)&c->scalars_t, (void**)&c->vpart,
                 (void**)&c->vout, &c->gr[0], &c->gr[1], &c->gr[2], (void**)&c->phi_hist[0],
                 (void**)&c->phi_hist[1], (void**)&c->phi_hist[2], (void**)&c->phi_t2, &c->v_t2,
                 (void**)&c->scalars_t2, (void**)&c->sfac, (void**)&c->cgst};
  for (void** p : ps) {
    ctx_free(c, *p);
    *p = nullptr;
  }
  c->n_hist = 0;
}

// Ion buffers: the phase tables hold nat * (n1 + n2 + n3h) entries, which depends on
// the grid; the charges/coordinates, force partials and forces depend on nat alone.
// Each has its own capacity, so a smaller grid with more ions still reallocates.
// Force kernels: whether one thread per ion runs (many ions), and the row chunks per ion
// (partial sums per ion and component) of that launch: about 4096 blocks in all, at most 1024.
static bool force_per_ion(const ofdft_ctx* c) {
  return c->nat > 0 && (c->ion_forces == 1 || (c->ion_forces < 0 && c->nat >= NT));
}
static int force_part_cap(const ofdft_ctx* c) {
  if (!force_per_ion(c)) return 1024;
  const int nby = (c->nat + NT - 1) / NT;
  return std::min(1024, std::max(1, (4096 + nby - 1) / nby));
}

int dev_alloc_ions(ofdft_ctx* c) {
  const long long M = c->g.n1 + c->g.n2 + c->g.n3h;
  const long long need_phase = (long long)c->nat * M;
  const long long need_part = std::max<long long>(3LL * c->nat * force_part_cap(c), 8LL * PW_BLOCKS + 12 * 1024);
  if (c->opt.alloc && c->stream && (c->phase_cap < need_phase || c->ion_cap < c->nat || c->fpart_cap < need_part))
    (void)hipStreamSynchronize(c->stream);
  if (c->phase_cap < need_phase) {
    ctx_free(c, c->phase);
    c->phase = nullptr;
    c->phase_cap = 0;
    if (!dalloc(c, &c->phase, 2 * (size_t)need_phase)) return OFDFT_E_DEVICE;
    c->phase_cap = need_phase;
  }
  if (c->ion_cap < c->nat) {
    ctx_free(c, c->dZ);
    ctx_free(c, c->dforces);
    c->dZ = nullptr; c->dforces = nullptr;
    c->ion_cap = 0;
    const size_t nat = (size_t)c->nat;
    if (!(dalloc(c, &c->dZ, nat + 4 * nat) && dalloc(c, &c->dforces, 3 * nat))) return OFDFT_E_DEVICE;
    c->ion_cap = c->nat;
  }
  if (c->fpart_cap < need_part) {
    ctx_free(c, c->fpart);
    c->fpart = nullptr;
    c->fpart_cap = 0;
    if (!dalloc(c, &c->fpart, (size_t)need_part)) return OFDFT_E_DEVICE;
    c->fpart_cap = need_part;
  }
  return OFDFT_OK;
}

static LppParams lpp_of(const ofdft_ctx* c) {
  return LppParams{c->opt.lpp == OFDFT_LPP_HA ? 1 : 0, c->opt.lpp_rc, c->opt.lpp_A, c->opt.lpp_qc};
}

// fractional coordinates f = tau . inv(lattice) (row vectors)
static void fractional(const ofdft_ctx* c, std::vector<double>& f) {
  const GridDesc& g = c->g;
  f.resize(3 * c->nat);
  for (int I = 0; I < c->nat; ++I)
    for (int a = 0; a < 3; ++a) {
      // b_a . tau / (2 pi)
      const double* t = &c->tau[3 * I];
      f[3 * I + a] = (g.b[3 * a] * t[0] + g.b[3 * a + 1] * t[1] + g.b[3 * a + 2] * t[2]) /
                     (2.0 * 3.141592653589793238462643383279502884);
    }
}

int dev_structure_factor(ofdft_ctx* c) {
  int rc = dev_alloc_ions(c);
  if (rc) return rc;
  std::vector<double> f;
  fractional(c, f);
  // upload fractional coordinates into the tail of dZ (nat + 3 nat)
  std::vector<double> zf(c->nat + 3 * (size_t)c->nat);
  for (int I = 0; I < c->nat; ++I) zf[I] = c->Z[I];
  for (size_t k = 0; k < f.size(); ++k) zf[c->nat + k] = f[k];
  if (!hip_ok(c, hipMemcpyAsync(c->dZ, zf.data(), zf.size() * sizeof(double), hipMemcpyHostToDevice, c->stream),
              "ions"))
    return OFDFT_E_DEVICE;
  const GridDesc& g = c->g;
  const long long M = g.n1 + g.n2 + g.n3h;
  const int nb1 = (int)std::min<long long>(4096, ((long long)c->nat * M + NT - 1) / NT);
  hipLaunchKernelGGL(k_phase_tables, dim3(nb1), dim3(NT), 0, c->stream, c->nat, c->dZ + c->nat, g,
                     (double2*)c->phase);
  const int nb2 = (int)std::min<long long>(8192, (g.NS + NT - 1) / NT);
  if (c->rsize == 4)
    hipLaunchKernelGGL(k_structure_factor<float>, dim3(nb2), dim3(NT), 0, c->stream, c->nat, c->dZ,
                       (const double2*)c->phase, g, lpp_of(c), (cplx<float>*)c->Vext, (double2*)c->sfac);
  else
    hipLaunchKernelGGL(k_structure_factor<double>, dim3(nb2), dim3(NT), 0, c->stream, c->nat, c->dZ,
                       (const double2*)c->phase, g, lpp_of(c), (cplx<double>*)c->Vext, (double2*)c->sfac);
  // reciprocal-space Ewald energy from S_Z (the host thread sums the rest)
  const int nbe = (int)std::min<long long>(1024, std::max<long long>(1, g.NS / (16LL * NT)));
  hipLaunchKernelGGL(k_ewald_recip, dim3(nbe), dim3(NT), 0, c->stream, (const double2*)c->sfac, g, c->ewald_split,
                     c->fpart);
  hipLaunchKernelGGL((k_vec_final<1>), dim3(1), dim3(NT), 0, c->stream, c->fpart, nbe, c->vout);
  if (!hip_ok(c, hipGetLastError(), "structure factor launch")) return OFDFT_E_DEVICE;
  double er = 0.0;
  rc = dev_read(c, c->vout, 1, &er);
  if (rc) return rc;
  c->E_rec = 0.5 * kFourPi / g.volume * er;
  hipError_t e = hipStreamSynchronize(c->stream);
  return hip_ok(c, e, "structure factor") ? OFDFT_OK : OFDFT_E_DEVICE;
}

template <typename R>
static int forces_impl(ofdft_ctx* c, double* out_host) {
  const GridDesc& g = c->g;
  // n(G) of the current density into A (forward transform, kept modes, 1/N)
  if (plane_mode(c)) {
    OFDFT_DISPATCH_PLANE(g.n3, (launch_plane_fwd_density<R, L_>(c, c->phi, c->A, nullptr)));
  } else {
    OFDFT_DISPATCH(g.n3, (launch_rpass_fwd<R, L_>(c, c->phi, c->A)));
    OFDFT_DISPATCH(g.n2, (launch_x2<R, L_, -1>(c, c->A, nullptr, nullptr, 1)));
  }
  OFDFT_DISPATCH(g.n1, (launch_x1_density<R, L_, X1_NHAT>(c, c->A, c->D, nullptr, nullptr)));
  int nbx;
  if (force_per_ion(c)) {
    // one tile of NT ions per block row; enough row chunks for about 4096 blocks (at most
    // force_part_cap, the partial-sum capacity per force component)
    const int nby = (c->nat + NT - 1) / NT;
    const int nrows = g.n1 * g.n3h;
    const int want = std::min(nrows, force_part_cap(c));
    const int rows_per_chunk = (nrows + want - 1) / want;
    nbx = (nrows + rows_per_chunk - 1) / rows_per_chunk;
    hipLaunchKernelGGL(k_forces_ions<R>, dim3(nbx, nby), dim3(NT), 0, c->stream, c->nat, c->dZ,
                       (const double2*)c->phase, (const cplx<R>*)c->D, (const double2*)c->sfac, c->ewald_split, g,
                       lpp_of(c), rows_per_chunk, c->fpart);
  } else {
    // about sixteen G vectors per thread, so the per-block reduction stays a small share
    nbx = (int)std::min<long long>(1024, std::max<long long>(1, g.NS / (16LL * NT)));
    const int nby = (c->nat + FORCE_IONS - 1) / FORCE_IONS;
    hipLaunchKernelGGL(k_forces<R>, dim3(nbx, nby), dim3(NT), 0, c->stream, c->nat, c->dZ,
                       (const double2*)c->phase, (const cplx<R>*)c->D, (const double2*)c->sfac, c->ewald_split, g,
                       lpp_of(c), c->fpart);
  }
  hipLaunchKernelGGL(k_forces_final, dim3((3 * c->nat + NT / 64 - 1) / (NT / 64)), dim3(NT), 0, c->stream, c->nat,
                     c->fpart, nbx, -g.volume, c->dforces);
  if (!hip_ok(c, hipMemcpyAsync(out_host, c->dforces, 3 * (size_t)c->nat * sizeof(double), hipMemcpyDeviceToHost,
                                c->stream),
              "forces copy"))
    return OFDFT_E_DEVICE;
  hipError_t e = hipStreamSynchronize(c->stream);
  return hip_ok(c, e, "forces") ? OFDFT_OK : OFDFT_E_DEVICE;
}

int dev_forces(ofdft_ctx* c, double* forces_host) {
  return c->rsize == 4 ? forces_impl<float>(c, forces_host) : forces_impl<double>(c, forces_host);
}

// Stress sums at the current density: out[0..7] the local sums of k_stress_local
// (times dv), out[8..19] the reciprocal sums of k_stress_recip.
template <typename R>
static int stress_impl(ofdft_ctx* c, double* out_host) {
  const GridDesc& g = c->g;
  const bool tf = c->opt.functional == OFDFT_TF;
  const EvalParams ep = make_params(c);
  // n(G) into D (kept modes, 1/N), and for a gradient functional grad n into gr[0..2]
  if (plane_mode(c)) {
    OFDFT_DISPATCH_PLANE(g.n3, (launch_plane_fwd_density<R, L_>(c, c->phi, c->A, nullptr)));
  } else {
    OFDFT_DISPATCH(g.n3, (launch_rpass_fwd<R, L_>(c, c->phi, c->A)));
    OFDFT_DISPATCH(g.n2, (launch_x2<R, L_, -1>(c, c->A, nullptr, nullptr, 1)));
  }
  OFDFT_DISPATCH(g.n1, (launch_x1_density<R, L_, X1_NHAT>(c, c->A, c->D, nullptr, nullptr)));
  if (!tf) {
    OFDFT_DISPATCH(g.n1, (launch_x1_density<R, L_, X1_GGA>(c, c->A, c->B[0], c->B[1], c->B[2])));
    if (plane_mode(c)) {
      OFDFT_DISPATCH_PLANE(g.n3, (launch_plane_inv_real<R, L_>(c, c->B[0], c->B[1], c->B[2], c->gr[0], c->gr[1],
                                                               c->gr[2], 3)));
    } else {
      OFDFT_DISPATCH(g.n2, (launch_x2<R, L_, +1>(c, c->B[0], c->B[1], c->B[2], 3)));
      OFDFT_DISPATCH(g.n3, (launch_rpass_inv_real3<R, L_>(c)));
    }
  }
  const int nbl = pw_blocks(g);
  if (tf)
    hipLaunchKernelGGL((k_stress_local<R, true>), dim3(nbl), dim3(NT), 0, c->stream, c->phi, (const R*)nullptr,
                       (const R*)nullptr, (const R*)nullptr, g.N, ep, c->fpart);
  else
    hipLaunchKernelGGL((k_stress_local<R, false>), dim3(nbl), dim3(NT), 0, c->stream, c->phi, (const R*)c->gr[0],
                       (const R*)c->gr[1], (const R*)c->gr[2], g.N, ep, c->fpart);
  hipLaunchKernelGGL((k_vec_final<8>), dim3(1), dim3(NT), 0, c->stream, c->fpart, nbl, c->vout);
  const int nbr = (int)std::min<long long>(1024, std::max<long long>(1, g.NS / (16LL * NT)));
  hipLaunchKernelGGL(k_stress_recip<R>, dim3(nbr), dim3(NT), 0, c->stream, (const double2*)c->sfac,
                     (const cplx<R>*)c->D, g, lpp_of(c), c->ewald_split, c->fpart + 8 * (size_t)nbl);
  hipLaunchKernelGGL((k_vec_final<12>), dim3(1), dim3(NT), 0, c->stream, c->fpart + 8 * (size_t)nbl, nbr,
                     c->vout + 8);
  if (!hip_ok(c, hipGetLastError(), "stress launch")) return OFDFT_E_DEVICE;
  double h[20];
  int rc = dev_read(c, c->vout, 20, h);
  if (rc) return rc;
  for (int k = 0; k < 8; ++k) out_host[k] = h[k] * g.dv;
  for (int k = 8; k < 20; ++k) out_host[k] = h[k];
  return OFDFT_OK;
}

int dev_stress(ofdft_ctx* c, double* sums) {
  return c->rsize == 4 ? stress_impl<float>(c, sums) : stress_impl<double>(c, sums);
}

// ---------------------------------------------------------------- vector-op launchers
template <int K, class Op>
static int run_vec(ofdft_ctx* c, const Op& op, double* out = nullptr) {
  hipLaunchKernelGGL((k_vec<K, Op>), dim3(VEC_BLOCKS), dim3(NT), 0, c->stream, c->g.N, op, c->vpart, c->g.gate);
  if constexpr (K > 0)
    hipLaunchKernelGGL((k_vec_final<K>), dim3(1), dim3(NT), 0, c->stream, c->vpart, VEC_BLOCKS,
                       out ? out : c->vout);
  return hip_ok(c, hipGetLastError(), "vector op") ? OFDFT_OK : OFDFT_E_DEVICE;
}

int dev_grad_dots(ofdft_ctx* c, const double* phi, const void* v, const double* sc, const double* gprev,
                  const double* d, double* out) {
  const double two_dv = 2.0 * c->g.dv;
  if (c->rsize == 4) return run_vec<4>(c, OpGradDots<float>{phi, (const float*)v, sc, gprev, d, two_dv}, out);
  return run_vec<4>(c, OpGradDots<double>{phi, (const double*)v, sc, gprev, d, two_dv}, out);
}

int dev_cg_direction(ofdft_ctx* c, double beta, double cproj) {
  const double two_dv = 2.0 * c->g.dv;
  if (c->rsize == 4)
    return run_vec<2>(c, OpDirection<float>{c->phi, (const float*)c->v, c->scalars, c->gprev, c->d, two_dv, beta,
                                            cproj, 0});
  return run_vec<2>(c, OpDirection<double>{c->phi, (const double*)c->v, c->scalars, c->gprev, c->d, two_dv, beta,
                                           cproj, 0});
}

template <typename R, int L>
static void launch_rpass_fwd_grad(ofdft_ctx* c, const double* phi, const void* v, const double* sc, double two_dv,
                                  void* out) {
  const GridDesc& g = c->g;
  hipLaunchKernelGGL((k_rpass_fwd_grad<R, L>), dim3(g.n2 / g.tr, g.n1), dim3(NT), (lds_rpass_fwd<R, L>(g.tr)),
                     c->stream, phi, (const R*)v, sc, two_dv, (cplx<R>*)out, (const cplx<R>*)c->tw[2], g);
}

// Reduce the K dots the op accumulates and form the CG coefficients (k_cg_dots_final).
template <int K, class Op>
static int run_cg_dots(ofdft_ctx* c, const Op& op, const CgCoef& cf) {
  hipLaunchKernelGGL((k_vec<K, Op>), dim3(VEC_BLOCKS), dim3(NT), 0, c->stream, c->g.N, op, c->vpart, c->g.gate);
  hipLaunchKernelGGL((k_cg_dots_final<K>), dim3(1), dim3(NT), 0, c->stream, c->vpart, VEC_BLOCKS, c->scalars, cf);
  return hip_ok(c, hipGetLastError(), "CG dots") ? OFDFT_OK : OFDFT_E_DEVICE;
}

// The direction pass of a CG step: d, gprev and its dots reduced by k_dir_final.
template <class Op>
static int run_direction(ofdft_ctx* c, const Op& op, const TrialCoef& tc) {
  hipLaunchKernelGGL((k_vec<2, Op>), dim3(VEC_BLOCKS), dim3(NT), 0, c->stream, c->g.N, op, c->vpart, c->g.gate);
  hipLaunchKernelGGL(k_dir_final, dim3(1), dim3(NT), 0, c->stream, c->vpart, VEC_BLOCKS, c->scalars, tc);
  return hip_ok(c, hipGetLastError(), "CG direction") ? OFDFT_OK : OFDFT_E_DEVICE;
}

// st (graph mode): have_prev, gg_prev, cproj, F_prev and kappa are read on the device from
// the CG state instead of the host arguments.
template <typename R>
static int cg_step_impl(ofdft_ctx* c, bool pcg, bool have_prev, double gg_prev, double cproj, double F_prev,
                        double r, double kappa, const double* st = nullptr) {
  const TrialCoef tc{F_prev, have_prev ? 1 : 0, r, c->g.dv, kappa, st, c->g.gate};
  const GridDesc& g = c->g;
  const double two_dv = 2.0 * g.dv;
  const double* phi = c->phi;
  const R* v = (const R*)c->v;
  const double* gprev = (have_prev || st) ? c->gprev : nullptr;
  const CgCoef cf{pcg ? 1 : 0, have_prev ? 1 : 0, gg_prev, g.dv, st, c->g.gate};
  int rc;
  if (pcg) {
    // w = (P - 1) g: forward 3D FFT of g, filter in the x1 pass, inverse 3D FFT into gr[0];
    // z = g + w, so the modes the passes drop (Nyquist) keep P = 1
    if (plane_mode(c)) {
      OFDFT_DISPATCH_PLANE(g.n3, (launch_plane_fwd_grad<R, L_>(c, phi, v, c->scalars, two_dv, c->B[0])));
      OFDFT_DISPATCH(g.n1, (launch_x1_density<R, L_, X1_PREC>(c, c->B[0], c->B[0], nullptr, nullptr)));
      OFDFT_DISPATCH_PLANE(g.n3, (launch_plane_inv_real<R, L_>(c, c->B[0], nullptr, nullptr, c->gr[0], nullptr,
                                                               nullptr, 1)));
    } else {
      OFDFT_DISPATCH(g.n3, (launch_rpass_fwd_grad<R, L_>(c, phi, v, c->scalars, two_dv, c->B[0])));
      OFDFT_DISPATCH(g.n2, (launch_x2<R, L_, -1>(c, c->B[0], nullptr, nullptr, 1)));
      OFDFT_DISPATCH(g.n1, (launch_x1_density<R, L_, X1_PREC>(c, c->B[0], c->B[0], nullptr, nullptr)));
      OFDFT_DISPATCH(g.n2, (launch_x2<R, L_, +1>(c, c->B[0], nullptr, nullptr, 1)));
      OFDFT_DISPATCH(g.n3, (launch_rpass_inv_real1<R, L_>(c, c->B[0], c->gr[0])));
    }

    rc = run_cg_dots<5>(c, OpPrecDots<R>{phi, v, (const R*)c->gr[0], c->scalars, gprev, two_dv, st}, cf);
    if (rc) return rc;
    return run_direction(
        c, OpPrecDirection<R>{phi, v, (const R*)c->gr[0], c->scalars, c->gprev, c->d, two_dv, cproj, 0, st}, tc);
  }
  rc = run_cg_dots<4>(c, OpGradDots<R>{phi, v, c->scalars, gprev, (have_prev || st) ? c->d : nullptr, two_dv, st},
                      cf);
  if (rc) return rc;
  return run_direction(c, OpDirection<R>{phi, v, c->scalars, c->gprev, c->d, two_dv, 0.0, cproj, 1, st}, tc);
}

int dev_cg_step(ofdft_ctx* c, bool pcg, bool have_prev, double gg_prev, double cproj, double F_prev, double r,
                double kappa) {
  return c->rsize == 4 ? cg_step_impl<float>(c, pcg, have_prev, gg_prev, cproj, F_prev, r, kappa)
                       : cg_step_impl<double>(c, pcg, have_prev, gg_prev, cproj, F_prev, r, kappa);
}

template <typename R>
static int cg_restart_impl(ofdft_ctx* c, bool pcg) {
  const double two_dv = 2.0 * c->g.dv;
  const R* v = (const R*)c->v;
  if (pcg)
    return run_vec<2>(c, OpPrecDirection<R>{c->phi, v, (const R*)c->gr[0], c->scalars, c->gprev, c->d, two_dv, 0.0, 1},
                      c->scalars + SC_DD);
  return run_vec<2>(c, OpDirection<R>{c->phi, v, c->scalars, c->gprev, c->d, two_dv, 0.0, 0.0, 0},
                    c->scalars + SC_DD);
}

int dev_cg_restart(ofdft_ctx* c, bool pcg) {
  return c->rsize == 4 ? cg_restart_impl<float>(c, pcg) : cg_restart_impl<double>(c, pcg);
}

int dev_rotate(ofdft_ctx* c, double* dst, const double* phi, double ca, const double* dir, double sb) {
  return run_vec<0>(c, OpRotate{dst, phi, dir, ca, sb});
}

int dev_dtheta(ofdft_ctx* c, const double* phi_t, const void* v_t, const double* sc_t, const double* phi,
               const double* d, double ms, double mc, double* out) {
  const double two_dv = 2.0 * c->g.dv;
  if (c->rsize == 4)
    return run_vec<1>(c, OpDtheta<float>{phi_t, (const float*)v_t, sc_t, phi, d, two_dv, ms, mc}, out);
  return run_vec<1>(c, OpDtheta<double>{phi_t, (const double*)v_t, sc_t, phi, d, two_dv, ms, mc}, out);
}

int dev_full_grad_acc(ofdft_ctx* c, double* out, const double* phi_t, const void* v_t, double sign) {
  const double two_dv = 2.0 * c->g.dv;
  const int init = sign > 0 ? 1 : 0;
  if (c->rsize == 4) return run_vec<0>(c, OpFullGradAcc<float>{out, phi_t, (const float*)v_t, two_dv, sign, init});
  return run_vec<0>(c, OpFullGradAcc<double>{out, phi_t, (const double*)v_t, two_dv, sign, init});
}

int dev_dot(ofdft_ctx* c, const double* a, const double* b) { return run_vec<1>(c, OpDot{a, b}); }

int dev_axpby(ofdft_ctx* c, double* y, double a, const double* x, double b) {
  return run_vec<0>(c, OpAxpby{y, x, a, b});
}

int dev_combine3(ofdft_ctx* c, double* dst, double c0, const double* x0, double c1, const double* x1, double c2,
                 const double* x2) {
  return run_vec<1>(c, OpCombine3{dst, x0, x1, c2 != 0.0 ? x2 : nullptr, c0, c1, c2});
}

int dev_tn_hess_finish(ofdft_ctx* c, double* hs, const double* phi, const double* s, double inv2e, double mu_term) {
  (void)s;
  (void)mu_term;
  return run_vec<1>(c, OpHessScale{hs, phi, inv2e});
}

// ---------------------------------------------------------------- HIP-graph CG iteration
// One CG iteration as a fixed sequence of launches that a HIP graph can replay, every
// decision taken on the device in FP64 from the CG state st (CgSlot):
//   CG step (gate ACTIVE)      preconditioned gradient, PR+ coefficients, direction d and
//                              the first trial angle theta1 (the rule of the host CG)
//   k_cg_check                 stop rule on the residual, max_iter, descent check
//   trial 1 (gate GATE1)       evaluation at theta1 with dF/dtheta
//   k_ls_decide1               accept theta1 (strong-Wolfe test of the host line search)
//                              or place theta2 by the secant of the slopes at 0 and theta1
//                              (or the quadratic through F(0), F'(0), F(theta1))
//   trial 2 (gate GATE2)       evaluation at theta2
//   k_ls_decide2               take the lower of the trials that decrease F, update the CG
//                              history and the energy-change stop, handle a stall; publish
//                              the status to the host
//   k_accept (gate GATEACC)    copy the taken trial (phi, v, scalars) into the current state
// A converged or failed minimisation clears ACTIVE, and every later launch returns at once.

__device__ __forceinline__ bool fin(double x) { return isfinite(x); }

// Resolution of F: FP64 rounding (1e-14 |F|), or in the mixed path the FP32 rounding of its
// terms, ~5e-10 of S = |F_s| + |E_xc| + |E_H| + |E_ext| + |E_alphaZ| (the magnitudes that are
// summed; a change of F below this is no resolvable progress).
__device__ __forceinline__ double term_scale(const double* sc) {
  return fabs(sc[SC_FS]) + fabs(sc[SC_EXC]) + fabs(sc[SC_EH]) + fabs(sc[SC_EEXT]) + fabs(sc[SC_EAZ]);
}
__device__ __forceinline__ double f_resolution(const double* sc, double F0, const CgConst& k) {
  return k.mixed ? 5e-10 * term_scale(sc) : 1e-14 * fabs(F0);
}

__global__ void k_cg_init(double* __restrict__ st, const double* __restrict__ sc) {
  if (threadIdx.x != 0) return;
  for (int k = 0; k < CG_COUNT; ++k) st[k] = 0.0;
  st[CG_F] = sc[SC_FTOT];
  st[CG_EVALS] = 1.0;   // the starting evaluation
  if (isfinite(sc[SC_FTOT])) {
    st[CG_ACTIVE] = 1.0;
  } else {
    st[CG_STATUS] = CGS_NONFINITE;
  }
}

// Stop rule and descent check after the direction kernels.
__global__ void k_cg_check(double* __restrict__ st, const double* __restrict__ sc, CgConst k) {
  if (threadIdx.x != 0) return;
  st[CG_GATE1] = 0.0;
  st[CG_GATE2] = 0.0;
  st[CG_GATEACC] = 0.0;
  st[CG_SRC] = 0.0;
  if (st[CG_ACTIVE] == 0.0) return;
  const double gg = sc[SC_DOT0];
  const double resid = sqrt(sc[SC_DOT0 + 3] / (sc[SC_NE] / k.dv));
  st[CG_GG] = gg;
  st[CG_RESID] = resid;
  if (gg <= 0.0 || (st[CG_SMALL] >= 2.0 && (k.tol_residual <= 0.0 || resid < k.tol_residual))) {
    st[CG_ACTIVE] = 0.0;
    st[CG_CONVERGED] = 1.0;
    st[CG_STATUS] = CGS_CONVERGED;
    return;
  }
  if (st[CG_ITERS] >= k.max_iter) {
    st[CG_ACTIVE] = 0.0;
    st[CG_STATUS] = CGS_MAXITER;
    return;
  }
  const double dd = sc[SC_DD], dg = sc[SC_DG];
  if (!(dg < 0.0) || !(dd > 0.0)) {
    // not a descent direction: the next iteration restarts along -g (-z)
    st[CG_HAVE_PREV] = 0.0;
    st[CG_KAPPA] = 0.0;
    st[CG_ITERS] += 1.0;
    return;
  }
  const double dn = sqrt(dd);
  st[CG_DN] = dn;
  st[CG_DF0] = k.r * dg / dn;
  st[CG_GATE1] = 1.0;
  st[CG_EVALS] += 1.0;
}

__device__ __forceinline__ void trial_coefs(double th, double r, double dn, double ne_over_dv, double* out) {
  const double ratio = r / sqrt(ne_over_dv);
  const double ct = cos(th), st_ = sin(th);
  out[0] = ct * ratio;
  out[1] = st_ * r / dn;
  out[2] = -st_ * ratio;
  out[3] = ct * r / dn;
}

// First trial: accept it, or place the second one.  Non-finite trial: restart once.
__global__ void k_ls_decide1(double* __restrict__ st, const double* __restrict__ sc,
                             const double* __restrict__ sc1, CgConst k) {
  if (threadIdx.x != 0) return;
  if (st[CG_GATE1] == 0.0) return;
  const double F0 = st[CG_F], dF0 = st[CG_DF0], th1 = sc[SC_TH1];
  double F1 = sc1[SC_FTOT];
  const double d1 = sc1[SC_DOT0];
  st[CG_TRIALS] += 1.0;
  if (k.inject_at != 0 && (k.inject_at < 0 || st[CG_TRIALS] == (double)k.inject_at)) F1 = NAN;
  if (!fin(F1) || !fin(d1)) {
    if (st[CG_NF_USED] == 0.0) {
      st[CG_NF_USED] = 1.0;
      st[CG_HAVE_PREV] = 0.0;
      st[CG_KAPPA] = 0.0;
      st[CG_SMALL] = 0.0;
    } else {
      st[CG_ACTIVE] = 0.0;
      st[CG_STATUS] = CGS_NONFINITE;
    }
    st[CG_GATE1] = 0.0;   // nothing to take from this iteration
    st[CG_ITERS] += 1.0;
    return;
  }
  st[CG_F1] = F1;
  st[CG_D1] = d1;
  const bool armijo = F1 <= F0 + 1e-4 * th1 * dF0;
  const bool flat = F1 <= F0 + f_resolution(sc, F0, k);
  if ((armijo || flat) && fabs(d1) <= 0.1 * fabs(dF0)) {
    st[CG_SRC] = 1.0;
    return;
  }
  double th2;
  if (armijo && d1 < 0.0) {
    // still descending at theta1: extrapolate with the secant of the slope
    th2 = d1 > dF0 ? th1 * dF0 / (dF0 - d1) : 4.0 * th1;
    th2 = fmin(fmax(th2, 1.5 * th1), 4.0 * th1);
  } else {
    // the minimum lies inside (0, theta1).  With only one more trial the secant is trusted
    // down to 1e-6 theta1: a first trial far past the minimum (a restart near convergence)
    // is then corrected in one step, where a bisecting search would need many.
    if (d1 > 0.0) {
      th2 = th1 * dF0 / (dF0 - d1);
    } else {
      const double curv = F1 - F0 - dF0 * th1;
      th2 = curv > 0.0 ? -0.5 * dF0 * th1 * th1 / curv : 0.5 * th1;
    }
    th2 = fmin(fmax(th2, 1e-6 * th1), 0.9 * th1);
  }
  st[CG_TH2] = th2;
  trial_coefs(th2, k.r, st[CG_DN], sc[SC_NE] / k.dv, st + CG_COEF2);
  st[CG_GATE2] = 1.0;
  st[CG_EVALS] += 1.0;
}

// Take a trial (or handle the stall), update the history and the stop rule, publish.
__global__ void k_ls_decide2(double* __restrict__ st, const double* __restrict__ sc,
                             const double* __restrict__ sc1, const double* __restrict__ sc2, CgConst k,
                             double* __restrict__ hmap) {
  if (threadIdx.x != 0) return;
  st[CG_LAUNCHES] += 1.0;
  if (st[CG_ACTIVE] != 0.0 && st[CG_GATE1] != 0.0) {
    const double F0 = st[CG_F], dF0 = st[CG_DF0];
    const double th1 = sc[SC_TH1];
    int take = (int)st[CG_SRC];
    double Ft = 0.0, dt = 0.0, tht = 0.0;
    if (take == 1) {
      Ft = st[CG_F1];
      dt = st[CG_D1];
      tht = th1;
    } else if (st[CG_GATE2] != 0.0) {
      // candidates: a trial that does not raise F beyond its rounding level; between two,
      // the lower F, or the smaller slope once both F sit at the rounding level (there the
      // slope, not F, still carries the information)
      const double F1 = st[CG_F1], d1 = st[CG_D1], F2 = sc2[SC_FTOT], d2 = sc2[SC_DOT0];
      const double th2 = st[CG_TH2];
      const double tol_flat = f_resolution(sc, F0, k);
      const bool ok1 = F1 <= F0 + tol_flat;
      const bool ok2 = fin(F2) && fin(d2) && F2 <= F0 + tol_flat;
      bool two;
      if (ok1 && ok2) {
        two = fabs(F2 - F1) <= tol_flat ? fabs(d2) <= fabs(d1) : F2 < F1;
      } else {
        two = ok2;
      }
      if (two) {
        take = 2; Ft = F2; dt = d2; tht = th2;
      } else if (ok1) {
        take = 1; Ft = F1; dt = d1; tht = th1;
      }
    }
    st[CG_ITERS] += 1.0;
    if (take) {
      const double dF = F0 - Ft;
      st[CG_LAST_DF] = dF;
      st[CG_F_PREV] = F0;
      st[CG_F] = Ft;
      st[CG_GG_PREV] = st[CG_GG];
      st[CG_KAPPA] = (tht > 0.0 && dt > dF0) ? (dt - dF0) / tht : 0.0;
      st[CG_CPROJ] = sin(tht) * st[CG_DN] / k.r;
      st[CG_HAVE_PREV] = 1.0;
      // mixed path: a change below the resolution of F counts toward the stop like a change
      // below tol_energy
      const double resolvable = k.mixed ? f_resolution(sc, F0, k) : 0.0;
      st[CG_SMALL] = fabs(dF) < fmax(k.tol_energy, resolvable) ? st[CG_SMALL] + 1.0 : 0.0;
      st[CG_SRC] = take;
      st[CG_GATEACC] = 1.0;
      st[CG_THCAP] = 0.0;
      if (st[CG_SMALL] >= 2.0 && k.tol_residual <= 0.0) {
        st[CG_ACTIVE] = 0.0;
        st[CG_CONVERGED] = 1.0;
        st[CG_STATUS] = CGS_CONVERGED;
      }
    } else {
      // no trial lowers F.  If F is convex along the line it lies nowhere below
      // F0 - |dF0| th_min (th_min the smallest angle tried): below the energy tolerance (or
      // the resolution of F) that counts as converged, like a small last step.  Otherwise
      // restart along -g with the first angle capped at a tenth of th_min, up to three times.
      const bool had_prev = st[CG_HAVE_PREV] != 0.0;
      const double th_min = st[CG_GATE2] != 0.0 ? fmin(th1, st[CG_TH2]) : th1;
      const double bound = fabs(dF0) * th_min;
      const double last = had_prev ? st[CG_LAST_DF] : bound;
      // the mixed path's noise floor (the host CG's 1e-6 |F_tot| in terms of the summed magnitudes)
      const bool floor_ok = k.mixed && fabs(last) < 1e-7 * term_scale(sc);
      const double resolvable = k.mixed ? f_resolution(sc, F0, k) : 0.0;
      const bool conv = k.tol_residual > 0.0
                            ? (st[CG_RESID] < k.tol_residual || floor_ok)
                            : (st[CG_SMALL] >= 1.0 || floor_ok || bound < fmax(k.tol_energy, resolvable));
      if (conv) {
        st[CG_ACTIVE] = 0.0;
        st[CG_CONVERGED] = 1.0;
        st[CG_STATUS] = CGS_CONVERGED;
      } else if (st[CG_LSR_USED] < 3.0) {
        // the last measured curvature still sets the first angle, within the cap
        st[CG_LSR_USED] += 1.0;
        st[CG_HAVE_PREV] = 0.0;
        st[CG_THCAP] = 0.1 * th_min;
      } else {
        st[CG_ACTIVE] = 0.0;
        st[CG_STATUS] = CGS_STALLED;
      }
    }
  }
  // status to the host: the data first, then the launch counter with a system-scope release
  hmap[kMapStatus + 1] = st[CG_ACTIVE];
  hmap[kMapStatus + 2] = st[CG_STATUS];
  hmap[kMapStatus + 3] = st[CG_ITERS];
  hmap[kMapStatus + 4] = st[CG_EVALS];
  hmap[kMapStatus + 5] = st[CG_F];
  __threadfence_system();
  __hip_atomic_store(hmap + kMapStatus, st[CG_LAUNCHES], __ATOMIC_RELEASE, __HIP_MEMORY_SCOPE_SYSTEM);
}

// Copy the taken trial into the current state: phi and v (grid-stride), scalars (block 0).
template <typename R>
__global__ void __launch_bounds__(NT) k_accept(const double* __restrict__ st, double* __restrict__ phi,
                                               R* __restrict__ v, double* __restrict__ sc,
                                               const double* __restrict__ phi1, const R* __restrict__ v1,
                                               const double* __restrict__ sc1, const double* __restrict__ phi2,
                                               const R* __restrict__ v2, const double* __restrict__ sc2, long long n) {
  if (st[CG_GATEACC] == 0.0) return;
  const bool two = st[CG_SRC] == 2.0;
  const double* ps = two ? phi2 : phi1;
  const R* vs = two ? v2 : v1;
  for (long long i = (long long)blockIdx.x * NT + threadIdx.x; i < n; i += (long long)gridDim.x * NT) {
    phi[i] = ps[i];
    v[i] = vs[i];
  }
  if (blockIdx.x == 0 && threadIdx.x < SC_COUNT) sc[threadIdx.x] = (two ? sc2 : sc1)[threadIdx.x];
}

template <typename R>
static int cg_graph_iteration(ofdft_ctx* c, bool pcg, const CgConst& k) {
  double* st = c->cgst;
  const GridDesc saved = c->g;
  int rc;
  // CG step
  c->g.gate = st + CG_ACTIVE;
  rc = cg_step_impl<R>(c, pcg, false, 0.0, 0.0, 0.0, k.r, 0.0, st);
  c->g.gate = nullptr;
  if (rc) { c->g = saved; return rc; }
  hipLaunchKernelGGL(k_cg_check, dim3(1), dim3(64), 0, c->stream, st, (const double*)c->scalars, k);
  // trial 1 at the device angle theta1 (coefficients in scalars[SC_CA..SC_MC])
  {
    c->g.gate = st + CG_GATE1;
    const Rotation rot{c->d, 0.0, 0.0, c->phi_t, c->scalars + SC_CA};
    const Slope sl{c->phi, c->d, 0.0, 0.0, c->scalars + SC_CA};
    rc = eval_impl<R>(c, c->phi, c->v_t, c->scalars_t, &rot, &sl, Publish{nullptr, nullptr, 0, nullptr, 0});
    c->g.gate = nullptr;
    if (rc) { c->g = saved; return rc; }
  }
  hipLaunchKernelGGL(k_ls_decide1, dim3(1), dim3(64), 0, c->stream, st, (const double*)c->scalars,
                     (const double*)c->scalars_t, k);
  {
    c->g.gate = st + CG_GATE2;
    const Rotation rot{c->d, 0.0, 0.0, c->phi_t2, st + CG_COEF2};
    const Slope sl{c->phi, c->d, 0.0, 0.0, st + CG_COEF2};
    rc = eval_impl<R>(c, c->phi, c->v_t2, c->scalars_t2, &rot, &sl, Publish{nullptr, nullptr, 0, nullptr, 0});
    c->g.gate = nullptr;
    if (rc) { c->g = saved; return rc; }
  }
  hipLaunchKernelGGL(k_ls_decide2, dim3(1), dim3(64), 0, c->stream, st, (const double*)c->scalars,
                     (const double*)c->scalars_t, (const double*)c->scalars_t2, k, c->dmap);
  const int nb = (int)std::min<long long>(2048, (c->g.N + NT - 1) / NT);
  hipLaunchKernelGGL((k_accept<R>), dim3(nb), dim3(NT), 0, c->stream, (const double*)st, c->phi, (R*)c->v,
                     c->scalars, (const double*)c->phi_t, (const R*)c->v_t, (const double*)c->scalars_t,
                     (const double*)c->phi_t2, (const R*)c->v_t2, (const double*)c->scalars_t2, c->g.N);
  c->g = saved;
  return hip_ok(c, hipGetLastError(), "graph CG iteration") ? OFDFT_OK : OFDFT_E_DEVICE;
}

void dev_cg_graph_release(ofdft_ctx* c) {
  if (c->cg_exec) (void)hipGraphExecDestroy(c->cg_exec);
  if (c->cg_graph) (void)hipGraphDestroy(c->cg_graph);
  c->cg_exec = nullptr;
  c->cg_graph = nullptr;
}

int dev_cg_graph_prepare(ofdft_ctx* c, bool pcg, const CgConst& k) {
  // the captured launches bake in the grid, tiles, evaluation parameters and constants
  GraphKey key{};
  key.g = c->g;
  key.ep = make_params(c);
  key.k = k;
  key.pcg = pcg;
  key.plane = plane_mode(c);
  const void* bufs[9] = {c->phi, c->v, c->scalars, c->phi_t, c->v_t, c->scalars_t, c->phi_t2, c->v_t2,
                         c->scalars_t2};
  for (int i = 0; i < 9; ++i) key.bufs[i] = bufs[i];
  if (c->cg_exec && std::memcmp(&key, &c->cg_key, sizeof(GraphKey)) == 0) return OFDFT_OK;
  dev_cg_graph_release(c);
  if (!hip_ok(c, hipStreamBeginCapture(c->stream, hipStreamCaptureModeThreadLocal), "graph capture"))
    return OFDFT_E_DEVICE;
  const int rc = c->rsize == 4 ? cg_graph_iteration<float>(c, pcg, k) : cg_graph_iteration<double>(c, pcg, k);
  hipGraph_t graph = nullptr;
  const hipError_t e = hipStreamEndCapture(c->stream, &graph);
  if (rc) {
    if (graph) (void)hipGraphDestroy(graph);
    return rc;
  }
  if (!hip_ok(c, e, "graph capture end")) return OFDFT_E_DEVICE;
  hipGraphExec_t exec = nullptr;
  if (!hip_ok(c, hipGraphInstantiate(&exec, graph, nullptr, nullptr, 0), "graph instantiate")) {
    (void)hipGraphDestroy(graph);
    return OFDFT_E_DEVICE;
  }
  c->cg_graph = graph;
  c->cg_exec = exec;
  c->cg_key = key;
  return OFDFT_OK;
}

int dev_cg_graph_start(ofdft_ctx* c) {
  hipLaunchKernelGGL(k_cg_init, dim3(1), dim3(64), 0, c->stream, c->cgst, (const double*)c->scalars);
  return hip_ok(c, hipGetLastError(), "CG state init") ? OFDFT_OK : OFDFT_E_DEVICE;
}

int dev_cg_graph_launch(ofdft_ctx* c) {
  return hip_ok(c, hipGraphLaunch(c->cg_exec, c->stream), "graph launch") ? OFDFT_OK : OFDFT_E_DEVICE;
}

int dev_read(ofdft_ctx* c, const double* dptr, int n, double* host) {
  if (n < 1 || n > kMapDoubles) return dev_fail(c, OFDFT_E_ARG, "readback size out of range");
  const Publish pub = next_publish(c);
  hipLaunchKernelGGL(k_publish, dim3(1), dim3(64), 0, c->stream, dptr, n, pub);
  if (!hip_ok(c, hipGetLastError(), "readback launch")) return OFDFT_E_DEVICE;
  return wait_published(c, pub.seq, n, host);
}

int dev_sync(ofdft_ctx* c) {
  return hip_ok(c, hipStreamSynchronize(c->stream), "sync") ? OFDFT_OK : OFDFT_E_DEVICE;
}

}  // namespace ofdft
