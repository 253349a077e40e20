// LDS-resident FFT building blocks for CDNA4 (wave64).
//
// The 3D R2C/C2R transforms of the density, its gradient and the divergence
// term (the reciprocal-space parts of arXiv:1406.0835 Sec. III B, Eqs. E2,
// E4A, vftGGA) are assembled from three passes; each pass stages a tile of
// rows in LDS and runs a Stockham auto-sort FFT over them:
//   * a contiguous-axis pass that packs two real rows into one complex row,
//   * passes along the two other axes on the transposed half spectrum
//     S[k3][i1][i2] (k3 slowest), so both are rows of N1 or N2 points.
// Plans are compile-time (radix 8, 4, 2, 3, 5 in that order of preference), so
// every index division in the butterflies is by a constant.
#pragma once
#include <hip/hip_runtime.h>

namespace ofdft {

template <typename R>
struct cplx {
  R x, y;
};

template <typename R>
__device__ __forceinline__ cplx<R> mk(R a, R b) { return cplx<R>{a, b}; }
template <typename R>
__device__ __forceinline__ cplx<R> operator+(cplx<R> a, cplx<R> b) { return {a.x + b.x, a.y + b.y}; }
template <typename R>
__device__ __forceinline__ cplx<R> operator-(cplx<R> a, cplx<R> b) { return {a.x - b.x, a.y - b.y}; }
template <typename R>
__device__ __forceinline__ cplx<R> cmul(cplx<R> a, cplx<R> b) {
  return {a.x * b.x - a.y * b.y, a.x * b.y + a.y * b.x};
}
template <typename R>
__device__ __forceinline__ cplx<R> cconj(cplx<R> a) { return {a.x, -a.y}; }
template <typename R>
__device__ __forceinline__ cplx<R> cscale(cplx<R> a, R s) { return {a.x * s, a.y * s}; }
// multiply by SIGN * i
template <typename R, int SIGN>
__device__ __forceinline__ cplx<R> mul_si(cplx<R> a) {
  return SIGN > 0 ? cplx<R>{-a.y, a.x} : cplx<R>{a.y, -a.x};
}

// ---------------------------------------------------------------- plans
// wide: FP32 transforms also take radix-16 stages (16 complex values per butterfly fit the
// registers in single precision; one LDS pass and two barriers fewer per 16x of length).
__host__ __device__ constexpr int first_radix(int L, bool wide = false) {
  return (wide && L % 16 == 0) ? 16
         : (L % 8 == 0) ? 8 : (L % 4 == 0) ? 4 : (L % 2 == 0) ? 2 : (L % 3 == 0) ? 3 : (L % 5 == 0) ? 5 : 0;
}
// FP32 transforms of length up to 128 take the radix-16 plan (at 128^3: 7.2 k -> 7.5 k
// evaluations/s); at 256 it was slower (946 -> 858 evaluations/s at 256^3), so longer
// transforms and FP64 keep radix 8 first.
template <typename R, int L>
__host__ __device__ constexpr bool wide_plan() {
  return sizeof(R) == 4 && L <= 128;
}
// radix of stage s for length L: stages peel the preferred radix off L
__host__ __device__ constexpr int radix_at(int L, int s, bool wide = false) {
  int rem = L;
  for (int i = 0; i < s; ++i) rem /= first_radix(rem, wide);
  return first_radix(rem, wide);
}
__host__ __device__ constexpr int n_stages(int L, bool wide = false) {
  int s = 0;
  for (int rem = L; rem > 1; rem /= first_radix(rem, wide)) ++s;
  return s;
}
__host__ __device__ constexpr bool supported_length(int L) {
  if (L < 2) return false;
  int rem = L;
  while (rem % 2 == 0) rem /= 2;
  while (rem % 3 == 0) rem /= 3;
  while (rem % 5 == 0) rem /= 5;
  return rem == 1;
}

// ---------------------------------------------------------------- butterflies
template <typename R, int SIGN, int RAD>
struct Bfly;

template <typename R, int SIGN>
struct Bfly<R, SIGN, 2> {
  __device__ __forceinline__ static void run(cplx<R>* v) {
    cplx<R> a = v[0];
    v[0] = a + v[1];
    v[1] = a - v[1];
  }
};

template <typename R, int SIGN>
struct Bfly<R, SIGN, 3> {
  __device__ __forceinline__ static void run(cplx<R>* v) {
    const R c = R(-0.5);
    const R s = R(SIGN) * R(0.86602540378443864676372317075294);
    cplx<R> t1 = v[1] + v[2];
    cplx<R> t2 = v[1] - v[2];
    cplx<R> m = {v[0].x + c * t1.x, v[0].y + c * t1.y};
    v[0] = v[0] + t1;
    v[1] = {m.x - s * t2.y, m.y + s * t2.x};
    v[2] = {m.x + s * t2.y, m.y - s * t2.x};
  }
};

// Five-point DFT y_k = sum_j x_j W^{jk}, W = exp(SIGN 2 pi i / 5), from the pairs
// x1 +- x4 and x2 +- x3: W^1, W^4 = c1 +- i SIGN s1 and W^2, W^3 = c2 +- i SIGN s2 with
// c1 = cos(2 pi/5), s1 = sin(2 pi/5), c2 = cos(4 pi/5), s2 = sin(4 pi/5).
template <typename R, int SIGN>
struct Bfly<R, SIGN, 5> {
  __device__ __forceinline__ static void run(cplx<R>* v) {
    const R c1 = R(0.30901699437494742410229341718281906);
    const R c2 = R(-0.80901699437494742410229341718281906);
    const R s1 = R(SIGN) * R(0.95105651629515357211643933337938214);
    const R s2 = R(SIGN) * R(0.58778525229247312916870595463907277);
    const cplx<R> t1 = v[1] + v[4], t2 = v[2] + v[3];
    const cplx<R> t3 = v[1] - v[4], t4 = v[2] - v[3];
    const cplx<R> a1 = {v[0].x + c1 * t1.x + c2 * t2.x, v[0].y + c1 * t1.y + c2 * t2.y};
    const cplx<R> a2 = {v[0].x + c2 * t1.x + c1 * t2.x, v[0].y + c2 * t1.y + c1 * t2.y};
    // b1 = i (s1 t3 + s2 t4), b2 = i (s2 t3 - s1 t4)
    const cplx<R> u1 = {s1 * t3.x + s2 * t4.x, s1 * t3.y + s2 * t4.y};
    const cplx<R> u2 = {s2 * t3.x - s1 * t4.x, s2 * t3.y - s1 * t4.y};
    v[0] = v[0] + t1 + t2;
    v[1] = {a1.x - u1.y, a1.y + u1.x};
    v[4] = {a1.x + u1.y, a1.y - u1.x};
    v[2] = {a2.x - u2.y, a2.y + u2.x};
    v[3] = {a2.x + u2.y, a2.y - u2.x};
  }
};

template <typename R, int SIGN>
struct Bfly<R, SIGN, 4> {
  __device__ __forceinline__ static void run(cplx<R>* v) {
    cplx<R> a = v[0] + v[2], b = v[0] - v[2];
    cplx<R> c = v[1] + v[3], d = mul_si<R, SIGN>(v[1] - v[3]);
    v[0] = a + c;
    v[2] = a - c;
    v[1] = b + d;
    v[3] = b - d;
  }
};

template <typename R, int SIGN>
struct Bfly<R, SIGN, 8> {
  __device__ __forceinline__ static void run(cplx<R>* v) {
    cplx<R> e[4] = {v[0], v[2], v[4], v[6]};
    cplx<R> o[4] = {v[1], v[3], v[5], v[7]};
    Bfly<R, SIGN, 4>::run(e);
    Bfly<R, SIGN, 4>::run(o);
    const R h = R(0.70710678118654752440084436210485);
    // W^k, W = exp(SIGN 2 pi i / 8)
    cplx<R> o1 = {h * (o[1].x - R(SIGN) * o[1].y), h * (o[1].y + R(SIGN) * o[1].x)};
    cplx<R> o2 = mul_si<R, SIGN>(o[2]);
    cplx<R> o3 = {h * (-o[3].x - R(SIGN) * o[3].y), h * (-o[3].y + R(SIGN) * o[3].x)};
    v[0] = e[0] + o[0];
    v[4] = e[0] - o[0];
    v[1] = e[1] + o1;
    v[5] = e[1] - o1;
    v[2] = e[2] + o2;
    v[6] = e[2] - o2;
    v[3] = e[3] + o3;
    v[7] = e[3] - o3;
  }
};

// Sixteen-point DFT as 4 x 4: with j = 4a + b and k = c + 4d,
//   y_{c+4d} = sum_b W4^{bd} W16^{bc} [sum_a x_{4a+b} W4^{ac}],  W16 = exp(SIGN 2 pi i/16):
// four radix-4 butterflies over a, the twiddles W16^{bc}, four radix-4 butterflies over b.
template <typename R, int SIGN>
struct Bfly<R, SIGN, 16> {
  __device__ __forceinline__ static void run(cplx<R>* v) {
    const R c1 = R(0.92387953251128675612818318939678829);   // cos(pi/8)
    const R s1 = R(0.38268343236508977172845998403039887);   // sin(pi/8)
    const R h = R(0.70710678118654752440084436210484904);
    const R S = R(SIGN);
    cplx<R> z[4][4];   // z[b][c]
#pragma unroll
    for (int b = 0; b < 4; ++b) {
      cplx<R> t[4] = {v[b], v[4 + b], v[8 + b], v[12 + b]};
      Bfly<R, SIGN, 4>::run(t);
#pragma unroll
      for (int c = 0; c < 4; ++c) z[b][c] = t[c];
    }
    // W16^m for m = b c in {1, 2, 3, 4, 6, 9}: (cos, SIGN sin) of 2 pi m/16
    const cplx<R> w1 = {c1, S * s1}, w2 = {h, S * h}, w3 = {s1, S * c1};
    z[1][1] = cmul(z[1][1], w1);
    z[1][2] = cmul(z[1][2], w2);
    z[1][3] = cmul(z[1][3], w3);
    z[2][1] = cmul(z[2][1], w2);
    z[2][2] = mul_si<R, SIGN>(z[2][2]);                       // W16^4 = SIGN i
    z[2][3] = cmul(z[2][3], cplx<R>{-h, S * h});              // W16^6
    z[3][1] = cmul(z[3][1], w3);
    z[3][2] = cmul(z[3][2], cplx<R>{-h, S * h});              // W16^6
    z[3][3] = cmul(z[3][3], cplx<R>{-c1, -S * s1});           // W16^9 = -W16^1
#pragma unroll
    for (int c = 0; c < 4; ++c) {
      cplx<R> t[4] = {z[0][c], z[1][c], z[2][c], z[3][c]};
      Bfly<R, SIGN, 4>::run(t);
#pragma unroll
      for (int d = 0; d < 4; ++d) v[c + 4 * d] = t[d];
    }
  }
};

// ---------------------------------------------------------------- LDS row layout
// FFT rows live in LDS with one padding slot after every 8 elements and one
// more per row: element i of row r sits at r*RS + i + i/8.  Strided Stockham
// accesses (stride 8 in the first stage, 8-element runs 64 apart in the
// second) and column-wise tile loads then fall on distinct banks.
template <int L>
struct Lay {
  static constexpr int RS = L + (L >> 3) + 1;   // padded row size in elements
  __device__ __forceinline__ static int at(int row, int i) { return row * RS + i + (i >> 3); }
};

// ---------------------------------------------------------------- Stockham stages
// nrows rows of length L in the padded layout; NT threads.  tw[m] = exp(-2 pi i m/L)
// in LDS; the inverse uses its conjugate.
template <typename R, int SIGN, int L, int NT, int S, int NS>
struct Stages {
  __device__ __forceinline__ static cplx<R>* run(cplx<R>* src, cplx<R>* dst, const cplx<R>* tw,
                                                 int nrows, int tid) {
    if constexpr (NS >= L) {
      return src;
    } else {
      constexpr int RAD = radix_at(L, S, wide_plan<R, L>());
      constexpr int LR = L / RAD;
      constexpr int TWSTEP = L / (NS * RAD);
      const int total = nrows * LR;
      for (int b = tid; b < total; b += NT) {
        const int row = b / LR;
        const int j = b - row * LR;
        const cplx<R>* in = src + row * Lay<L>::RS;
        cplx<R>* out = dst + row * Lay<L>::RS;
        const int k = j % NS;
        cplx<R> v[RAD];
#pragma unroll
        for (int q = 0; q < RAD; ++q) {
          const int i = j + q * LR;
          v[q] = in[i + (i >> 3)];
        }
        if constexpr (NS > 1) {
#pragma unroll
          for (int q = 1; q < RAD; ++q) {
            cplx<R> w = tw[q * k * TWSTEP];
            if constexpr (SIGN > 0) w.y = -w.y;
            v[q] = cmul(v[q], w);
          }
        }
        Bfly<R, SIGN, RAD>::run(v);
        const int base = (j / NS) * NS * RAD + k;
#pragma unroll
        for (int q = 0; q < RAD; ++q) {
          const int i = base + q * NS;
          out[i + (i >> 3)] = v[q];
        }
      }
      __syncthreads();
      return Stages<R, SIGN, L, NT, S + 1, NS * RAD>::run(dst, src, tw, nrows, tid);
    }
  }
};

// In-LDS FFT of nrows rows of length L (padded layout); returns the buffer that
// holds the result (a or b).  Callers __syncthreads() before (data and
// twiddles in place); the routine ends with a barrier.
template <typename R, int SIGN, int L, int NT>
__device__ __forceinline__ cplx<R>* lds_fft(cplx<R>* a, cplx<R>* b, const cplx<R>* tw, int nrows,
                                            int tid) {
  return Stages<R, SIGN, L, NT, 0, 1>::run(a, b, tw, nrows, tid);
}

// ---------------------------------------------------------------- in-place stages
// The same Stockham stages on one buffer: every thread first reads all the
// butterflies it owns into registers, the block synchronises, and then the
// outputs are written.  Half the LDS of the ping-pong form for two barriers
// per stage.  MAXE bounds the elements per thread (nrows * L <= MAXE * NTP,
// checked by the caller), so a thread owns at most ceil(MAXE / RAD) butterflies.
template <typename R, int SIGN, int L, int NTP, int MAXE, int S, int NS>
struct StagesInPlace {
  __device__ __forceinline__ static void run(cplx<R>* buf, const cplx<R>* tw, int nrows, int tid) {
    if constexpr (NS < L) {
      constexpr int RAD = radix_at(L, S, wide_plan<R, L>());
      constexpr int LR = L / RAD;
      constexpr int TWSTEP = L / (NS * RAD);
      constexpr int MAXB = (MAXE + RAD - 1) / RAD;
      const int total = nrows * LR;
      cplx<R> v[MAXB][RAD];
#pragma unroll
      for (int m = 0; m < MAXB; ++m) {
        const int b = tid + m * NTP;
        if (b < total) {
          const int row = b / LR, j = b - row * LR;
          const cplx<R>* in = buf + row * Lay<L>::RS;
#pragma unroll
          for (int q = 0; q < RAD; ++q) {
            const int i = j + q * LR;
            v[m][q] = in[i + (i >> 3)];
          }
        }
      }
      __syncthreads();
#pragma unroll
      for (int m = 0; m < MAXB; ++m) {
        const int b = tid + m * NTP;
        if (b < total) {
          const int row = b / LR, j = b - row * LR;
          const int k = j % NS;
          if constexpr (NS > 1) {
#pragma unroll
            for (int q = 1; q < RAD; ++q) {
              cplx<R> w = tw[q * k * TWSTEP];
              if constexpr (SIGN > 0) w.y = -w.y;
              v[m][q] = cmul(v[m][q], w);
            }
          }
          Bfly<R, SIGN, RAD>::run(v[m]);
          cplx<R>* out = buf + row * Lay<L>::RS;
          const int base = (j / NS) * NS * RAD + k;
#pragma unroll
          for (int q = 0; q < RAD; ++q) {
            const int i = base + q * NS;
            out[i + (i >> 3)] = v[m][q];
          }
        }
      }
      __syncthreads();
      StagesInPlace<R, SIGN, L, NTP, MAXE, S + 1, NS * RAD>::run(buf, tw, nrows, tid);
    }
  }
};

// In-place LDS FFT of nrows rows of length L (padded layout).  Callers
// __syncthreads() before; the routine ends with a barrier.
template <typename R, int SIGN, int L, int NTP, int MAXE>
__device__ __forceinline__ void lds_fft_inplace(cplx<R>* buf, const cplx<R>* tw, int nrows, int tid) {
  StagesInPlace<R, SIGN, L, NTP, MAXE, 0, 1>::run(buf, tw, nrows, tid);
}

}  // namespace ofdft
