// gfx950 kernels around the hot path, all FP64 reductions of small data:
//
//   k_psum     batch power spectrum over the stored alignment spectrum (snap)
//   k_moments  intensity moments of reconstructed fields (snap of beam
//              centre and waist)
//   k_tm_gram  Gram matrix of the batch transfer matrix (its eigenvalues are
//              the squared singular values)
//   k_tm_rows  row statistics of the matrix the diagonal metrics are taken on
//   k_tm_diag  the Gram matrix's diagonal (IL is its trace over n)
//   k_summ, k_isum  batch summary: the sums of each plane's parameters, and
//              the intensity summed over the batch
//   k_heig     eigenvalues of the Gram matrix (FP64 Householder reduction to
//              a tridiagonal, then bisection; one workgroup): the squared
//              singular values for MDL
//   k_q16      fields to int16 real and imaginary parts with one scale each
//   k_basis    HG coefficients to another basis (LG, custom): one matrix product
//   k_m0y, k_m0x  IFFT mode 0 field export: the window zero-padded to the FFT
//              grid and inverse transformed along y, then x (LDS FFTs)
//   k_fptr, k_avg_rot, k_comb_*   wavelength sweeps and frame averaging: the
//              frame of each staged position, the phase of each repetition,
//              and the outputs combined from the staged results
#include "dh_fft.hpp"
#include "dh_internal.hpp"

namespace dh {

// k_psum: pw[p][j][i] = sum over frames of |spec[b][p][j][i]|^2
__global__ void k_psum(const float2* __restrict__ spec, int nb, int npol, size_t plane, float* __restrict__ pw) {
  const size_t e = (size_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (e >= npol * plane) return;
  const int p = (int)(e / plane);
  const size_t k = e - (size_t)p * plane;
  float s = 0.f;
  for (int b = 0; b < nb; ++b) {
    const float2 v = spec[((size_t)b * npol + p) * plane + k];
    s = fmaf(v.x, v.x, fmaf(v.y, v.y, s));
  }
  pw[e] = s;
}

// k_moments: grid (nb * npol); block e reduces field e ([wy][wx]) to the FP64
// sums of I, x I, y I, x^2 I, y^2 I, I = |E|^2, on the coarse grid
// x = (k - wx/2) px, y = (l - wy/2) py, in a fixed order.
__global__ void __launch_bounds__(256) k_moments(const float2* __restrict__ f, int wx, int wy, double px, double py,
                                                 double* __restrict__ out) {
  __shared__ double red[5][256];
  const int tid = threadIdx.x;
  const float2* e = f + (size_t)blockIdx.x * wx * wy;
  double s[5] = {0.0, 0.0, 0.0, 0.0, 0.0};
  for (int t = tid; t < wx * wy; t += 256) {
    const int l = t / wx, k = t - l * wx;
    const float2 v = e[t];
    const double i = (double)v.x * v.x + (double)v.y * v.y;
    const double x = (k - 0.5 * wx) * px, y = (l - 0.5 * wy) * py;
    s[0] += i;
    s[1] += x * i;
    s[2] += y * i;
    s[3] += x * x * i;
    s[4] += y * y * i;
  }
#pragma unroll
  for (int q = 0; q < 5; ++q) red[q][tid] = s[q];
  __syncthreads();
  for (int w = 128; w > 0; w >>= 1) {
    if (tid < w)
#pragma unroll
      for (int q = 0; q < 5; ++q) red[q][tid] += red[q][tid + w];
    __syncthreads();
  }
  if (tid < 5) out[(size_t)blockIdx.x * 5 + tid] = red[tid][0];
}

// ---------------------------------------------------------------------------
// Transfer-matrix metrics, FP64. A is rows x cols with cols = P M:
// combined, row b = frame b and A(b, p M + m) = c[b][p][m]; independent, row
// p B + b holds c[b][p][m] in pol p's columns and zero in the others.
__device__ __forceinline__ double2 tm_a(const TmArgs& t, int r, int col) {
  int b = r;
  if (t.indep) {
    const int p = r / t.B;
    b = r - p * t.B;
    if (col / t.M != p) return make_double2(0.0, 0.0);
  }
  const float2 v = t.c[(size_t)b * t.P * t.M + col];
  return make_double2((double)v.x, (double)v.y);
}

// G = X X^H, n x n, column-major: X = A (by rows, K = cols) or X = A^H
// (K = rows). One wave per element, four per block: lane l takes
// k = l, l + 64, ..., and the partial sums meet in a fixed butterfly, so an
// element does not depend on the launch.
__global__ void __launch_bounds__(256) k_tm_gram(TmArgs t, int by_rows, int n, double2* __restrict__ g) {
  const int lane = threadIdx.x & 63;
  const long e = (long)blockIdx.x * 4 + (threadIdx.x >> 6);
  if (e >= (long)n * n) return;                 // the whole wave
  const int i = (int)(e % n), j = (int)(e / n);
  const int K = by_rows ? t.cols : t.rows;
  double re = 0.0, im = 0.0;
  for (int k = lane; k < K; k += 64) {
    // X(i,k) conj(X(j,k)); X = A^H: X(i,k) = conj(A(k,i))
    const double2 x = by_rows ? tm_a(t, i, k) : tm_a(t, k, i);
    const double2 y = by_rows ? tm_a(t, j, k) : tm_a(t, k, j);
    const double xr = x.x, xi = by_rows ? x.y : -x.y;
    const double yr = y.x, yi = by_rows ? y.y : -y.y;
    re += xr * yr + xi * yi;
    im += xi * yr - xr * yi;
  }
#pragma unroll
  for (int off = 32; off > 0; off >>= 1) {
    re += __shfl_xor(re, off, 64);
    im += __shfl_xor(im, off, 64);
  }
  if (lane == 0) g[(size_t)i + (size_t)j * n] = make_double2(re, im);
}

// mode key of transfer-matrix index k: (pol, mode group); past the modes, unique
__device__ __forceinline__ long tm_key(const TmArgs& t, int k) {
  if (k >= t.P * t.M) return -1 - (long)k;
  const int p = k / t.M;
  if (t.grp) return (long)p * t.ngrp + t.grp[k - p * t.M];
  const short2 mn = t.modes[k - p * t.M];
  return (long)p * 256 + mn.x + mn.y;      // groups m + n < 100
}

// Per row i of D (D = A, or the Gram A A^H in g, rows x rows): the row's
// power sum_j |D_ij|^2, and for i < nd its diagonal |D_ii|^2 and the power in
// the columns whose mode shares row i's mode key.
__global__ void __launch_bounds__(256) k_tm_rows(TmArgs t, const double2* __restrict__ g, int nrow, int ncol,
                                                 int nd, double* __restrict__ rowpow, double* __restrict__ diag,
                                                 double* __restrict__ same) {
  // one wave per row, four per block: lane l takes the columns l, l + 64, ...,
  // and the partial sums meet in a fixed butterfly
  const int lane = threadIdx.x & 63;
  const int i = blockIdx.x * 4 + (threadIdx.x >> 6);
  if (i >= nrow) return;                        // the whole wave
  const long ki = tm_key(t, i);
  double tot = 0.0, sg = 0.0, dg = 0.0;
  for (int j = lane; j < ncol; j += 64) {
    const double2 v = g ? g[(size_t)i + (size_t)j * nrow] : tm_a(t, i, j);
    const double pw = v.x * v.x + v.y * v.y;
    tot += pw;
    if (i < nd) {
      if (j == i) dg = pw;
      if (tm_key(t, j) == ki) sg += pw;
    }
  }
#pragma unroll
  for (int off = 32; off > 0; off >>= 1) {
    tot += __shfl_xor(tot, off, 64);
    sg += __shfl_xor(sg, off, 64);
    dg += __shfl_xor(dg, off, 64);
  }
  if (lane == 0) {
    rowpow[i] = tot;
    if (i < nd) {
      diag[i] = dg;
      same[i] = sg;
    }
  }
}

hipError_t launch_tm_gram(const TmArgs& t, int by_rows, int n, double2* g, hipStream_t s) {
  if (n < 1) return hipSuccess;
  const long blocks = ((long)n * n + 3) / 4;
  if (blocks > 0x7fffffffL) return hipErrorInvalidValue;
  hipLaunchKernelGGL(k_tm_gram, dim3((unsigned)blocks), dim3(256), 0, s, t, by_rows, n, g);
  return hipGetLastError();
}

hipError_t launch_tm_rows(const TmArgs& t, const double2* g, int nrow, int ncol, int nd, double* rowpow, double* diag,
                          double* same, hipStream_t s) {
  if (nrow < 1) return hipSuccess;
  hipLaunchKernelGGL(k_tm_rows, dim3((nrow + 3) / 4), dim3(256), 0, s, t, g, nrow, ncol, nd, rowpow, diag, same);
  return hipGetLastError();
}

// the real diagonal of an n x n complex matrix (its trace's terms)
__global__ void k_tm_diag(const double2* __restrict__ g, int n, double* __restrict__ out) {
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i < n) out[i] = g[(size_t)i * (n + 1)].x;
}

hipError_t launch_tm_diag(const double2* g, int n, double* out, hipStream_t s) {
  if (n < 1) return hipSuccess;
  hipLaunchKernelGGL(k_tm_diag, dim3((n + 255) / 256), dim3(256), 0, s, g, n, out);
  return hipGetLastError();
}

// ---------------------------------------------------------------------------
// k_heig: every eigenvalue of an n x n Hermitian matrix (FP64 complex,
// column-major, overwritten), in one workgroup, in two textbook steps:
//  1. Householder reduction to a real symmetric tridiagonal matrix. The input
//     is first replaced by its Hermitian part (A + A^H) / 2, both triangles
//     stored. For column k, x = A(k+1.., k): a reflector H = I - tau u u^H
//     (u(0) = 1) with H^H x = beta e1, beta = -sign(Re x0) |x| real, then
//     A22 <- H^H A22 H on the trailing block as the rank-2 update
//     A22 - u w^H - w u^H, p = tau A22 u, w = p - (tau / 2)(p^H u) u.
//     The tridiagonal keeps d_k = A(k, k) and the off-diagonal beta_k (real:
//     a Hermitian tridiagonal with off-diagonal e_k has the same eigenvalues
//     as the real one with |e_k|).
//  2. Bisection with Sturm counts: the number of eigenvalues below x is the
//     number of negative q_i in q_0 = d_0 - x, q_i = d_i - x - e_{i-1}^2 /
//     q_{i-1}; thread t narrows the Gershgorin interval to eigenvalue t until
//     it is a few ulps wide, so w comes out in ascending order.
// The reduction is backward stable in FP64, so every eigenvalue is within a
// small multiple of n eps |A| of the exact one. info = 0, or -1 when the
// tridiagonal is not finite (w is then NaN). Matrices up to kHeigLds rows
// are worked on in LDS, larger ones (up to kHeigMaxN) in place in global
// memory.
constexpr int kHeigLds = 96;
constexpr int kHeigMaxN = 2048;
constexpr int kHeigThreads = 1024;
constexpr int kHeigParts = 4;        // column ranges of the in-LDS matrix-vector product

__device__ __forceinline__ double2 zmul(double2 a, double2 b) {
  return make_double2(a.x * b.x - a.y * b.y, a.x * b.y + a.y * b.x);
}
__device__ __forceinline__ double2 zcmul(double2 a, double2 b) {     // conj(a) b
  return make_double2(a.x * b.x + a.y * b.y, a.x * b.y - a.y * b.x);
}

// sum over the workgroup of (x, y); every thread gets it. buf: 2 NW doubles,
// alternated between calls by the caller so that one barrier suffices
template <int NW>
__device__ __forceinline__ double2 heig_sum(double2 v, double* buf, int tid) {
  for (int off = 32; off > 0; off >>= 1) {
    v.x += __shfl_xor(v.x, off, 64);
    v.y += __shfl_xor(v.y, off, 64);
  }
  if ((tid & 63) == 0) {
    buf[2 * (tid >> 6)] = v.x;
    buf[2 * (tid >> 6) + 1] = v.y;
  }
  __syncthreads();
  double2 r = make_double2(0.0, 0.0);
  for (int k = 0; k < NW; ++k) {
    r.x += buf[2 * k];
    r.y += buf[2 * k + 1];
  }
  return r;
}

template <bool IN_LDS>
__global__ void __launch_bounds__(kHeigThreads) k_heig(double2* __restrict__ g, int n, double* __restrict__ w,
                                                       int* __restrict__ info) {
  constexpr int NV = IN_LDS ? kHeigLds : kHeigMaxN;
  constexpr int NW = kHeigThreads / 64;
  __shared__ double2 lds[IN_LDS ? kHeigLds * kHeigLds : 1];
  // u of this step and (in LDS) of the next. The in-global form keeps one:
  // its larger LDS allocation measured 45-55 % slower at n = 97 .. 250
  __shared__ double2 s_u[IN_LDS ? 2 : 1][NV], s_w[NV];
  __shared__ double s_d[NV], s_e2[NV];
  __shared__ double s_red[2][2 * NW];
  __shared__ double s_mm[4][NW];
  __shared__ double2 s_part[IN_LDS ? kHeigParts : 1][IN_LDS ? kHeigLds : 1];  // matrix-vector product, by column range
  __shared__ double s_nrm;
  __shared__ double2 s_ref;                        // the next step's tau, when s_rdy
  __shared__ double s_beta;
  __shared__ int s_rdy;
  const int tid = threadIdx.x, lane = tid & 63, wv = tid >> 6;
  double2* a = IN_LDS ? lds : g;
  // the Hermitian part, both triangles (each pair read and written by one thread)
  for (int e = tid; e < n * n; e += kHeigThreads) {
    const int i = e % n, j = e / n;
    if (i < j) continue;
    const double2 x = g[i + (size_t)j * n], y = g[j + (size_t)i * n];
    const double2 h = make_double2(0.5 * (x.x + y.x), 0.5 * (x.y - y.y));
    if (i == j) {
      a[i + (size_t)j * n] = make_double2(h.x, 0.0);
    } else {
      a[i + (size_t)j * n] = h;
      a[j + (size_t)i * n] = make_double2(h.x, -h.y);
    }
  }
  __syncthreads();
  int rb = 0;                                    // s_red half for the next sum
  // squared norm of the first column's part below the subdiagonal; later
  // steps get it from the wave that updates that column
  double ss_next;
  {
    double2 part = make_double2(0.0, 0.0);
    for (int i = 2 + tid; i < n; i += kHeigThreads) part.x += a[i].x * a[i].x + a[i].y * a[i].y;
    ss_next = heig_sum<NW>(part, s_red[rb], tid).x;
    rb ^= 1;
  }
  // In LDS the wave that updates column 0 of the trailing block also forms
  // the next step's reflector (its u in the other half of s_u, beta and tau in
  // s_beta, s_ref); `ready` (uniform) says this step's reflector is there.
  bool ready = false;
  int ub = 0;                                    // s_u half of this step
  for (int k = 0; k + 2 < n; ++k) {
    const int k1 = k + 1, m = n - k1;
    const double2* col = a + k1 + (size_t)k * n;   // x = A(k1 .., k), m entries
    double beta;
    double2 tau;
    bool ident = false;
    if (ready) {
      beta = s_beta;
      tau = s_ref;
    } else {
      // every thread forms the same reflector from the same values
      const double ss = ss_next;
      const double2 x0 = col[0];
      ident = ss == 0.0 && x0.y == 0.0;
      const double nrm = sqrt(x0.x * x0.x + x0.y * x0.y + ss);
      beta = ident ? x0.x : (x0.x >= 0.0 ? -nrm : nrm);
      tau = make_double2((beta - x0.x) / beta, -x0.y / beta);
    }
    if (tid == 0) {
      s_d[k] = a[k + (size_t)k * n].x;
      s_e2[k] = beta * beta;
    }
    if (ident) {                                  // H = I (uniform across the workgroup)
      double2 part = make_double2(0.0, 0.0);
      const double2* nx = a + k1 + (size_t)k1 * n;  // the next column, unchanged
      for (int i = 2 + tid; i < m; i += kHeigThreads) part.x += nx[i].x * nx[i].x + nx[i].y * nx[i].y;
      ss_next = heig_sum<NW>(part, s_red[rb], tid).x;
      rb ^= 1;
      continue;
    }
    double2* su = s_u[IN_LDS ? ub : 0];
    if (!ready) {
      // u = x / (x0 - beta), u(0) = 1
      const double2 x0 = col[0];
      const double2 den = make_double2(x0.x - beta, x0.y);
      const double dd = den.x * den.x + den.y * den.y;
      const double2 sc = make_double2(den.x / dd, -den.y / dd);
      for (int i = tid; i < m; i += kHeigThreads) su[i] = i == 0 ? make_double2(1.0, 0.0) : zmul(col[i], sc);
      __syncthreads();
    }
    // p = tau A22 u (into s_w) and the partial sums of p^H u. Rows across the
    // lanes of a wave (consecutive rows of each column: both triangles are
    // stored); in LDS the columns are split into kHeigParts ranges summed by
    // separate threads, then added in range order.
    double2 kp = make_double2(0.0, 0.0);
    if constexpr (IN_LDS) {
      const int i = tid & 127, part = tid >> 7;
      const int q = (m + kHeigParts - 1) / kHeigParts, j0 = part * q, j1 = j0 + q < m ? j0 + q : m;
      if (part < kHeigParts && i < m) {
        const double2* ri = a + k1 + i + (size_t)k1 * n;
        double2 acc = make_double2(0.0, 0.0), acc2 = make_double2(0.0, 0.0);
        int j = j0;
        for (; j + 4 <= j1; j += 4) {
#pragma unroll
          for (int t = 0; t < 4; t += 2) {
            const double2 x = zmul(ri[(size_t)(j + t) * n], su[j + t]);
            const double2 x2 = zmul(ri[(size_t)(j + t + 1) * n], su[j + t + 1]);
            acc.x += x.x;
            acc.y += x.y;
            acc2.x += x2.x;
            acc2.y += x2.y;
          }
        }
        for (; j < j1; ++j) {
          const double2 x = zmul(ri[(size_t)j * n], su[j]);
          acc.x += x.x;
          acc.y += x.y;
        }
        s_part[part][i] = make_double2(acc.x + acc2.x, acc.y + acc2.y);
      }
      __syncthreads();
      if (tid < m) {
        double2 pr = s_part[0][tid];
#pragma unroll
        for (int q2 = 1; q2 < kHeigParts; ++q2) pr = make_double2(pr.x + s_part[q2][tid].x, pr.y + s_part[q2][tid].y);
        const double2 pw = zmul(tau, pr);
        s_w[tid] = pw;
        kp = zcmul(pw, su[tid]);
      }
    } else {
      for (int i = tid; i < m; i += kHeigThreads) {
        const double2* ri = a + k1 + i + (size_t)k1 * n;
        // (unrolled so that several loads are in flight; two partial sums)
        double2 acc = make_double2(0.0, 0.0), acc2 = make_double2(0.0, 0.0);
        int j = 0;
        for (; j + 8 <= m; j += 8) {
#pragma unroll
          for (int q = 0; q < 8; q += 2) {
            const double2 t = zmul(ri[(size_t)(j + q) * n], su[j + q]);
            const double2 t2 = zmul(ri[(size_t)(j + q + 1) * n], su[j + q + 1]);
            acc.x += t.x;
            acc.y += t.y;
            acc2.x += t2.x;
            acc2.y += t2.y;
          }
        }
        for (; j < m; ++j) {
          const double2 t = zmul(ri[(size_t)j * n], su[j]);
          acc.x += t.x;
          acc.y += t.y;
        }
        const double2 pw = zmul(tau, make_double2(acc.x + acc2.x, acc.y + acc2.y));
        s_w[i] = pw;
        const double2 t = zcmul(pw, su[i]);
        kp.x += t.x;
        kp.y += t.y;
      }
    }
    // w = p - (tau / 2) (p^H u) u, formed where it is used
    const double2 K = heig_sum<NW>(kp, s_red[rb], tid);
    rb ^= 1;
    const double2 al = zmul(make_double2(-0.5 * tau.x, -0.5 * tau.y), K);
    // A22 <- A22 - u w^H - w u^H, column by column, rows across the lanes; the
    // wave of column 0 also sums the squared moduli of its new entries below
    // row 1, the next step's norm
    double nx2 = 0.0;
    if constexpr (IN_LDS) {
      // each lane's u_i and w_i (at most two rows) held in registers across the columns
      constexpr int RI = (kHeigLds + 63) / 64;
      double2 ur[RI], wr[RI];
#pragma unroll
      for (int r = 0; r < RI; ++r) {
        const int i = lane + 64 * r;
        ur[r] = i < m ? su[i] : make_double2(0.0, 0.0);
        const double2 t = zmul(al, ur[r]);
        wr[r] = i < m ? make_double2(s_w[i].x + t.x, s_w[i].y + t.y) : make_double2(0.0, 0.0);
      }
      if (wv == 0) {
        // column 0 first, then the next step's reflector from its rows 1 ..
        // (x0 = row 1, norm over rows 2 ..), with the same formulas as above
        const double2 cw = make_double2(wr[0].x, -wr[0].y);   // w_0 and u_0 = 1 sit in lane 0
        const double2 w0 = make_double2(__shfl(cw.x, 0, 64), __shfl(cw.y, 0, 64));
        const double2 cu = make_double2(1.0, 0.0);
        double2 nv[RI];
#pragma unroll
        for (int r = 0; r < RI; ++r) {
          const int i = lane + 64 * r;
          nv[r] = make_double2(0.0, 0.0);
          if (i < m) {
            double2* c0 = a + k1 + (size_t)k1 * n;
            const double2 t1 = zmul(ur[r], w0), t2 = zmul(wr[r], cu);
            nv[r] = make_double2(c0[i].x - t1.x - t2.x, c0[i].y - t1.y - t2.y);
            c0[i] = nv[r];
            if (i >= 2) nx2 += nv[r].x * nv[r].x + nv[r].y * nv[r].y;
          }
        }
        for (int off = 32; off > 0; off >>= 1) nx2 += __shfl_xor(nx2, off, 64);
        const double2 x0n = make_double2(__shfl(nv[0].x, 1, 64), __shfl(nv[0].y, 1, 64));
        const bool next = k + 3 < n && !(nx2 == 0.0 && x0n.y == 0.0);
        if (next) {
          const double nrm = sqrt(x0n.x * x0n.x + x0n.y * x0n.y + nx2);
          const double bn = x0n.x >= 0.0 ? -nrm : nrm;
          const double2 den = make_double2(x0n.x - bn, x0n.y);
          const double dd = den.x * den.x + den.y * den.y;
          const double2 sc = make_double2(den.x / dd, -den.y / dd);
          double2* un = s_u[IN_LDS ? ub ^ 1 : 0];
#pragma unroll
          for (int r = 0; r < RI; ++r) {
            const int i = lane + 64 * r;
            if (i >= 1 && i < m) un[i - 1] = i == 1 ? make_double2(1.0, 0.0) : zmul(nv[r], sc);
          }
          if (lane == 0) {
            s_beta = bn;
            s_ref = make_double2((bn - x0n.x) / bn, -x0n.y / bn);
          }
        }
        if (lane == 0) {
          s_nrm = nx2;
          s_rdy = next;
        }
      }
#pragma unroll 2
      for (int j = wv == 0 ? NW : wv; j < m; j += NW) {
        const double2 uj = su[j], tj = zmul(al, uj);
        const double2 cw = make_double2(s_w[j].x + tj.x, -(s_w[j].y + tj.y)), cu = make_double2(uj.x, -uj.y);
        double2* cj = a + k1 + (size_t)(k1 + j) * n;
#pragma unroll
        for (int r = 0; r < RI; ++r) {
          const int i = lane + 64 * r;
          if (i < m) {
            const double2 t1 = zmul(ur[r], cw), t2 = zmul(wr[r], cu);
            cj[i] = make_double2(cj[i].x - t1.x - t2.x, cj[i].y - t1.y - t2.y);
          }
        }
      }
    } else {
      for (int j = wv; j < m; j += NW) {
        const double2 uj = su[j], tj = zmul(al, uj);
        const double2 cw = make_double2(s_w[j].x + tj.x, -(s_w[j].y + tj.y)), cu = make_double2(uj.x, -uj.y);
        double2* cj = a + k1 + (size_t)(k1 + j) * n;
        for (int i = lane; i < m; i += 64) {
          const double2 ui = su[i], ti = zmul(al, ui);
          const double2 wi = make_double2(s_w[i].x + ti.x, s_w[i].y + ti.y);
          const double2 t1 = zmul(ui, cw), t2 = zmul(wi, cu);
          const double2 nv = make_double2(cj[i].x - t1.x - t2.x, cj[i].y - t1.y - t2.y);
          cj[i] = nv;
          if (j == 0 && i >= 2) nx2 += nv.x * nv.x + nv.y * nv.y;
        }
      }
      if (wv == 0) {
        for (int off = 32; off > 0; off >>= 1) nx2 += __shfl_xor(nx2, off, 64);
        if (lane == 0) {
          s_nrm = nx2;
          s_rdy = 0;
        }
      }
    }
    __syncthreads();
    ss_next = s_nrm;
    ready = s_rdy != 0;
    if (ready) ub ^= 1;
  }
  if (tid == 0) {
    if (n >= 2) {
      const double2 l = a[(n - 1) + (size_t)(n - 2) * n];
      s_d[n - 2] = a[(n - 2) + (size_t)(n - 2) * n].x;
      s_e2[n - 2] = l.x * l.x + l.y * l.y;
    }
    s_d[n - 1] = a[(n - 1) + (size_t)(n - 1) * n].x;
  }
  __syncthreads();
  // Gershgorin interval of the tridiagonal: each thread its rows, then the
  // workgroup's extremes (every thread gets them)
  // (fmin and fmax pass over NaN, so entries that are not finite are flagged
  // on their own)
  double lo = HUGE_VAL, hi = -HUGE_VAL, emax = 0.0, bad = 0.0;
  for (int i = tid; i < n; i += kHeigThreads) {
    const double el = i > 0 ? sqrt(s_e2[i - 1]) : 0.0, er = i + 1 < n ? sqrt(s_e2[i]) : 0.0;
    lo = fmin(lo, s_d[i] - el - er);
    hi = fmax(hi, s_d[i] + el + er);
    if (i + 1 < n) emax = fmax(emax, s_e2[i]);
    const double e2 = i + 1 < n ? s_e2[i] : 0.0;
    if (!(s_d[i] - s_d[i] == 0.0) || !(e2 - e2 == 0.0)) bad = 1.0;
  }
  for (int off = 32; off > 0; off >>= 1) {
    lo = fmin(lo, __shfl_xor(lo, off, 64));
    hi = fmax(hi, __shfl_xor(hi, off, 64));
    emax = fmax(emax, __shfl_xor(emax, off, 64));
    bad = fmax(bad, __shfl_xor(bad, off, 64));
  }
  if (lane == 0) {
    s_mm[0][wv] = lo;
    s_mm[1][wv] = hi;
    s_mm[2][wv] = emax;
    s_mm[3][wv] = bad;
  }
  __syncthreads();
  for (int k = 0; k < NW; ++k) {
    lo = fmin(lo, s_mm[0][k]);
    hi = fmax(hi, s_mm[1][k]);
    emax = fmax(emax, s_mm[2][k]);
    bad = fmax(bad, s_mm[3][k]);
  }
  const bool finite = bad == 0.0 && lo - lo == 0.0 && hi - hi == 0.0;
  // a pivot never smaller than this (keeps the Sturm recurrence finite)
  const double pivmin = 2.2250738585072014e-308 * fmax(1.0, emax);
  const double span = fmax(fabs(lo), fabs(hi));
  lo -= 2.2e-16 * span + pivmin;
  hi += 2.2e-16 * span + pivmin;
  // K adjacent lanes per eigenvalue (a power of two up to 8, as the
  // workgroup allows): each step they count at the K interior points that
  // cut the interval into K + 1 equal parts, and the interval becomes the
  // part where the count first exceeds the eigenvalue's index
  const int K = n * 8 <= kHeigThreads ? 8 : n * 4 <= kHeigThreads ? 4 : n * 2 <= kHeigThreads ? 2 : 1;
  const int per = kHeigThreads / K, sub = tid % K, g0 = lane & ~(K - 1);
  for (int b0 = 0; b0 < n; b0 += per) {
    const int t = b0 + tid / K;                   // this group's eigenvalue
    double x0 = lo, x1 = hi;
    for (int it = 0; it < 128; ++it) {
      const bool live = t < n && finite && x1 - x0 > 4.5e-16 * fmax(fabs(x0), fabs(x1)) + 2.0 * pivmin;
      if (__ballot(live) == 0) break;             // the wave's groups are all done
      const double h = (x1 - x0) / (K + 1);
      const double xs = x0 + h * (sub + 1);
      int cnt = 0;
      double q = s_d[0] - xs;
      if (fabs(q) < pivmin) q = -pivmin;
      cnt += q < 0.0;
#pragma unroll 4
      for (int i = 1; i < n; ++i) {
        // 1 / q: the hardware estimate refined by two Newton steps
        double r = __builtin_amdgcn_rcp(q);
        r = fma(r, fma(-q, r, 1.0), r);
        r = fma(r, fma(-q, r, 1.0), r);
        q = (s_d[i] - xs) - s_e2[i - 1] * r;
        if (fabs(q) < pivmin) q = -pivmin;
        cnt += q < 0.0;
      }
      const unsigned long long gb = (__ballot(cnt > t) >> g0) & ((1ull << K) - 1);
      const int s1 = gb ? __builtin_ctzll(gb) : K;  // first point past the eigenvalue
      if (live) {                                   // every lane of the group alike
        const double nx0 = s1 > 0 ? x0 + h * s1 : x0;
        const double nx1 = s1 < K ? x0 + h * (s1 + 1) : x1;
        x0 = nx0;
        x1 = nx1;
      }
    }
    if (t < n && sub == 0) w[t] = finite ? 0.5 * (x0 + x1) : NAN;
  }
  if (tid == 0) *info = finite ? 0 : -1;
}

hipError_t launch_heig(double2* g, int n, double* w, int* info, hipStream_t s) {
  if (n < 1) return hipSuccess;
  if (n > kHeigMaxN) return hipErrorInvalidValue;
  if (n <= kHeigLds)
    hipLaunchKernelGGL(k_heig<true>, dim3(1), dim3(kHeigThreads), 0, s, g, n, w, info);
  else
    hipLaunchKernelGGL(k_heig<false>, dim3(1), dim3(kHeigThreads), 0, s, g, n, w, info);
  return hipGetLastError();
}

// ---------------------------------------------------------------------------
// Batch summary ("Analysis parameter types"). A plane is H x W values, value
// (l, k) (row l of the y axis, column k of the x axis) at base + l sy + k sx;
// the intensity is |z|^2 of a complex64 value, taken in FP64 from its FP32
// parts, or an FP64 intensity map. Sums run over the plane in memory order.
struct SumPlane {
  const float2* z;         // complex planes (or null)
  const double* map;       // FP64 intensity planes (or null)
  long long pstride;       // elements between consecutive planes
  int w, h, sx, sy;        // sx == 1: rows contiguous; else columns contiguous (sy == 1)
};

__device__ __forceinline__ double plane_at(const SumPlane& P, long long base, int l, int k) {
  const long long a = base + (long long)l * P.sy + (long long)k * P.sx;
  if (P.map) return P.map[a];
  const float2 v = P.z[a];
  return (double)v.x * v.x + (double)v.y * v.y;
}

// k_summ: grid (n planes), 256 threads. out[e][8] = sum I, sum k I, sum l I,
// sum I^2, sum cos(2 pi l / H) I, sum sin(2 pi l / H) I, max I, its index
// l W + k (the lowest index on ties). Fixed order: per thread a fixed stride,
// then a fixed tree.
__global__ void __launch_bounds__(256) k_summ(SumPlane P, double* __restrict__ out) {
  __shared__ double red[6][256];
  __shared__ double rmax[256];
  __shared__ int ridx[256];
  const int tid = threadIdx.x;
  const long long base = (long long)blockIdx.x * P.pstride;
  const int n = P.w * P.h;
  double s[6] = {0.0, 0.0, 0.0, 0.0, 0.0, 0.0};
  double best = -1.0;
  int bidx = 0x7fffffff;
  for (int e = tid; e < n; e += 256) {
    int l, k;
    if (P.sx == 1) {
      l = e / P.w;
      k = e - l * P.w;
    } else {
      k = e / P.h;
      l = e - k * P.h;
    }
    const double v = plane_at(P, base, l, k);
    double sn, cs;
    sincospi(2.0 * l / P.h, &sn, &cs);
    s[0] += v;
    s[1] += k * v;
    s[2] += l * v;
    s[3] += v * v;
    s[4] += cs * v;
    s[5] += sn * v;
    const int idx = l * P.w + k;
    if (v > best || (v == best && idx < bidx)) {
      best = v;
      bidx = idx;
    }
  }
#pragma unroll
  for (int q = 0; q < 6; ++q) red[q][tid] = s[q];
  rmax[tid] = best;
  ridx[tid] = bidx;
  __syncthreads();
  for (int w = 128; w > 0; w >>= 1) {
    if (tid < w) {
#pragma unroll
      for (int q = 0; q < 6; ++q) red[q][tid] += red[q][tid + w];
      const double o = rmax[tid + w];
      const int oi = ridx[tid + w];
      if (o > rmax[tid] || (o == rmax[tid] && oi < ridx[tid])) {
        rmax[tid] = o;
        ridx[tid] = oi;
      }
    }
    __syncthreads();
  }
  if (tid == 0) {
    double* o = out + (size_t)blockIdx.x * 8;
#pragma unroll
    for (int q = 0; q < 6; ++q) o[q] = red[q][0];
    o[6] = rmax[0] > 0.0 ? rmax[0] : 0.0;
    o[7] = rmax[0] > 0.0 ? (double)ridx[0] : 0.0;
  }
}

// k_isum: map[p][l][k] (+)= sum over the nb planes of pol p (plane b npol + p)
// of their intensity, frames in order (row-major map, one thread per pixel)
__global__ void k_isum(SumPlane P, int nb, int npol, int accumulate, double* __restrict__ map) {
  const long long e = (long long)blockIdx.x * blockDim.x + threadIdx.x;
  const long long n = (long long)P.w * P.h;
  if (e >= n * npol) return;
  const int p = (int)(e / n);
  const int r = (int)(e - (long long)p * n);
  int l, k;
  if (P.sx == 1) {
    l = r / P.w;
    k = r - l * P.w;
  } else {
    k = r / P.h;
    l = r - k * P.h;
  }
  double acc = accumulate ? map[(size_t)p * n + (size_t)l * P.w + k] : 0.0;
  for (int b = 0; b < nb; ++b) acc += plane_at(P, (long long)(b * npol + p) * P.pstride, l, k);
  map[(size_t)p * n + (size_t)l * P.w + k] = acc;
}

hipError_t launch_summ(const float2* z, const double* map, long long pstride, int w, int h, int sx, int sy, int n,
                       double* out, hipStream_t s) {
  if (n < 1) return hipSuccess;
  SumPlane P{z, map, pstride, w, h, sx, sy};
  hipLaunchKernelGGL(k_summ, dim3(n), dim3(256), 0, s, P, out);
  return hipGetLastError();
}

hipError_t launch_isum(const float2* z, long long pstride, int w, int h, int sx, int sy, int nb, int npol,
                       int accumulate, double* map, hipStream_t s) {
  const long long n = (long long)w * h * npol;
  if (n < 1 || nb < 1) return hipSuccess;
  SumPlane P{z, nullptr, pstride, w, h, sx, sy};
  hipLaunchKernelGGL(k_isum, dim3((unsigned)((n + 255) / 256)), dim3(256), 0, s, P, nb, npol, accumulate, map);
  return hipGetLastError();
}

hipError_t launch_psum(const float2* spec, int nb, int npol, size_t plane, float* pw, hipStream_t s) {
  const size_t n = (size_t)npol * plane;
  hipLaunchKernelGGL(k_psum, dim3((unsigned)((n + 255) / 256)), dim3(256), 0, s, spec, nb, npol, plane, pw);
  return hipGetLastError();
}

hipError_t launch_moments(const float2* fields, int n, int wx, int wy, double px, double py, double* out,
                          hipStream_t s) {
  if (n < 1) return hipSuccess;
  hipLaunchKernelGGL(k_moments, dim3(n), dim3(256), 0, s, fields, wx, wy, px, py, out);
  return hipGetLastError();
}

// k_q16: grid (n fields), TPB threads; block e: scale = 32767 / max(|Re|,
// |Im|) over field e (1 if it is all zero), correctly rounded, then each part
// times the scale rounded to the nearest integer, ties to even (all in FP32).
// NV > 0: the field (len <= NV TPB) is read once into registers; NV = 0: read
// twice (the second time mostly from L2).
template <int TPB, int NV>
__global__ void __launch_bounds__(TPB) k_q16(const float2* __restrict__ f, long long len, short* __restrict__ re,
                                             short* __restrict__ im, float* __restrict__ scale) {
  __shared__ float red[TPB];
  const int tid = threadIdx.x;
  const size_t base = (size_t)blockIdx.x * (size_t)len;
  float2 v[NV > 0 ? NV : 1];
  float m = 0.f;
  if constexpr (NV > 0) {
#pragma unroll
    for (int k = 0; k < NV; ++k) {
      const long long t = tid + (long long)k * TPB;
      v[k] = t < len ? f[base + t] : make_float2(0.f, 0.f);
      m = fmaxf(m, fmaxf(fabsf(v[k].x), fabsf(v[k].y)));
    }
  } else {
    for (long long t = tid; t < len; t += TPB) {
      const float2 x = f[base + t];
      m = fmaxf(m, fmaxf(fabsf(x.x), fabsf(x.y)));
    }
  }
  red[tid] = m;
  __syncthreads();
  for (int w = TPB / 2; w > 0; w >>= 1) {
    if (tid < w) red[tid] = fmaxf(red[tid], red[tid + w]);
    __syncthreads();
  }
  const float peak = red[0];
  const float s = peak > 0.f ? __fdiv_rn(32767.0f, peak) : 1.0f;
  if constexpr (NV > 0) {
#pragma unroll
    for (int k = 0; k < NV; ++k) {
      const long long t = tid + (long long)k * TPB;
      if (t < len) {
        re[base + t] = (short)rintf(v[k].x * s);
        im[base + t] = (short)rintf(v[k].y * s);
      }
    }
  } else {
    for (long long t = tid; t < len; t += TPB) {
      const float2 x = f[base + t];
      re[base + t] = (short)rintf(x.x * s);
      im[base + t] = (short)rintf(x.y * s);
    }
  }
  if (tid == 0) scale[blockIdx.x] = s;
}

hipError_t launch_q16(const float2* fields, int n, long long len, short* re, short* im, float* scale, hipStream_t s) {
  if (n < 1) return hipSuccess;
  if (len <= 8 * 1024)
    hipLaunchKernelGGL((k_q16<1024, 8>), dim3(n), dim3(1024), 0, s, fields, len, re, im, scale);
  else if (len <= 24 * 1024)
    hipLaunchKernelGGL((k_q16<1024, 24>), dim3(n), dim3(1024), 0, s, fields, len, re, im, scale);
  else
    hipLaunchKernelGGL((k_q16<1024, 0>), dim3(n), dim3(1024), 0, s, fields, len, re, im, scale);
  return hipGetLastError();
}

// k_basis: grid (n, 2); block (e, y) maps coefficient vector e (a frame and
// pol) of the raw (y = 0) or normalised (y = 1) HG coefficients to the basis:
// out[e][k] = sum_{i < cnt_k} tt[off_k + i stride_k] in[e][first_k + i],
// FP32, i in order, with (first, cnt, off, stride) = rng[k]: the HG modes an
// output mode takes (all of them for a dense transform, its own group for
// LG), entries laid out so that the threads of a block read consecutive ones.
constexpr int kBasisMaxIn = kMaxGroups * (kMaxGroups + 1) / 2;
__global__ void __launch_bounds__(256) k_basis(const float2* __restrict__ in, const float2* __restrict__ in_norm,
                                               int nin, int nused, const int4* __restrict__ rng,
                                               const float2* __restrict__ tt, int nout, float2* __restrict__ out,
                                               float2* __restrict__ out_norm) {
  __shared__ float2 c[kBasisMaxIn];
  const int e = blockIdx.x;
  const float2* src = (blockIdx.y ? in_norm : in) + (size_t)e * nin;
  float2* dst = (blockIdx.y ? out_norm : out) + (size_t)e * nout;
  for (int j = threadIdx.x; j < nused; j += 256) c[j] = src[j];
  __syncthreads();
  for (int k = threadIdx.x; k < nout; k += 256) {
    const int4 r = rng[k];
    float re = 0.f, im = 0.f;
    for (int i = 0; i < r.y; ++i) {
      const float2 t = tt[(size_t)r.z + (size_t)i * r.w];
      const float2 v = c[r.x + i];
      re = fmaf(t.x, v.x, fmaf(-t.y, v.y, re));
      im = fmaf(t.x, v.y, fmaf(t.y, v.x, im));
    }
    dst[k] = make_float2(re, im);
  }
}

hipError_t launch_basis(const float2* in, const float2* in_norm, int nin, int nused, const int4* rng,
                        const float2* tt, int nout, float2* out, float2* out_norm, int n, hipStream_t s) {
  if (n < 1) return hipSuccess;
  if (nused > kBasisMaxIn) return hipErrorInvalidValue;
  hipLaunchKernelGGL(k_basis, dim3(n, 2), dim3(256), 0, s, in, in_norm, nin, nused, rng, tt, nout, out, out_norm);
  return hipGetLastError();
}

// staged position of output o's repetition a
__device__ __forceinline__ size_t stage_of(const Comb& c, int o, int a) {
  int i, w;
  if (c.out_order == 0) {
    i = o / c.L;
    w = o - i * c.L;
  } else {
    w = o / c.I;
    i = o - w * c.I;
  }
  return ((size_t)w * c.I + i) * c.A + a;
}

__global__ void k_fptr(const char* base, unsigned long long fbytes, int n_out, int L, int I, int A, int avg_mode,
                       int in_order, const void** __restrict__ sptr) {
  const int s = blockIdx.x * blockDim.x + threadIdx.x;
  if (s >= n_out * A) return;
  const int a = s % A, r = s / A, i = r % I, w = r / I;
  const long long j0 = in_order == 0 ? (long long)i * L + w : (long long)w * I + i;
  long long j;
  if (avg_mode == 0)
    j = j0 * A + a;                              // sequential: AAABBB
  else if (avg_mode == 1)
    j = (long long)a * n_out + j0;               // interlaced: ABCABC
  else
    j = ((long long)i * A + a) * L + w;          // sequential sweeps: {A}{A}{B}{B}
  sptr[s] = base + (size_t)j * fbytes;
}

__global__ void __launch_bounds__(256) k_avg_rot(const float2* __restrict__ win, long long per, Comb c,
                                                 double2* __restrict__ rot) {
  __shared__ double rr[256], ri[256];
  const int o = blockIdx.x, a = blockIdx.y, tid = threadIdx.x;
  if (a == 0) {
    if (tid == 0) rot[(size_t)o * c.A] = make_double2(1.0, 0.0);
    return;
  }
  const float2* wa = win + stage_of(c, o, a) * per;
  const float2* w0 = win + stage_of(c, o, 0) * per;
  double re = 0.0, im = 0.0;
  for (long long e = tid; e < per; e += 256) {
    const float2 x = wa[e], y = w0[e];               // x conj(y)
    re += (double)x.x * y.x + (double)x.y * y.y;
    im += (double)x.y * y.x - (double)x.x * y.y;
  }
  rr[tid] = re;
  ri[tid] = im;
  __syncthreads();
  for (int w = 128; w > 0; w >>= 1) {
    if (tid < w) {
      rr[tid] += rr[tid + w];
      ri[tid] += ri[tid + w];
    }
    __syncthreads();
  }
  if (tid == 0) {
    const double m = sqrt(rr[0] * rr[0] + ri[0] * ri[0]);
    rot[(size_t)o * c.A + a] = m > 0.0 ? make_double2(rr[0] / m, -ri[0] / m) : make_double2(1.0, 0.0);
  }
}

__global__ void __launch_bounds__(256) k_comb_coefs(const float2* __restrict__ sc, const float2* __restrict__ scn,
                                                    const double2* __restrict__ rot, int per, Comb c,
                                                    float2* __restrict__ out, float2* __restrict__ out_norm) {
  __shared__ double red[256];
  const int o = blockIdx.x, tid = threadIdx.x;
  double pw = 0.0;
  for (int e = tid; e < per; e += 256) {
    double re = 0.0, im = 0.0;
    for (int a = 0; a < c.A; ++a) {
      const float2 v = sc[stage_of(c, o, a) * per + e];
      const double2 r = rot ? rot[(size_t)o * c.A + a] : make_double2(1.0, 0.0);
      re += r.x * v.x - r.y * v.y;
      im += r.x * v.y + r.y * v.x;
    }
    const float2 f = make_float2((float)(re / c.A), (float)(im / c.A));
    out[(size_t)o * per + e] = f;
    pw += (double)f.x * f.x + (double)f.y * f.y;
  }
  if (c.A == 1) {   // a reordering: the staged normalised values as they are
    for (int e = tid; e < per; e += 256) out_norm[(size_t)o * per + e] = scn[stage_of(c, o, 0) * per + e];
    return;
  }
  red[tid] = pw;
  __syncthreads();
  for (int w = 128; w > 0; w >>= 1) {
    if (tid < w) red[tid] += red[tid + w];
    __syncthreads();
  }
  const double inv = red[0] > 0.0 ? 1.0 / sqrt(red[0]) : 0.0;
  for (int e = tid; e < per; e += 256) {
    const float2 f = out[(size_t)o * per + e];
    out_norm[(size_t)o * per + e] = make_float2((float)(f.x * inv), (float)(f.y * inv));
  }
}

__global__ void __launch_bounds__(256) k_comb_plane(const float2* __restrict__ in, const double2* __restrict__ rot,
                                                    long long per, Comb c, int n_out, float2* __restrict__ out) {
  for (int o = blockIdx.y; o < n_out; o += gridDim.y) {
    const long long e0 = (long long)blockIdx.x * 1024;
    const long long e1 = e0 + 1024 < per ? e0 + 1024 : per;
    for (long long e = e0 + threadIdx.x; e < e1; e += 256) {
      double re = 0.0, im = 0.0;
      for (int a = 0; a < c.A; ++a) {
        const float2 v = in[stage_of(c, o, a) * per + e];
        const double2 r = rot ? rot[(size_t)o * c.A + a] : make_double2(1.0, 0.0);
        re += r.x * v.x - r.y * v.y;
        im += r.x * v.y + r.y * v.x;
      }
      out[(size_t)o * per + e] = make_float2((float)(re / c.A), (float)(im / c.A));
    }
  }
}

hipError_t launch_fptr(const char* base, size_t fbytes, int n_out, int L, int I, int A, int avg_mode, int in_order,
                       const void** sptr, hipStream_t s) {
  const int n = n_out * A;
  if (n < 1) return hipSuccess;
  hipLaunchKernelGGL(k_fptr, dim3((n + 255) / 256), dim3(256), 0, s, base, (unsigned long long)fbytes, n_out, L, I, A,
                     avg_mode, in_order, sptr);
  return hipGetLastError();
}

hipError_t launch_avg_rot(const float2* win, long long per, const Comb& c, int n_out, double2* rot, hipStream_t s) {
  if (n_out < 1) return hipSuccess;
  hipLaunchKernelGGL(k_avg_rot, dim3(n_out, c.A), dim3(256), 0, s, win, per, c, rot);
  return hipGetLastError();
}

hipError_t launch_comb_coefs(const float2* sc, const float2* scn, const double2* rot, int per, const Comb& c, int n_out,
                             float2* out, float2* out_norm, hipStream_t s) {
  if (n_out < 1) return hipSuccess;
  hipLaunchKernelGGL(k_comb_coefs, dim3(n_out), dim3(256), 0, s, sc, scn, rot, per, c, out, out_norm);
  return hipGetLastError();
}

hipError_t launch_comb_plane(const float2* in, const double2* rot, long long per, const Comb& c, int n_out, float2* out,
                             hipStream_t s) {
  if (n_out < 1 || per < 1) return hipSuccess;
  const long long bx = (per + 1023) / 1024;
  hipLaunchKernelGGL(k_comb_plane, dim3((unsigned)bx, (unsigned)(n_out < 65535 ? n_out : 65535)), dim3(256), 0, s, in,
                     rot, per, c, n_out, out);
  return hipGetLastError();
}

// The t2 intermediate and the fields are streamed (each element written and
// read once): non-temporal stores and loads.
typedef float m0_floatx2 __attribute__((ext_vector_type(2)));
__device__ __forceinline__ void m0_st_nt(float2* p, float2 v) {
  const m0_floatx2 t = {v.x, v.y};
  __builtin_nontemporal_store(t, reinterpret_cast<m0_floatx2*>(p));
}
__device__ __forceinline__ float2 m0_ld_nt(const float2* p) {
  const m0_floatx2 t = __builtin_nontemporal_load(reinterpret_cast<const m0_floatx2*>(p));
  return make_float2(t.x, t.y);
}

// k_m0y: grid (ceil(bx / CG), npol, frames). Column j of the box (bin
// u = uhi - j) of output frame first + z stride: its window bins v = vhi - i
// (cell (v mod wy, u mod wx)) placed at v mod Ny with the factor (-1)^v of
// the grid origin, inverse transformed (forward FFT of the conjugate,
// conjugated back), times the y phase: t2[z][p][l][j].
template <int NY, int CG>
__global__ void __launch_bounds__(256) k_m0y(M0Args m) {
  using LN = Lds<NY>;
  constexpr int ST = LN::STRIDE;
  __shared__ float2 buf[CG * ST];
  const int tid = threadIdx.x, p = blockIdx.y, z = blockIdx.z;
  const int jc0 = blockIdx.x * CG;
  const auto& P = m.pol[p];
  const size_t fr = (size_t)m.first + (size_t)z * m.stride;
  const float2* win = m.win + (fr * m.npol + p) * m.wy * m.wx;
  for (int e = tid; e < CG * ST; e += 256) buf[e] = make_float2(0.f, 0.f);
  __syncthreads();
  for (int e = tid; e < CG * P.byq; e += 256) {
    const int c = e % CG, i = e / CG, j = jc0 + c;
    if (j >= P.bxq) continue;
    const int u = P.uhi - j, v = P.vhi - i;
    int qu = u % m.wx, qv = v % m.wy, rv = v % NY;
    if (qu < 0) qu += m.wx;
    if (qv < 0) qv += m.wy;
    if (rv < 0) rv += NY;
    const float2 w = win[(size_t)qv * m.wx + qu];
    const float sg = (v & 1) ? -1.f : 1.f;
    buf[c * ST + LN::at(rv)] = make_float2(sg * w.x, -sg * w.y);
  }
  __syncthreads();
  fft_lds<NY, CG, ST, 256>(buf, m.tw_ny, tid);
  __syncthreads();
  float2* out = m.t2 + ((size_t)z * m.npol + p) * NY * m.bxp;
  for (int e = tid; e < CG * NY; e += 256) {
    const int c = e % CG, l = e / CG, j = jc0 + c;
    if (j >= P.bxq) continue;
    const float2 y = buf[c * ST + LN::at(l)];
    const float2 ph = P.phy[l];
    // conj(y) * ph
    m0_st_nt(out + (size_t)l * m.bxp + j, make_float2(y.x * ph.x + y.y * ph.y, y.x * ph.y - y.y * ph.x));
  }
}

// k_m0x: grid (ceil(Ny / TR), npol, frames). Rows l of t2: the box columns
// placed at u mod Nx with the factor (-1)^u, inverse transformed as above,
// times the x phase: the field row fields[fr][p][l][0..Nx).
template <int NX, int TR>
__global__ void __launch_bounds__(256) k_m0x(M0Args m) {
  using LN = Lds<NX>;
  constexpr int ST = LN::STRIDE;
  __shared__ float2 buf[TR * ST];
  const int tid = threadIdx.x, p = blockIdx.y, z = blockIdx.z;
  const int l0 = blockIdx.x * TR;
  const auto& P = m.pol[p];
  const size_t fr = (size_t)m.first + (size_t)z * m.stride;
  const float2* in = m.t2 + ((size_t)z * m.npol + p) * m.ny * m.bxp;
  for (int e = tid; e < TR * ST; e += 256) buf[e] = make_float2(0.f, 0.f);
  __syncthreads();
  for (int e = tid; e < TR * P.bxq; e += 256) {
    const int r = e / P.bxq, j = e % P.bxq, l = l0 + r;
    if (l >= m.ny) continue;
    const int u = P.uhi - j;
    int ru = u % NX;
    if (ru < 0) ru += NX;
    const float2 t = m0_ld_nt(in + (size_t)l * m.bxp + j);
    const float sg = (u & 1) ? -1.f : 1.f;
    buf[r * ST + LN::at(ru)] = make_float2(sg * t.x, -sg * t.y);
  }
  __syncthreads();
  fft_lds<NX, TR, ST, 256>(buf, m.tw_nx, tid);
  __syncthreads();
  float2* out = m.fields + (fr * m.npol + p) * (size_t)m.ny * NX;
  for (int e = tid; e < TR * NX; e += 256) {
    const int r = e / NX, k = e % NX, l = l0 + r;
    if (l >= m.ny) continue;
    const float2 y = buf[r * ST + LN::at(k)];
    const float2 ph = P.phx[k];
    m0_st_nt(out + (size_t)l * NX + k, make_float2(y.x * ph.x + y.y * ph.y, y.x * ph.y - y.y * ph.x));
  }
}

#define DH_M0_SIZES(X) X(64) X(128) X(256) X(320) X(512) X(640) X(1024) X(2048)

hipError_t launch_m0y(const M0Args& m, int nb, hipStream_t s) {
  if (nb < 1) return hipSuccess;
  const int bx = std::max(m.pol[0].bxq, m.npol > 1 ? m.pol[1].bxq : 0);
  if (m.gy.np > 0) return launch_m0y_gen(m, bx, nb, s);
#define X(N)                                                                                           \
  if (m.ny == N) {                                                                                    \
    constexpr int CG = N >= 1024 ? 4 : 8;                                                             \
    hipLaunchKernelGGL((k_m0y<N, CG>), dim3((bx + CG - 1) / CG, m.npol, nb), dim3(256), 0, s, m);     \
    return hipGetLastError();                                                                         \
  }
  DH_M0_SIZES(X)
#undef X
  return hipErrorInvalidValue;
}

hipError_t launch_m0x(const M0Args& m, int nb, hipStream_t s) {
  if (nb < 1) return hipSuccess;
  if (m.gx.np > 0) return launch_m0x_gen(m, nb, s);
#define X(N)                                                                                           \
  if (m.nx == N) {                                                                                    \
    constexpr int TR = N >= 2048 ? 2 : N >= 1024 ? 4 : 8;                                             \
    hipLaunchKernelGGL((k_m0x<N, TR>), dim3((m.ny + TR - 1) / TR, m.npol, nb), dim3(256), 0, s, m);   \
    return hipGetLastError();                                                                         \
  }
  DH_M0_SIZES(X)
#undef X
  return hipErrorInvalidValue;
}

}  // namespace dh
