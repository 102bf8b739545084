// Kernels for window sizes without a compiled transform ("Window sizes": the
// FFT window is any multiple of 16; the Fourier window radius is free, so the
// IFFT grid W is any length the size rule gives). A runtime-length
// mixed-radix Stockham FFT works on transforms held contiguously in LDS, with
// a second LDS buffer to write each pass into:
//   n = r0 r1 ... r(np-1), radices 2, 3, 4, 5, 7, 8, 11, 13, 16 done in
//   registers by the same DFT building blocks as the compiled kernels, and at
//   most one prime factor above 13 (n <= 2048 leaves room for one: 16 * 17 *
//   19 > 2048) as a direct DFT of that length, one output per thread.
// Pass s reads elements b + r n/R (b < n/R), multiplies element r by
// e^{-2 pi i k r / (NS R)} (NS: the product of the earlier radices, k = b mod
// NS), transforms over r and writes NS apart from (b / NS) NS R + k: natural
// order in and out.
//
//   k_row_gen    the row pass for any N_x (as k_row: two real rows packed as
//                one complex transform, the box columns kept via the
//                two-for-one split)
//   k_cspec_gen  the spectral column pass for any N_y, W_y and mode count (as
//                k_cspec, its contraction on the vector units)
//   k_m0y_gen, k_m0x_gen  the mode-0 field export for any N_y, N_x (as k_m0y, k_m0x)
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <vector>

#include "dh_fft.hpp"
#include "dh_internal.hpp"

namespace dh {

namespace {

// t1 element (box column j, row y): tiles of 16 rows (the layout of k_row)
__device__ __forceinline__ size_t gt1_at(int j, int y, int bx) { return ((size_t)(y >> 4) * bx + j) * 16 + (y & 15); }

template <int R>
__device__ __forceinline__ void gpass(const float2* __restrict__ src, float2* __restrict__ dst, int n, int ns, int ntr,
                                      const float2* __restrict__ tw, int tid, int nth) {
  const int nb = n / R;
  for (int g = tid; g < ntr * nb; g += nth) {
    const int tr = g / nb, b = g - tr * nb, k = b % ns;
    const float2* s = src + (size_t)tr * n;
    float2 v[R];
#pragma unroll
    for (int r = 0; r < R; ++r) v[r] = s[b + r * nb];
    if (ns > 1) {
#pragma unroll
      for (int r = 1; r < R; ++r) v[r] = cmul(v[r], tw[(r - 1) * ns + k]);
    }
    dft<R>(v);
    float2* d = dst + (size_t)tr * n + (b / ns) * ns * R + k;
#pragma unroll
    for (int r = 0; r < R; ++r) d[r * ns] = v[r];
  }
}

// a prime radix R > 16: each output a direct sum over its butterfly's R inputs
__device__ __forceinline__ void gpass_prime(const float2* __restrict__ src, float2* __restrict__ dst, int n, int R,
                                            int ns, int ntr, const float2* __restrict__ tw,
                                            const float2* __restrict__ roots, int tid, int nth) {
  const int nb = n / R;
  for (int g = tid; g < ntr * n; g += nth) {
    const int tr = g / n, e = g - tr * n;
    const int b = e % nb, q = e / nb, k = b % ns;
    const float2* s = src + (size_t)tr * n;
    float2 acc = make_float2(0.f, 0.f);
    int m = 0;                                   // r q mod R
    for (int r = 0; r < R; ++r) {
      float2 x = s[b + r * nb];
      if (ns > 1 && r > 0) x = cmul(x, tw[(r - 1) * ns + k]);
      const float2 w = roots[m];
      acc.x = fmaf(x.x, w.x, fmaf(-x.y, w.y, acc.x));
      acc.y = fmaf(x.x, w.y, fmaf(x.y, w.x, acc.y));
      m += q;
      if (m >= R) m -= R;
    }
    dst[(size_t)tr * n + (b / ns) * ns * R + k + q * ns] = acc;
  }
}

// Forward FFT of ntr transforms of length G.n held contiguously in a (LDS);
// b is scratch of the same size. Returns the buffer with the result. Starts
// and ends with a barrier; every thread of the workgroup calls it.
__device__ float2* fft_gen(float2* a, float2* b, int ntr, const GenFft& G, const float2* __restrict__ tw, int tid,
                           int nth) {
  __syncthreads();
  float2* src = a;
  float2* dst = b;
  int ns = 1;
  for (int s = 0; s < G.np; ++s) {
    const int R = G.r[s];
    const float2* t = tw + G.off[s];
    switch (R) {
      case 2: gpass<2>(src, dst, G.n, ns, ntr, t, tid, nth); break;
      case 3: gpass<3>(src, dst, G.n, ns, ntr, t, tid, nth); break;
      case 4: gpass<4>(src, dst, G.n, ns, ntr, t, tid, nth); break;
      case 5: gpass<5>(src, dst, G.n, ns, ntr, t, tid, nth); break;
      case 7: gpass<7>(src, dst, G.n, ns, ntr, t, tid, nth); break;
      case 8: gpass<8>(src, dst, G.n, ns, ntr, t, tid, nth); break;
      case 11: gpass<11>(src, dst, G.n, ns, ntr, t, tid, nth); break;
      case 13: gpass<13>(src, dst, G.n, ns, ntr, t, tid, nth); break;
      case 16: gpass<16>(src, dst, G.n, ns, ntr, t, tid, nth); break;
      default: gpass_prime(src, dst, G.n, R, ns, ntr, t, tw + G.roots, tid, nth); break;
    }
    __syncthreads();
    float2* x = src;
    src = dst;
    dst = x;
    ns *= R;
  }
  return src;
}

__device__ __forceinline__ float gpx(const float* p) { return *p; }
__device__ __forceinline__ float gpx(const unsigned short* p) { return (float)*p; }

}  // namespace

// k_row_gen: grid (ceil(ny / (2 trg)), npol, nb), 256 threads, dynamic LDS
// 2 trg nx float2: trg transforms of the row pairs (2t, 2t + 1) of the tile.
template <typename TIn>
__global__ void __launch_bounds__(256) k_row_gen(KArgs A, const TIn* __restrict__ frames, int b0, int trg) {
  extern __shared__ float2 dsm[];
  const int tid = threadIdx.x, p = blockIdx.y, bl = blockIdx.z;
  const int nx = A.nx;
  const PolTab& P = A.pol[p];
  const TIn* fr = A.fptr ? static_cast<const TIn*>(A.fptr[b0 + bl]) : frames + (size_t)(b0 + bl) * A.frame_h * A.frame_w;
  const TIn* win = fr + (size_t)P.y0 * A.frame_w + P.x0;
  const int y0 = blockIdx.x * 2 * trg;
  float2* a = dsm;
  float2* b = dsm + (size_t)trg * nx;
  for (int e = tid; e < trg * nx; e += 256) {
    const int t = e / nx, x = e - t * nx, y = y0 + 2 * t;
    float2 v = make_float2(0.f, 0.f);
    if (y < A.ny) {
      const TIn* r0 = win + (size_t)y * A.frame_w + x;
      v = make_float2(gpx(r0), gpx(r0 + A.frame_w));
    }
    a[e] = v;
  }
  const float2* res = fft_gen(a, b, trg, A.gx, A.tw_nx, tid, 256);
  float2* out = A.t1 + (size_t)(bl * A.npol + p) * A.bx * A.ny;
  for (int e = tid; e < trg * A.bx; e += 256) {
    const int t = e % trg, j = e / trg, y = y0 + 2 * t;
    if (y >= A.ny) continue;
    const int k = ((P.k0 + j) % nx + nx) % nx;
    const int km = k == 0 ? 0 : nx - k;
    const float2 z1 = res[(size_t)t * nx + k];
    const float2 z2 = conjf2(res[(size_t)t * nx + km]);
    const float2 d = csub(z1, z2);
    // rows y and y + 1 of box column j (ny is even)
    *reinterpret_cast<float4*>(out + gt1_at(j, y, A.bx)) =
        make_float4(0.5f * (z1.x + z2.x), 0.5f * (z1.y + z2.y), 0.5f * d.y, -0.5f * d.x);
  }
}

// k_cspec_gen: grid (ceil(bx / cg), npol, nb), 256 threads, dynamic LDS
// (2 cg ny + cg gp) float2. The column FFT of cg box columns, the window (if
// kept), then
//   Q[c][n] = sum_i mask(j, i) conj(S[j][i]) ys[i][n]   (j = jc0 + c)
//   partial[m][n] = sum_c xs[j][m] Q[c][n]
// and the block's field power by Parseval, as in k_cspec.
__global__ void __launch_bounds__(256) k_cspec_gen(KArgs A, int b0, int cg) {
  extern __shared__ float2 dsm[];
  __shared__ float s_pw[4];
  const int tid = threadIdx.x, p = blockIdx.y, bl = blockIdx.z;
  const int ny = A.ny, gp = A.gp, jc0 = blockIdx.x * cg;
  const PolTab& P = A.pol[p];
  float2* a = dsm;
  float2* b = dsm + (size_t)cg * ny;
  float2* q = dsm + (size_t)2 * cg * ny;
  const float2* in = A.t1 + (size_t)(bl * A.npol + p) * A.bx * ny;
  for (int e = tid; e < cg * ny; e += 256) {
    const int c = e / ny, y = e - c * ny, j = jc0 + c;
    a[e] = j < A.bx ? in[gt1_at(j, y, A.bx)] : make_float2(0.f, 0.f);
  }
  const float2* res = fft_gen(a, b, cg, A.gy, A.tw_ny, tid, 256);
  if (A.window) {
    // window = M * I~ = conj(val) (-1)^(u+v) Nx Ny at (v mod wy, u mod wx), as in k_cspec
    float2* win = A.window + ((size_t)(b0 + bl) * A.npol + p) * A.wy * A.wx;
    for (int e = tid; e < cg * A.by; e += 256) {
      const int c = e % cg, i = e / cg, j = jc0 + c;
      if (j >= A.bx || i >= P.byq) continue;
      const int2 mr = P.mrow[i];
      if (j < mr.x || j > mr.y) continue;
      int vv = (P.ky0 + i) % ny;
      if (vv < 0) vv += ny;
      const float2 val = cmul(cmul(res[(size_t)c * ny + vv], conjf2(P.rhox[j])), conjf2(P.rhoy[i]));
      const int u = -(P.k0 + j), v = -(P.ky0 + i);
      int qu = u % A.wx, qv = v % A.wy;
      if (qu < 0) qu += A.wx;
      if (qv < 0) qv += A.wy;
      const float sg = ((u + v) & 1) ? -A.nxny : A.nxny;
      win[(size_t)qv * A.wx + qu] = make_float2(sg * val.x, -sg * val.y);
    }
  }
  float pw = 0.f;
  for (int e = tid; e < cg * gp; e += 256) {
    const int c = e / gp, n = e - c * gp, j = jc0 + c;
    float2 acc = make_float2(0.f, 0.f);
    if (j < A.bx) {
      for (int i = 0; i < A.by; ++i) {
        const int2 mr = P.mrow[i];
        if (j < mr.x || j > mr.y) continue;
        int vv = (P.ky0 + i) % ny;
        if (vv < 0) vv += ny;
        const float2 s = res[(size_t)c * ny + vv];
        acc = cadd(acc, cmul(conjf2(s), P.ys[(size_t)i * gp + n]));
        if (n == 0) pw = fmaf(s.x, s.x, fmaf(s.y, s.y, pw));
      }
    }
    q[e] = acc;
  }
#pragma unroll
  for (int off = 32; off > 0; off >>= 1) pw += __shfl_xor(pw, off, 64);
  if ((tid & 63) == 0) s_pw[tid >> 6] = pw;
  __syncthreads();
  const int pstride = A.nmodes + 1;
  float2* part = A.partial + ((size_t)(bl * A.nblk + blockIdx.x) * A.npol + p) * pstride;
  if (tid == 0)
    part[A.nmodes] = make_float2(A.capt ? (((s_pw[0] + s_pw[1]) + s_pw[2]) + s_pw[3]) * A.spow : 0.f, 0.f);
  for (int e = tid; e < A.nmodes; e += 256) {
    const short2 mn = A.modes[e];
    float2 acc = make_float2(0.f, 0.f);
    for (int c = 0; c < cg && jc0 + c < A.bx; ++c)
      acc = cadd(acc, cmul(P.xs[(size_t)(jc0 + c) * gp + mn.x], q[c * gp + mn.y]));
    part[e] = acc;
  }
}

// k_m0y_gen: grid (ceil(bx / cg), npol, frames), dynamic LDS 2 cg ny float2;
// as k_m0y.
__global__ void __launch_bounds__(256) k_m0y_gen(M0Args m, int cg) {
  extern __shared__ float2 dsm[];
  const int tid = threadIdx.x, p = blockIdx.y, z = blockIdx.z;
  const int ny = m.ny, jc0 = blockIdx.x * cg;
  const auto& P = m.pol[p];
  const size_t fr = (size_t)m.first + (size_t)z * m.stride;
  const float2* win = m.win + (fr * m.npol + p) * m.wy * m.wx;
  float2* a = dsm;
  float2* b = dsm + (size_t)cg * ny;
  for (int e = tid; e < cg * ny; e += 256) a[e] = make_float2(0.f, 0.f);
  __syncthreads();
  for (int e = tid; e < cg * P.byq; e += 256) {
    const int c = e % cg, i = e / cg, j = jc0 + c;
    if (j >= P.bxq) continue;
    const int u = P.uhi - j, v = P.vhi - i;
    int qu = u % m.wx, qv = v % m.wy, rv = v % ny;
    if (qu < 0) qu += m.wx;
    if (qv < 0) qv += m.wy;
    if (rv < 0) rv += ny;
    const float2 w = win[(size_t)qv * m.wx + qu];
    const float sg = (v & 1) ? -1.f : 1.f;
    a[(size_t)c * ny + rv] = make_float2(sg * w.x, -sg * w.y);
  }
  const float2* res = fft_gen(a, b, cg, m.gy, m.tw_ny, tid, 256);
  float2* out = m.t2 + ((size_t)z * m.npol + p) * ny * m.bxp;
  for (int e = tid; e < cg * ny; e += 256) {
    const int c = e % cg, l = e / cg, j = jc0 + c;
    if (j >= P.bxq) continue;
    const float2 y = res[(size_t)c * ny + l];
    const float2 ph = P.phy[l];
    // conj(y) * ph
    out[(size_t)l * m.bxp + j] = make_float2(y.x * ph.x + y.y * ph.y, y.x * ph.y - y.y * ph.x);
  }
}

// k_m0x_gen: grid (ceil(ny / tr), npol, frames), dynamic LDS 2 tr nx float2;
// as k_m0x.
__global__ void __launch_bounds__(256) k_m0x_gen(M0Args m, int tr) {
  extern __shared__ float2 dsm[];
  const int tid = threadIdx.x, p = blockIdx.y, z = blockIdx.z;
  const int nx = m.nx, l0 = blockIdx.x * tr;
  const auto& P = m.pol[p];
  const size_t fr = (size_t)m.first + (size_t)z * m.stride;
  const float2* in = m.t2 + ((size_t)z * m.npol + p) * m.ny * m.bxp;
  float2* a = dsm;
  float2* b = dsm + (size_t)tr * nx;
  for (int e = tid; e < tr * nx; e += 256) a[e] = make_float2(0.f, 0.f);
  __syncthreads();
  for (int e = tid; e < tr * P.bxq; e += 256) {
    const int r = e / P.bxq, j = e % P.bxq, l = l0 + r;
    if (l >= m.ny) continue;
    const int u = P.uhi - j;
    int ru = u % nx;
    if (ru < 0) ru += nx;
    const float2 t = in[(size_t)l * m.bxp + j];
    const float sg = (u & 1) ? -1.f : 1.f;
    a[(size_t)r * nx + ru] = make_float2(sg * t.x, -sg * t.y);
  }
  const float2* res = fft_gen(a, b, tr, m.gx, m.tw_nx, tid, 256);
  float2* out = m.fields + (fr * m.npol + p) * (size_t)m.ny * nx;
  for (int e = tid; e < tr * nx; e += 256) {
    const int r = e / nx, k = e % nx, l = l0 + r;
    if (l >= m.ny) continue;
    const float2 y = res[(size_t)r * nx + k];
    const float2 ph = P.phx[k];
    out[(size_t)l * nx + k] = make_float2(y.x * ph.x + y.y * ph.y, y.x * ph.y - y.y * ph.x);
  }
}

// ---------------------------------------------------------------------------
// host side

int gen_rows_per_block(int nx) { return std::max(1, std::min(16, 4096 / nx)); }     // 2 trg nx float2 <= 64 KB
int gen_cols_per_block(int ny, int gp) { return std::max(1, std::min(8, 65536 / (16 * ny + 8 * gp))); }

bool gen_plan(int n, GenFft* g) {
  *g = GenFft{};
  if (n < 2 || n > kGenMaxN) return false;
  g->n = n;
  int m = n, np = 0;
  static const int small[] = {16, 8, 4, 2, 3, 5, 7, 11, 13};
  for (int r : small)
    while (m % r == 0) {
      if (np == kGenMaxPasses) return false;
      g->r[np++] = r;
      m /= r;
    }
  if (m > 1) {                                  // one prime factor above 13
    for (int d = 2; d * d <= m; ++d)
      if (m % d == 0) return false;
    if (np == kGenMaxPasses) return false;
    g->r[np++] = m;
  }
  g->np = np;
  int off = 0, ns = 1;
  for (int s = 0; s < np; ++s) {
    g->off[s] = off;
    off += (g->r[s] - 1) * ns;
    ns *= g->r[s];
  }
  g->roots = off;
  return true;
}

std::vector<float2> gen_twiddles(const GenFft& g) {
  constexpr double kPi2 = 6.283185307179586476925286766559;
  std::vector<float2> t;
  int ns = 1;
  for (int s = 0; s < g.np; ++s) {
    const int R = g.r[s];
    for (int r = 1; r < R; ++r)
      for (int k = 0; k < ns; ++k) {
        const double a = -kPi2 * (double)k * r / ((double)ns * R);
        t.push_back(make_float2((float)std::cos(a), (float)std::sin(a)));
      }
    ns *= R;
  }
  const int p = g.np ? g.r[g.np - 1] : 1;
  if (p > 16)
    for (int q = 0; q < p; ++q) {
      const double a = -kPi2 * (double)q / p;
      t.push_back(make_float2((float)std::cos(a), (float)std::sin(a)));
    }
  if (t.empty()) t.push_back(make_float2(1.f, 0.f));
  return t;
}

size_t gen_twiddle_count(int n) { return (size_t)n + (size_t)n / 16 + 1; }

hipError_t launch_row_gen(const KArgs& a, const void* frames, int u16, int b0, int nb, hipStream_t s) {
  const int trg = gen_rows_per_block(a.nx);
  const size_t lds = (size_t)2 * trg * a.nx * sizeof(float2);
  dim3 grid((a.ny + 2 * trg - 1) / (2 * trg), a.npol, nb);
  if (u16)
    hipLaunchKernelGGL(k_row_gen<unsigned short>, grid, dim3(256), lds, s, a, (const unsigned short*)frames, b0, trg);
  else
    hipLaunchKernelGGL(k_row_gen<float>, grid, dim3(256), lds, s, a, (const float*)frames, b0, trg);
  return hipGetLastError();
}

hipError_t launch_cspec_gen(const KArgs& a, int b0, int nb, hipStream_t s) {
  const int cg = gen_cols_per_block(a.ny, a.gp);
  const size_t lds = ((size_t)2 * cg * a.ny + (size_t)cg * a.gp) * sizeof(float2);
  dim3 grid((a.bx + cg - 1) / cg, a.npol, nb);
  hipLaunchKernelGGL(k_cspec_gen, grid, dim3(256), lds, s, a, b0, cg);
  return hipGetLastError();
}

hipError_t launch_m0y_gen(const M0Args& m, int bx, int nb, hipStream_t s) {
  const int cg = gen_rows_per_block(m.ny);
  const size_t lds = (size_t)2 * cg * m.ny * sizeof(float2);
  hipLaunchKernelGGL(k_m0y_gen, dim3((bx + cg - 1) / cg, m.npol, nb), dim3(256), lds, s, m, cg);
  return hipGetLastError();
}

hipError_t launch_m0x_gen(const M0Args& m, int nb, hipStream_t s) {
  const int tr = gen_rows_per_block(m.nx);
  const size_t lds = (size_t)2 * tr * m.nx * sizeof(float2);
  hipLaunchKernelGGL(k_m0x_gen, dim3((m.ny + tr - 1) / tr, m.npol, nb), dim3(256), lds, s, m, tr);
  return hipGetLastError();
}

}  // namespace dh
