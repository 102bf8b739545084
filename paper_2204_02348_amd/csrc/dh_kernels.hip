// gfx950 kernels of the off-axis holography path.
//
//   k_row   pipeline step 1: frame window load (u16/f32 -> f32), real FFT
//           along x of two rows at a time (packed as one complex row), and
//           only the spectrum columns that hold the Fourier window are kept.
//   k_col   pipeline step 2, first half: FFT along y of the kept columns,
//           crop of the window rows around the reference-tilt peak, the
//           circular window (mask), the beam-centre ramp, and the inverse
//           FFT along y at the Fourier-window size (IFFT resolution mode 1).
//   k_fld   pipeline step 2, second half + step 3: inverse FFT along x,
//           removal of the reference tilt and defocus, and the separable
//           Hermite-Gaussian overlap as two real MFMA contractions per
//           16-row block (x first, then y), in FP32.
//   k_norm  per-frame total power over both polarisations in FP64 and the
//           power-normalised coefficients.
//   k_hg    Hermite-Gaussian 1D tables by the normalised FP64 recurrence.
//
// Layouts: frames [b][frame_h][frame_w] row-major (x fastest); spectra and
// fields complex64 interleaved; every intermediate row-major with the
// contiguous axis the one the next kernel reads along.
#include <algorithm>

#include "dh_fft.hpp"
#include "dh_internal.hpp"

namespace dh {

typedef float floatx4 __attribute__((ext_vector_type(4)));

constexpr int kTPB = 256;

typedef short shortx4 __attribute__((ext_vector_type(4)));
typedef _Float16 halfx4 __attribute__((ext_vector_type(4)));

// Streamed intermediates (t1 written by the row pass and read by the column
// pass, f2 written by the column pass and read by the field pass) use
// non-temporal loads and stores: each element is touched once, and keeping it
// out of the caches measured a few per cent faster. Frame loads are ordinary:
// several load instructions share each cache line.
typedef float floatx2 __attribute__((ext_vector_type(2)));
__device__ __forceinline__ float2 ld_nt(const float2* p) {
  const floatx2 t = __builtin_nontemporal_load(reinterpret_cast<const floatx2*>(p));
  return make_float2(t.x, t.y);
}
__device__ __forceinline__ void st_nt(float2* p, float2 v) {
  const floatx2 t = {v.x, v.y};
  __builtin_nontemporal_store(t, reinterpret_cast<floatx2*>(p));
}
// Pointers the compiler cannot place in the global address space (loaded from
// memory, or a select between such pointers) would be accessed with flat
// instructions, which also hold the LDS counter; the frames are always global.
template <typename T>
using gptr = const __attribute__((address_space(1))) T*;
template <typename T>
__device__ __forceinline__ gptr<T> as_global(const T* p) { return (gptr<T>)p; }

template <typename T>
__device__ __forceinline__ float load_px(gptr<T> p) { return (float)(*p); }

// round-to-nearest-even FP32 -> BF16 (finite inputs)
__device__ __forceinline__ unsigned short bf16_rne(float x) {
  unsigned int u = __float_as_uint(x);
  u += 0x7fffu + ((u >> 16) & 1u);
  return (unsigned short)(u >> 16);
}
__device__ __forceinline__ float bf16_to_f32(unsigned short b) { return __uint_as_float((unsigned int)b << 16); }


// Raw buffer access (32-bit lane offsets; the per-load stride goes in the
// scalar offset): descriptor word 3 of the gfx9 family, non-temporal loads.
__device__ __forceinline__ __amdgpu_buffer_rsrc_t make_rsrc(const void* p, unsigned bytes) {
  return __builtin_amdgcn_make_buffer_rsrc(const_cast<void*>(p), (short)0, (int)bytes, 0x00020000);
}
__device__ __forceinline__ float2 buf_ld_nt(__amdgpu_buffer_rsrc_t r, int voff, int soff) {
  return __builtin_bit_cast(float2, __builtin_amdgcn_raw_buffer_load_b64(r, voff, soff, 2));
}
// t1 travels non-temporally unless the build asks for cached t1 traffic
// (-DDH_T1_CACHED=1), the form for launches whose t1 fits the caches
#ifndef DH_T1_CACHED
#define DH_T1_CACHED 0
#endif
constexpr bool kT1Nt = !DH_T1_CACHED;
__device__ __forceinline__ float2 buf_ld_t1(__amdgpu_buffer_rsrc_t r, int voff, int soff) {
  return __builtin_bit_cast(float2, __builtin_amdgcn_raw_buffer_load_b64(r, voff, soff, kT1Nt ? 2 : 0));
}
template <int AUX>
__device__ __forceinline__ float2 buf_ld_aux(__amdgpu_buffer_rsrc_t r, int voff, int soff) {
  return __builtin_bit_cast(float2, __builtin_amdgcn_raw_buffer_load_b64(r, voff, soff, AUX));
}

// t1 element (box column j, row y) of one frame and pol: tiles of 16 rows,
// [y / 16][j][y % 16], so that a row-pass block's writes are contiguous
__device__ __forceinline__ size_t t1_at(int j, int y, int bx) { return ((size_t)(y >> 4) * bx + j) * 16 + (y & 15); }

// Box row / column held by IFFT row / column q: bin u sits at q = u mod W and
// box index j = u_hi - u, so j = (u_hi - q) mod W; -1 if j is outside the pol's
// box. (u_hi = -k0, v_hi = -ky0.)
__device__ __forceinline__ int box_of(int uhi, int q, int w, int nbox) {
  int j = (uhi - q) % w;
  if (j < 0) j += w;
  return j < nbox ? j : -1;
}

// Twiddle tables of a transform length (entries after the first pass), staged
// into LDS once per workgroup; their loads overlap the first pass's operands.
template <int N> constexpr int twn() { return N > FftPlan<N>::R0 ? N - FftPlan<N>::R0 : 1; }

template <int N, int TPB>
__device__ __forceinline__ void stage_twiddles(float2* dst, const float2* __restrict__ src, int tid) {
  for (int e = tid; e < twn<N>(); e += TPB) dst[e] = src[e];
}

// A small table bound for LDS, held in registers between its loads and its
// LDS stores: the loads are issued ahead of a kernel's main operand loads and
// the stores wait only for them, so the table costs one memory latency that
// overlaps the main loads. Entries [n, N) get `fill`; n >= 1.
template <typename T, int N, int TPB>
struct Staged {
  static constexpr int IT = (N + TPB - 1) / TPB;
  T v[IT];
  __device__ __forceinline__ void load(const T* __restrict__ src, int n, int tid) {
#pragma unroll
    for (int i = 0; i < IT; ++i) {
      const int e = tid + i * TPB;
      v[i] = src[e < n ? e : n - 1];
    }
  }
  __device__ __forceinline__ void store(T* dst, int n, T fill, int tid) const {
#pragma unroll
    for (int i = 0; i < IT; ++i) {
      const int e = tid + i * TPB;
      if (N % TPB == 0 || e < N) dst[e] = e < n ? v[i] : fill;
    }
  }
};

// ---------------------------------------------------------------------------
// k_row: grid (ceil(ny / (2 TR TT)), npol, nb), TPB = TR * NX / R0 threads;
// TT row tiles per workgroup, each TR complex transforms of NX, each the pair
// of real rows (2t, 2t+1) packed as re + i im. The first pass takes its
// operands straight from the frame; all tiles' loads are issued up front.
// t1 at (box column j, row y) = sum_x I[y][x] e^{-2 pi i k x / NX},
// k = k0 + j (mod NX), stored at t1_at(j, y)
template <int NX, int TR> struct RowShape {
  using L = Lds<NX>;
  static constexpr int TPB = TR * NX / FftPlan<NX>::R0;
  // 2048-point rows: the twiddles (16 KB) are read through the caches, so
  // that two 512-thread workgroups fit on a CU
  static constexpr bool TWG = NX >= 2048;
  static constexpr int BUF = TR * L::STRIDE;            // float2 of LDS: the transforms
  static constexpr int TWS = TWG ? 1 : twn<NX>();       // float2 of LDS: the twiddles
};

// The row pass of row-tile group `tg` of frame `bl` (within the launch, frames
// from b0), pol p, into `out` (that frame and pol's t1); buf and tws: LDS of
// RowShape's sizes.
template <int NX, int TR, typename TIn, int TT>
__device__ __forceinline__ void row_tiles(const KArgs& A, const TIn* __restrict__ frames, int b0, int tg, int p,
                                          int bl, float2* __restrict__ out, float2* buf, float2* tws, int tid) {
  using RS = RowShape<NX, TR>;
  using L = typename RS::L;
  constexpr int TPB = RS::TPB;
  using Q = Pass1<NX, TR, TPB>;
  static_assert(Q::IT == 1, "one first-pass butterfly per thread");
  constexpr bool TWG = RS::TWG;
  const PolTab& P = A.pol[p];
  Staged<float2, TWG ? 1 : twn<NX>(), TPB> stw;
  if constexpr (!TWG) stw.load(A.tw_nx, twn<NX>(), tid);
  const TIn* fr = A.fptr ? static_cast<const TIn*>(A.fptr[b0 + bl]) : frames + (size_t)(b0 + bl) * A.frame_h * A.frame_w;
  const gptr<TIn> win = as_global(fr) + ((size_t)P.y0 * A.frame_w + P.x0);
  // the operands of every tile are requested up front: later tiles' loads are
  // in flight while the earlier tiles' transforms run. A tile past the last
  // row (odd tile count) loads row pair 0 instead and stores nothing.
  float2 v[TT][Q::R0];
  {
    const int t = tid / Q::NB, b = tid % Q::NB;
#pragma unroll
    for (int tt = 0; tt < TT; ++tt) {
      const int y0 = (tg * TT + tt) * (2 * TR);
      const int y = (y0 < A.ny ? y0 : 0) + 2 * t;      // ny is a multiple of 2 TR
      const gptr<TIn> r0 = win + ((size_t)y * A.frame_w + b);
      const gptr<TIn> r1 = r0 + A.frame_w;
#pragma unroll
      for (int r = 0; r < Q::R0; ++r) {
        v[tt][r].x = load_px(r0 + r * Q::NB);
        v[tt][r].y = load_px(r1 + r * Q::NB);
      }
      if constexpr (!TWG) if (tt == 0) stw.store(tws, twn<NX>(), make_float2(0.f, 0.f), tid);
    }
  }
#pragma unroll
  for (int tt = 0; tt < TT; ++tt) {
    const int ybase = (tg * TT + tt) * (2 * TR);
    if (tt > 0) __syncthreads();           // the previous tile's split has read buf
    fft_pass1_regs<NX, TR, L::STRIDE, TPB>(v + tt, buf, tid);
    if constexpr (TWG)
      fft_rest<NX, TR, L::STRIDE, TPB>(buf, as_global(A.tw_nx), tid);
    else
      fft_rest<NX, TR, L::STRIDE, TPB>(buf, static_cast<const float2*>(tws), tid);
    // two-for-one split at the kept bins: both rows of a pair from Z[k], Z[NX-k]
    {
      for (int e = tid; e < TR * A.bx; e += TPB) {
        const int t = e % TR, j = e / TR;
        const int y = ybase + 2 * t;
        if (y >= A.ny) continue;
        // bins are periodic: a tilt of any size reaches its window through k mod NX
        const int k = ((P.k0 + j) % NX + NX) % NX;
        const int km = (k == 0) ? 0 : NX - k;
        const float2* tb = buf + t * L::STRIDE;
        const float2 z1 = tb[L::at(k)];
        const float2 z2 = conjf2(tb[L::at(km)]);
        const float2 d = csub(z1, z2);
        const float4 x = make_float4(0.5f * (z1.x + z2.x), 0.5f * (z1.y + z2.y), 0.5f * d.y, -0.5f * d.x);
        float2* o = out + t1_at(j, y, A.bx);
        // rows y, y+1 (ny is even). A workgroup writes 2 TR rows of each
        // 16-row tile per phase: from 64 B on, non-temporal stores are faster;
        // the 32 B pieces of TR = 2 need the cache to merge them into lines
        if constexpr (2 * TR >= 8 && kT1Nt) {
          const floatx4 t4 = {x.x, x.y, x.z, x.w};
          __builtin_nontemporal_store(t4, reinterpret_cast<floatx4*>(o));
        } else {
          *reinterpret_cast<float4*>(o) = x;
        }
      }
    }
  }
}

// Resident row-pass workgroups. The f32 two-tile passes measured faster with
// fewer of them in flight per CU; the uint16 passes measured slower.
//  - 320 points (640-wide two-pol frames): compiled for three waves per SIMD,
//    so the compiler keeps all 64 frame loads of a thread in registers (129
//    VGPRs instead of 89) and a CU runs four workgroups instead of six (1000
//    frames: 0.378 -> 0.368 ms).
//  - 512 points (1024-wide two-pol frames): the LDS footprint is raised so
//    that two workgroups fit on a CU instead of four; the register budget
//    alone does not limit residency (543 frames: 0.686 -> 0.613 ms).
template <int NX, typename TIn, int TT> constexpr int row_wpe() {
  return NX == 320 && TT == 2 && sizeof(TIn) == 4 ? 3 : 8;
}
template <int NX, typename TIn, int TT> constexpr int row_lds_floor() {   // bytes
  return NX == 512 && TT == 2 && sizeof(TIn) == 4 ? 56 * 1024 : 0;
}

template <int NX, int TR, typename TIn, int TT>
__global__ void __launch_bounds__(TR * NX / FftPlan<NX>::R0) __attribute__((amdgpu_waves_per_eu(1, row_wpe<NX, TIn, TT>())))
k_row(KArgs A, const TIn* __restrict__ frames, int b0) {
  using RS = RowShape<NX, TR>;
  constexpr int FLOOR = (row_lds_floor<NX, TIn, TT>() - RS::TWS * 8) / 8;
  __shared__ float2 buf[RS::BUF > FLOOR ? RS::BUF : FLOOR];
  __shared__ float2 tws[RS::TWS];
  const int p = blockIdx.y, bl = blockIdx.z;
  float2* out = A.t1 + (size_t)(bl * A.npol + p) * A.bx * A.ny;
  row_tiles<NX, TR, TIn, TT>(A, frames, b0, blockIdx.x, p, bl, out, buf, tws, threadIdx.x);
}

// ---------------------------------------------------------------------------
// k_col: grid (ceil(bx / CG), npol, nb). CG box columns per block: FFT along
// y (first pass straight from the tiled t1), gather of the masked
// window rows (stored as conj of the IFFT input), IFFT along y at the window
// size; f2 rows have pitch bxp.
template <int NY, int WY, int CG>
__global__ void __launch_bounds__(kTPB) k_col(KArgs A, int b0) {
  using LN = Lds<NY>;
  using LW = Lds<WY>;
  using Q = Pass1<NY, CG, kTPB>;
  constexpr int ST = (LN::STRIDE > LW::STRIDE) ? LN::STRIDE : LW::STRIDE;
  // at 2048 rows the twiddles of both transforms and the box-row ramp are read
  // through the caches: the workgroup's LDS drops from 102 to 75 KB and two
  // workgroups fit on a CU
  constexpr bool TWG = NY >= 2048;
  __shared__ float2 buf[CG * ST];
  __shared__ float2 twy[TWG ? 1 : twn<NY>()];
  __shared__ float2 tww[TWG ? 1 : twn<WY>()];
  __shared__ int2 s_mrow[WY];
  __shared__ float2 s_crx[CG];              // conj(rho_x) of this block's columns
  __shared__ float2 s_cry[TWG ? 1 : WY];    // conj(rho_y) by box row
  const int tid = threadIdx.x;
  const int p = blockIdx.y;
  const int bl = blockIdx.z;
  const PolTab& P = A.pol[p];
  const int jc0 = blockIdx.x * CG;
  Staged<float2, TWG ? 1 : twn<NY>(), kTPB> stwy;
  Staged<float2, TWG ? 1 : twn<WY>(), kTPB> stww;
  Staged<int2, WY, kTPB> smr;
  Staged<float2, TWG ? 1 : WY, kTPB> scy;
  Staged<float2, CG, kTPB> scx;
  if constexpr (!TWG) {
    stwy.load(A.tw_ny, twn<NY>(), tid);
    stww.load(A.tw_wy, twn<WY>(), tid);
    scy.load(P.rhoy, A.by, tid);
  }
  smr.load(P.mrow, A.by, tid);
  const int ncx = A.bx - jc0 < CG ? A.bx - jc0 : CG;
  scx.load(P.rhox + jc0, ncx, tid);
  const float2* in = A.t1 + ((size_t)(bl * A.npol + p) * A.bx) * NY;
  {
    float2 v[Q::IT][Q::R0];
    // element (j, b + r NB) of the tiled t1 at byte t1_at * 8; where NB is a
    // multiple of 16 the row tile advances by NB / 16 per r at a fixed offset
    // within the tile, and that step goes in the scalar offset
    const __amdgpu_buffer_rsrc_t rt = make_rsrc(in, (unsigned)(A.bx * NY * 8));
#pragma unroll
    for (int it = 0; it < Q::IT; ++it) {
      const int g = tid + it * kTPB;
      const int c = g / Q::NB, b = g % Q::NB;
      const int j = (Q::TOTAL % kTPB == 0 || g < Q::TOTAL) && jc0 + c < A.bx ? jc0 + c : 0;
      if constexpr (Q::NB % 16 == 0) {
        const int voff = ((b >> 4) * A.bx + j) * 128 + (b & 15) * 8;
        const int rstride = (Q::NB / 16) * A.bx * 128;
#pragma unroll
        for (int r = 0; r < Q::R0; ++r) v[it][r] = buf_ld_t1(rt, voff, r * rstride);
      } else {
#pragma unroll
        for (int r = 0; r < Q::R0; ++r) v[it][r] = buf_ld_t1(rt, (int)t1_at(j, b + r * Q::NB, A.bx) * 8, 0);
      }
    }
#pragma unroll
    for (int i = 0; i < scx.IT; ++i) scx.v[i] = conjf2(scx.v[i]);
    if constexpr (!TWG) {
#pragma unroll
      for (int i = 0; i < scy.IT; ++i) scy.v[i] = conjf2(scy.v[i]);
      stwy.store(twy, twn<NY>(), make_float2(0.f, 0.f), tid);
      stww.store(tww, twn<WY>(), make_float2(0.f, 0.f), tid);
      scy.store(s_cry, A.by, make_float2(0.f, 0.f), tid);
    }
    smr.store(s_mrow, A.by, make_int2(1, 0), tid);
    scx.store(s_crx, ncx, make_float2(0.f, 0.f), tid);
    fft_pass1_regs<NY, CG, ST, kTPB>(v, buf, tid);
  }
  if constexpr (TWG)
    fft_rest<NY, CG, ST, kTPB>(buf, as_global(A.tw_ny), tid);
  else
    fft_rest<NY, CG, ST, kTPB>(buf, static_cast<const float2*>(twy), tid);
  constexpr int NE = (CG * WY + kTPB - 1) / kTPB;
  float2 z[NE];
  const bool keep_win = A.window != nullptr;
  float2* win = keep_win ? A.window + ((size_t)(b0 + bl) * A.npol + p) * A.wy * A.wx : nullptr;
#pragma unroll
  for (int it = 0; it < NE; ++it) {
    const int e = tid + it * kTPB;
    float2 val = make_float2(0.f, 0.f);
    if (e < CG * WY) {
      const int c = e / WY, q = e % WY;
      const int j = jc0 + c;
      const int i = box_of(-P.ky0, q, WY, P.byq);
      if (i >= 0 && j < A.bx) {
        const int2 mr = s_mrow[i];
        if (j >= mr.x && j <= mr.y) {
          int vv = (P.ky0 + i) % NY;
          if (vv < 0) vv += NY;
          const float2 f = buf[c * ST + LN::at(vv)];
          float2 cry;
          if constexpr (TWG)
            cry = conjf2(ld_tw(as_global(P.rhoy), i));
          else
            cry = s_cry[i];
          val = cmul(cmul(f, s_crx[c]), cry);
          if (keep_win) {
            // window = M * I~ = conj(val) (-1)^(u+v) Nx Ny at (v mod wy, u mod wx)
            const int u = -(P.k0 + j), v = -(P.ky0 + i);
            int qu = u % A.wx;
            if (qu < 0) qu += A.wx;
            const float sg = ((u + v) & 1) ? -A.nxny : A.nxny;
            win[(size_t)q * A.wx + qu] = make_float2(sg * val.x, -sg * val.y);
          }
        }
      }
    }
    z[it] = val;
  }
  __syncthreads();
#pragma unroll
  for (int it = 0; it < NE; ++it) {
    const int e = tid + it * kTPB;
    if (e < CG * WY) buf[(e / WY) * ST + LW::at(e % WY)] = z[it];
  }
  __syncthreads();
  if constexpr (TWG)
    fft_lds<WY, CG, ST, kTPB>(buf, as_global(A.tw_wy), tid);
  else
    fft_lds<WY, CG, ST, kTPB>(buf, static_cast<const float2*>(tww), tid);
  float2* out = A.f2 + ((size_t)(bl * A.npol + p) * WY) * A.bxp;
  constexpr int NO = (CG * WY + kTPB - 1) / kTPB;
  float2 ov[NO];
#pragma unroll
  for (int it = 0; it < NO; ++it) {
    const int e = tid + it * kTPB;
    const int c = e % CG, l = e / CG;
    if ((CG * WY) % kTPB == 0 || e < CG * WY) ov[it] = buf[c * ST + LW::at(l)];
  }
#pragma unroll
  for (int it = 0; it < NO; ++it) {
    const int e = tid + it * kTPB;
    const int c = e % CG, l = e / CG;
    const int j = jc0 + c;
    if (((CG * WY) % kTPB == 0 || e < CG * WY) && j < A.bx) st_nt(out + (size_t)l * A.bxp + j, conjf2(ov[it]));
  }
}

// ---------------------------------------------------------------------------
// k_cspec (spectral path): grid (ceil(bx / CG), npol, nb). The column FFT as
// in k_col, then the block's masked window contracted with the folded tables
// (PolTab::xs, ys):
//   Q[j][n] = sum_i mask(j, i) conj(S[j][i]) ys[i][n]   FP32 MFMA, K = box rows
//   c[m][n] = sum_j xs[j][m] Q[j][n]                    this block's share
// MFMA operands (16x16x4): A row r = part CG + j (part 0: Re S, 1: Im S) in
// tiles of 16 rows, column k = box row i = 4 s + k of step s; the steps go to
// the four waves round robin. B = Re ys and Im ys of the same rows. With
// S = a + ib and ys = c + id, conj(S) ys = (ac + bd) + i(ad - bc).
// The block's field power follows from Parseval: sum |E|^2 = wx wy sum |S|^2 / (Nx Ny)^2.
// NT mode tiles of 16 are contracted at a time. MC: the plan has more mode
// tiles (gp > 16 NT, up to kMaxGp); the contraction then runs once per chunk
// of NT tiles over the same window in LDS, each chunk's Q columns collected in
// LDS before the final product (tables of gp columns; MC = false: gp = 16 NT).
// ROT (swizzled layouts): the column FFT's last pass writes the bins in plain
// order rotated so that window row i (bin ky0 + i) sits at slot B + i, B < the
// last pass's block; the A operands are then read at fixed offsets per step,
// each lane reading its own real or imaginary part, and a transform stride of
// 2 mod 16 puts the 32 lanes of a read in distinct banks.
// NWV waves per workgroup; each MFMA step takes 4 box rows per wave, so the
// window rows are padded to a multiple of 4 NWV (the ys table has a multiple
// of 32 rows, zero past the box, so either width reads inside it).
template <int NY, int WY, int CG, int NT, bool MC, int NWV = 4>
struct CspecShape {
  static_assert(NWV == 4 || NWV == 8, "four or eight waves");
  static constexpr int TPB = 64 * NWV;
  static constexpr int RS = 4 * NWV;                      // box rows per round of steps
  static constexpr int WYP = (WY + RS - 1) / RS * RS;
  static constexpr bool ROT = Lds<NY>::SWZ && last_ns<NY>() + WYP <= NY;
  static constexpr int ST = ROT ? NY + 2 : Lds<NY>::STRIDE;
  static constexpr int MT = (2 * CG + 15) / 16;          // A-row tiles
  static constexpr int KSW = WYP / RS;                    // K steps per wave
  static constexpr int GP = 16 * NT;                      // mode columns per chunk
  static constexpr int GPM = MC ? kMaxGp : GP;            // mode columns held in LDS, at most
  static constexpr int NRED = NWV * MT * NT * 2 * 256;    // floats: the waves' MFMA results
  static constexpr int NQ = CG * GP;                      // float2: one chunk of Q
  // with several chunks the window stays in buf until the last one
  static constexpr bool IN_BUF = !MC && NRED * 4 + NQ * 8 <= CG * ST * 8;
  // From 1024 rows on, the twiddles are read through the caches instead of LDS
  // wherever that lets one more workgroup onto a CU (160 KB of LDS each); at
  // 512 rows the extra workgroup measured slower than the LDS reads it saves.
  static constexpr int LDS_REST =
      CG * ST * 8 + WYP * 8 + CG * GPM * 8 + 16 + (IN_BUF ? 8 : (NRED / 2 + CG * GPM) * 8);
  static constexpr int LDS_CU = 160 * 1024;
  static constexpr bool TWG = NY >= 1024 && LDS_CU / LDS_REST > LDS_CU / (LDS_REST + twn<NY>() * 8);
  // LDS of the pass, float2 (int2 for the mask rows, float for the powers)
  static constexpr int BUF = CG * ST, TWY = TWG ? 1 : twn<NY>(), MROW = WYP, SX = CG * GPM;
  static constexpr int SPILL = IN_BUF ? 1 : (NRED / 2 + CG * GPM);
  // workgroups per CU that the LDS allows
  static constexpr int WG_PER_CU = LDS_CU / ((BUF + TWY + MROW + SX + SPILL) * 8 + 16);
};

// The spectral column pass of box-column block cb of frame bl (within the
// launch, frames from b0), pol p, from `in` (that frame and pol's t1; loads
// with cache policy T1AUX); LDS arrays of CspecShape's sizes.
template <int NY, int WY, int CG, int NT, bool MC, int T1AUX, int NWV = 4>
__device__ __forceinline__ void cspec_block(const KArgs& A, int b0, int cb, int p, int bl, const float2* in,
                                            float2* buf, float2* twy, int2* s_mrow, float2* s_x, float* s_pw,
                                            float2* s_spill, int tid) {
  using SH = CspecShape<NY, WY, CG, NT, MC, NWV>;
  using LN = Lds<NY>;
  constexpr int TPB = SH::TPB, RS = SH::RS;
  using Q = Pass1<NY, CG, TPB>;
  constexpr int ST = SH::ST, MT = SH::MT, WYP = SH::WYP, KSW = SH::KSW, GP = SH::GP, GPM = SH::GPM;
  constexpr int NRED = SH::NRED, NQ = SH::NQ;
  constexpr bool IN_BUF = SH::IN_BUF, TWG = SH::TWG, ROT = SH::ROT;
  static_assert(!ROT || MT == 1, "rotated reads take one A-row tile");
  static_assert(KSW * NT <= 96, "B operands are held in registers");
  const int lane = tid & 63, wv = tid >> 6;
  const PolTab& P = A.pol[p];
  const int jc0 = cb * CG;
  const int gpt = MC ? A.gp : GP;                  // table row stride (mode columns)
  const int nch = MC ? gpt / GP : 1;               // chunks of NT mode tiles
  // tables first: their loads are in flight with the column loads
  Staged<float2, TWG ? 1 : twn<NY>(), TPB> stwy;
  Staged<int2, WYP, TPB> smr;
  Staged<float2, CG * GPM, TPB> sx;
  if constexpr (!TWG) stwy.load(A.tw_ny, twn<NY>(), tid);
  smr.load(P.mrow, A.by, tid);
  const int ncx = A.bx - jc0 < CG ? A.bx - jc0 : CG;
  sx.load(P.xs + (size_t)jc0 * gpt, ncx * gpt, tid);
  // this wave's B operands: steps s = wv + NWV t, box rows i = 4 s + lane / 16;
  // the ys table has at least WYP rows, zero from row by on.
  // The first DB steps' operands are loaded before the column FFT, the rest
  // DB steps ahead of their use (DB = KSW where they all fit in registers)
  // (up to 48 steps x tiles held where the LDS already limits a SIMD to two
  // waves, so the registers are there)
  constexpr int DB = KSW * NT <= (SH::WG_PER_CU * NWV / 4 <= 2 ? 48 : 24) ? KSW : 12 / NT;
  float bre[KSW][NT], bim[KSW][NT];
  const float2* yrow = P.ys + (4 * wv + (lane >> 4)) * gpt + (lane & 15);
#pragma unroll
  for (int t = 0; t < DB; ++t)
#pragma unroll
    for (int nt = 0; nt < NT; ++nt) {
      const float2 y = yrow[t * RS * gpt + nt * 16];
      bre[t][nt] = y.x;
      bim[t][nt] = y.y;
    }
  {
    float2 v[Q::IT][Q::R0];
    // element (j, b + r NB) of the tiled t1 at byte t1_at * 8; where NB is a
    // multiple of 16 the row tile advances by NB / 16 per r at a fixed offset
    // within the tile, and that step goes in the scalar offset
    const __amdgpu_buffer_rsrc_t rt = make_rsrc(in, (unsigned)(A.bx * NY * 8));
#pragma unroll
    for (int it = 0; it < Q::IT; ++it) {
      const int g = tid + it * TPB;
      const int c = g / Q::NB, b = g % Q::NB;
      const int j = (Q::TOTAL % TPB == 0 || g < Q::TOTAL) && jc0 + c < A.bx ? jc0 + c : 0;
      if constexpr (Q::NB % 16 == 0) {
        const int voff = ((b >> 4) * A.bx + j) * 128 + (b & 15) * 8;
        const int rstride = (Q::NB / 16) * A.bx * 128;
#pragma unroll
        for (int r = 0; r < Q::R0; ++r) v[it][r] = buf_ld_aux<T1AUX>(rt, voff, r * rstride);
      } else {
#pragma unroll
        for (int r = 0; r < Q::R0; ++r) v[it][r] = buf_ld_aux<T1AUX>(rt, (int)t1_at(j, b + r * Q::NB, A.bx) * 8, 0);
      }
    }
    if constexpr (!TWG) stwy.store(twy, twn<NY>(), make_float2(0.f, 0.f), tid);
    smr.store(s_mrow, A.by, make_int2(1, 0), tid);
    sx.store(s_x, ncx * gpt, make_float2(0.f, 0.f), tid);
    fft_pass1_regs<NY, CG, ST, TPB>(v, buf, tid);
  }
  // window row i is bin (ky0 + i) mod NY; with ROT at slot rb + i
  int kyn = P.ky0 % NY;
  if (kyn < 0) kyn += NY;
  const int rrot = kyn / last_ns<NY>(), rb = kyn - rrot * last_ns<NY>();
  if constexpr (ROT) {
    if constexpr (TWG)
      fft_rest_rot<NY, CG, ST, TPB>(buf, as_global(A.tw_ny), tid, rrot);
    else
      fft_rest_rot<NY, CG, ST, TPB>(buf, static_cast<const float2*>(twy), tid, rrot);
  } else {
    if constexpr (TWG)
      fft_rest<NY, CG, ST, TPB>(buf, as_global(A.tw_ny), tid);
    else
      fft_rest<NY, CG, ST, TPB>(buf, static_cast<const float2*>(twy), tid);
  }
  if (A.window) {
    // window = M * I~ = conj(val) (-1)^(u+v) Nx Ny at (v mod wy, u mod wx), as in k_col
    float2* win = A.window + ((size_t)(b0 + bl) * A.npol + p) * A.wy * A.wx;
    // the block's columns fastest across the threads: neighbouring box columns
    // are neighbouring cells of one window row (CG cells per row and lane group)
    for (int e = tid; e < CG * WY; e += TPB) {
      const int c = e % CG, q = e / CG;
      const int j = jc0 + c;
      const int i = box_of(-P.ky0, q, WY, P.byq);
      if (i < 0 || j >= A.bx) continue;
      const int2 mr = s_mrow[i];
      if (j < mr.x || j > mr.y) continue;
      int vv = (P.ky0 + i) % NY;
      if (vv < 0) vv += NY;
      const float2 val = cmul(cmul(buf[c * ST + (ROT ? rb + i : LN::at(vv))], conjf2(P.rhox[j])), conjf2(P.rhoy[i]));
      const int u = -(P.k0 + j), v = -(P.ky0 + i);
      int qu = u % A.wx;
      if (qu < 0) qu += A.wx;
      const float sg = ((u + v) & 1) ? -A.nxny : A.nxny;
      win[(size_t)q * A.wx + qu] = make_float2(sg * val.x, -sg * val.y);
    }
  }
  float pw = 0.f;
  float* red = IN_BUF ? reinterpret_cast<float*>(buf) : reinterpret_cast<float*>(s_spill);
  float2* s_q = reinterpret_cast<float2*>(red + NRED);
  for (int ch = 0; ch < nch; ++ch) {
    if (ch > 0) {
      // the next chunk's first B operands (chunk 0's were loaded before the FFT)
#pragma unroll
      for (int t = 0; t < DB; ++t)
#pragma unroll
        for (int nt = 0; nt < NT; ++nt) {
          const float2 y = yrow[t * RS * gpt + ch * GP + nt * 16];
          bre[t][nt] = y.x;
          bim[t][nt] = y.y;
        }
    }
    floatx4 d1[MT][NT], d2[MT][NT];
#pragma unroll
    for (int mt = 0; mt < MT; ++mt)
#pragma unroll
      for (int nt = 0; nt < NT; ++nt) {
        d1[mt][nt] = floatx4{0.f, 0.f, 0.f, 0.f};
        d2[mt][nt] = floatx4{0.f, 0.f, 0.f, 0.f};
      }
    {
      // the A operands (mask interval and spectrum value of each step) are read
      // DA steps ahead of their MFMAs (all of them first where they fit in
      // registers); every address is valid: rows past the box have empty mask
      // intervals and zero B operands. The mask is applied as a select.
      constexpr int DA = KSW <= 16 ? KSW : 12;
      int2 mv[KSW];
      float2 fv[KSW][MT];
      float fr[KSW];                                // ROT: this lane's part of the step's value
      int i = 4 * wv + (lane >> 4);                 // box row of the next step to read
      int vv = (P.ky0 + i) % NY;                    // its column-FFT bin
      if (vv < 0) vv += NY;
      // ROT: float index of (column, part) at window row i; a step moves 16 rows
      const float* bfl = reinterpret_cast<const float*>(buf) +
                         2 * (((lane & 15) % CG) * ST + rb + i) + (((lane & 15) / CG) & 1);
#pragma unroll
      for (int t = 0; t < KSW + DA; ++t) {
        if (t < KSW) {                              // read step t (compile-time after unrolling)
          mv[t] = s_mrow[i];                        // i < 16 KSW = WYP
          if constexpr (ROT) {
            fr[t] = bfl[2 * RS * t];
          } else {
#pragma unroll
            for (int mt = 0; mt < MT; ++mt) fv[t][mt] = buf[((mt * 16 + (lane & 15)) % CG) * ST + LN::at(vv)];
          }
          i += RS;
          vv += RS;
          if (vv >= NY) vv -= NY;
        }
        const int u = t - DA;                       // step whose MFMAs run now
        if (u >= 0) {
          if (u + DB < KSW) {
#pragma unroll
            for (int nt = 0; nt < NT; ++nt) {
              const float2 y = yrow[(u + DB) * RS * gpt + ch * GP + nt * 16];
              bre[u + DB][nt] = y.x;
              bim[u + DB][nt] = y.y;
            }
          }
#pragma unroll
          for (int mt = 0; mt < MT; ++mt) {
            const int r = mt * 16 + (lane & 15);
            const int part = r / CG;
            const int ja = jc0 + r % CG;
            const bool ok = part < 2 && ja >= mv[u].x && ja <= mv[u].y;
            float a;
            if constexpr (ROT)
              a = ok ? fr[u] : 0.f;
            else
              a = ok ? (part ? fv[u][mt].y : fv[u][mt].x) : 0.f;
            if (ch == 0) pw = fmaf(a, a, pw);
#pragma unroll
            for (int nt = 0; nt < NT; ++nt) {
              d1[mt][nt] = __builtin_amdgcn_mfma_f32_16x16x4f32(a, bre[u][nt], d1[mt][nt], 0, 0, 0);
              d2[mt][nt] = __builtin_amdgcn_mfma_f32_16x16x4f32(a, bim[u][nt], d2[mt][nt], 0, 0, 0);
            }
          }
        }
      }
    }
    __syncthreads();                              // every wave is done with buf (and the last chunk's red)
    // red[(((w MT + mt) NT + nt) 2 + h) 256 + row 16 + n], h = 0: d1, 1: d2
#pragma unroll
    for (int mt = 0; mt < MT; ++mt)
#pragma unroll
      for (int nt = 0; nt < NT; ++nt)
#pragma unroll
        for (int r = 0; r < 4; ++r) {
          const int el = (4 * (lane >> 4) + r) * 16 + (lane & 15);
          red[(((wv * MT + mt) * NT + nt) * 2 + 0) * 256 + el] = d1[mt][nt][r];
          red[(((wv * MT + mt) * NT + nt) * 2 + 1) * 256 + el] = d2[mt][nt][r];
        }
    if (ch == 0) {
#pragma unroll
      for (int off = 32; off > 0; off >>= 1) pw += __shfl_xor(pw, off, 64);
      if (lane == 0) s_pw[wv] = pw;
    }
    __syncthreads();
    // Q[j][ch GP + n], the waves summed in order
    for (int e = tid; e < NQ; e += TPB) {
      const int j = e / GP, n = e % GP;
      const int nt = n >> 4, nn = n & 15;
      const int r0 = j, r1 = CG + j;              // rows of Re S and Im S
      float qr = 0.f, qi = 0.f;
#pragma unroll
      for (int w = 0; w < NWV; ++w) {
        const float* b0r = red + (((w * MT + (r0 >> 4)) * NT + nt) * 2) * 256 + (r0 & 15) * 16 + nn;
        const float* b1r = red + (((w * MT + (r1 >> 4)) * NT + nt) * 2) * 256 + (r1 & 15) * 16 + nn;
        qr += b0r[0] + b1r[256];                  // a c + b d
        qi += b0r[256] - b1r[0];                  // a d - b c
      }
      s_q[j * gpt + ch * GP + n] = make_float2(qr, qi);
    }
    __syncthreads();
  }
  const int pstride = A.nmodes + 1;
  float2* part = A.partial + ((size_t)(bl * A.nblk + cb) * A.npol + p) * pstride;
  if (tid == 0) {
    float pwt = 0.f;
#pragma unroll
    for (int w = 0; w < NWV; ++w) pwt += s_pw[w];
    part[A.nmodes] = make_float2(A.capt ? pwt * A.spow : 0.f, 0.f);
  }
  for (int e = tid; e < A.nmodes; e += TPB) {
    const short2 mn = A.modes[e];
    float2 acc = make_float2(0.f, 0.f);
#pragma unroll
    for (int j = 0; j < CG; ++j) acc = cadd(acc, cmul(s_x[j * gpt + mn.x], s_q[j * gpt + mn.y]));
    part[e] = acc;
  }
}

template <int NY, int WY, int CG, int NT, bool MC, int NWV>
__global__ void __launch_bounds__(64 * NWV) k_cspec(KArgs A, int b0) {
  using SH = CspecShape<NY, WY, CG, NT, MC, NWV>;
  __shared__ float2 buf[SH::BUF];
  __shared__ float2 twy[SH::TWY];
  __shared__ int2 s_mrow[SH::MROW];
  __shared__ float2 s_x[SH::SX];                 // xs rows of the block's columns
  __shared__ float s_pw[NWV];
  __shared__ float2 s_spill[SH::SPILL];
  const int p = blockIdx.y, bl = blockIdx.z;
  const float2* in = A.t1 + ((size_t)(bl * A.npol + p) * A.bx) * NY;
  cspec_block<NY, WY, CG, NT, MC, kT1Nt ? 2 : 0, NWV>(A, b0, blockIdx.x, p, bl, in, buf, twy, s_mrow, s_x, s_pw,
                                                      s_spill, threadIdx.x);
}

// ---------------------------------------------------------------------------
// Alignment: the spectrum around the cross term is computed once per batch
// and kept; every trial of tilt / defocus / waist re-runs only the window
// gather, the IFFTs and the overlap from it.
//
// k_spec: grid (ceil(bx / CG), npol, nb): FFT along y of CG columns of the
// (extended) row-pass result, rows v' = ky0 + i (mod NY), i < nrow, stored
// to spec[b][p][j][i].
template <int NY, int CG>
__global__ void __launch_bounds__(kTPB) k_spec(KArgs A, float2* __restrict__ spec, int nrow) {
  using LN = Lds<NY>;
  using Q = Pass1<NY, CG, kTPB>;
  constexpr int ST = LN::STRIDE;
  __shared__ float2 buf[CG * ST];
  const int tid = threadIdx.x;
  const int p = blockIdx.y;
  const int bl = blockIdx.z;
  const PolTab& P = A.pol[p];
  const int jc0 = blockIdx.x * CG;
  const float2* in = A.t1 + ((size_t)(bl * A.npol + p) * A.bx) * NY;
  {
    float2 v[Q::IT][Q::R0];
#pragma unroll
    for (int it = 0; it < Q::IT; ++it) {
      const int g = tid + it * kTPB;
      const int c = g / Q::NB, b = g % Q::NB;
      const int j = jc0 + c;
      const bool ok = (Q::TOTAL % kTPB == 0 || g < Q::TOTAL) && j < A.bx;
#pragma unroll
      for (int r = 0; r < Q::R0; ++r) v[it][r] = ok ? in[t1_at(j, b + r * Q::NB, A.bx)] : make_float2(0.f, 0.f);
    }
    fft_pass1_regs<NY, CG, ST, kTPB>(v, buf, tid);
  }
  fft_rest<NY, CG, ST, kTPB>(buf, A.tw_ny, tid);
  for (int c = 0; c < CG; ++c) {
    const int j = jc0 + c;
    if (j >= A.bx) break;
    float2* o = spec + ((size_t)(bl * A.npol + p) * A.bx + j) * nrow;
    for (int i = tid; i < nrow; i += kTPB) {
      int vv = (P.ky0 + i) % NY;
      if (vv < 0) vv += NY;
      o[i] = buf[c * ST + LN::at(vv)];
    }
  }
}

// k_gather: grid (ceil(bx / CG), npol, nb): the window of the current plan
// gathered from the stored spectrum (box column j, row i of pol p at spectrum
// column offj[p] + j, row offi[p] + i), then the IFFT along y, as in k_col.
struct SpecRef {
  const float2* spec;
  int bxe, nrow;
  int offj[2], offi[2];
};

template <int WY, int CG>
__global__ void __launch_bounds__(kTPB) k_gather(KArgs A, SpecRef S) {
  using LW = Lds<WY>;
  constexpr int ST = LW::STRIDE;
  __shared__ float2 buf[CG * ST];
  const int tid = threadIdx.x;
  const int p = blockIdx.y;
  const int bl = blockIdx.z;
  const PolTab& P = A.pol[p];
  const int jc0 = blockIdx.x * CG;
  const float2* sp = S.spec + (size_t)(bl * A.npol + p) * S.bxe * S.nrow;
  for (int e = tid; e < CG * WY; e += kTPB) {
    const int c = e / WY, q = e % WY;
    const int j = jc0 + c;
    const int i = box_of(-P.ky0, q, WY, P.byq);
    float2 val = make_float2(0.f, 0.f);
    if (i >= 0 && j < A.bx) {
      const int2 mr = P.mrow[i];
      if (j >= mr.x && j <= mr.y) {
        const float2 f = sp[(size_t)(S.offj[p] + j) * S.nrow + S.offi[p] + i];
        val = cmul(f, conjf2(cmul(P.rhox[j], P.rhoy[i])));
      }
    }
    buf[c * ST + LW::at(q)] = val;
  }
  __syncthreads();
  fft_lds<WY, CG, ST, kTPB>(buf, A.tw_wy, tid);
  float2* out = A.f2 + ((size_t)(bl * A.npol + p) * WY) * A.bxp;
  for (int e = tid; e < CG * WY; e += kTPB) {
    const int c = e % CG, l = e / CG;
    const int j = jc0 + c;
    if (j < A.bx) st_nt(out + (size_t)l * A.bxp + j, conjf2(buf[c * ST + LW::at(l)]));
  }
}

// ---------------------------------------------------------------------------
// k_fld: grid (nblk, npol, nb); one block of 16 field rows per workgroup,
// 4 waves: x-IFFT of the 16 rows, tilt/defocus removal, then the separable
// HG overlap as two real MFMA contractions: T = E Ux over this wave's share
// of x, then C = Uy^T T with T taken straight from the accumulators. The four
// waves' partial C tiles are summed in LDS, in wave order.
//   PREC 0: FP32 MFMA 16x16x4.
//   PREC 1/2: split BF16 / FP16 MFMA 16x16x16, x = hi + lo for both operands,
//   products hi*hi + hi*lo + lo*hi accumulated in FP32. FP16 operands carry
//   power-of-two prescales (field: block max; T: wave max; tables: static)
//   that are divided out exactly.
template <int PREC>
struct Split4 {
  shortx4 bh, bl;
  halfx4 hh, hl;
};

template <int PREC>
__device__ __forceinline__ void split4(const float* v, float s, Split4<PREC>& o) {
#pragma unroll
  for (int j = 0; j < 4; ++j) {
    if constexpr (PREC == 1) {
      const unsigned short h = bf16_rne(v[j]);
      o.bh[j] = (short)h;
      o.bl[j] = (short)bf16_rne(v[j] - bf16_to_f32(h));
    } else {
      const float x = v[j] * s;
      const _Float16 h = (_Float16)x;
      o.hh[j] = h;
      o.hl[j] = (_Float16)(x - (float)h);
    }
  }
}

template <int PREC>
__device__ __forceinline__ floatx4 mfma3(const Split4<PREC>& a, const Split4<PREC>& b, floatx4 c) {
  if constexpr (PREC == 1) {
    c = __builtin_amdgcn_mfma_f32_16x16x16bf16_1k(a.bh, b.bh, c, 0, 0, 0);
    c = __builtin_amdgcn_mfma_f32_16x16x16bf16_1k(a.bh, b.bl, c, 0, 0, 0);
    c = __builtin_amdgcn_mfma_f32_16x16x16bf16_1k(a.bl, b.bh, c, 0, 0, 0);
  } else {
    c = __builtin_amdgcn_mfma_f32_16x16x16f16(a.hh, b.hh, c, 0, 0, 0);
    c = __builtin_amdgcn_mfma_f32_16x16x16f16(a.hh, b.hl, c, 0, 0, 0);
    c = __builtin_amdgcn_mfma_f32_16x16x16f16(a.hl, b.hh, c, 0, 0, 0);
  }
  return c;
}

// four consecutive samples (k0..k0+3) of mode `mode` from a packed split table
template <int PREC>
__device__ __forceinline__ void table4(const unsigned short* bh, const unsigned short* bl, const _Float16* hh,
                                       const _Float16* hl, int k0, int gp, int mode, Split4<PREC>& o) {
  const size_t at = ((size_t)(k0 >> 2) * gp + mode) * 4;
  if constexpr (PREC == 1) {
    o.bh = *reinterpret_cast<const shortx4*>(bh + at);
    o.bl = *reinterpret_cast<const shortx4*>(bl + at);
  } else {
    o.hh = *reinterpret_cast<const halfx4*>(hh + at);
    o.hl = *reinterpret_cast<const halfx4*>(hl + at);
  }
}

__device__ __forceinline__ float wave_max(float v) {
#pragma unroll
  for (int off = 32; off > 0; off >>= 1) v = fmaxf(v, __shfl_xor(v, off, 64));
  return v;
}

// power of two s with max * s in [2^13, 2^14) (1 if max is 0)
__device__ __forceinline__ float fp16_prescale(float mx) {
  if (!(mx > 0.f)) return 1.f;
  int e;
  frexpf(mx, &e);            // mx = f 2^e, f in [0.5, 1)
  return ldexpf(1.f, 14 - e);
}

template <int WX, int MT, int PREC>
__global__ void __launch_bounds__(kTPB) k_fld(KArgs A, int b0) {
  using L = Lds<WX>;
  constexpr int ST = L::STRIDE;
  constexpr int NPAIR = (MT == 1) ? 1 : 3;        // (n-tile, m-tile) pairs that can hold m+n < 32
  __shared__ float2 buf[16 * ST];
  __shared__ float red[4][NPAIR][2][256];
  __shared__ float bmax[4];
  __shared__ float bpow[4];
  __shared__ float2 tww[twn<WX>()];
  __shared__ float2 s_tx[WX];
  const int tid = threadIdx.x;
  const int lane = tid & 63, wv = tid >> 6;
  const int rb = blockIdx.x;
  const int p = blockIdx.y;
  const int bl = blockIdx.z;
  const int bg = b0 + bl;
  const PolTab& P = A.pol[p];
  const float2* in = A.f2 + ((size_t)(bl * A.npol + p) * A.wy) * A.bxp;
  float2* fld = A.fields ? A.fields + ((size_t)bg * A.npol + p) * A.wy * WX : nullptr;
  const int gp = A.gp;
  // the FP32 path's HG operands, loaded before the IFFT so their latency hides
  constexpr int KSP = (PREC == 0 && (WX / 16) * MT <= 16) ? WX / 16 : 1;
  float ubp[MT][KSP];
  float uap[NPAIR][4];
  if constexpr (PREC == 0) {
    if constexpr ((WX / 16) * MT <= 16) {
#pragma unroll
      for (int s = 0; s < KSP; ++s)
#pragma unroll
        for (int mt = 0; mt < MT; ++mt)
          ubp[mt][s] = P.ux[(wv * (WX / 4) + 4 * s + (lane >> 4)) * gp + mt * 16 + (lane & 15)];
    }
#pragma unroll
    for (int q = 0; q < NPAIR; ++q)
#pragma unroll
      for (int r = 0; r < 4; ++r)
        uap[q][r] = P.uy[(rb * 16 + 4 * (lane >> 4) + r) * gp + ((q == 2) ? 16 : 0) + (lane & 15)];
  }
  static_assert(WX % 16 == 0 && kTPB == 256, "tilt pass: 16 rows x 16 lanes");
  Staged<float2, twn<WX>(), kTPB> stw;
  Staged<float2, WX, kTPB> stx;
  stw.load(A.tw_wx, twn<WX>(), tid);
  stx.load(P.tx, WX, tid);
  // tilt pass mapping: thread (row r_t, lane c_t) takes columns c_t + 16 k
  const int r_t = tid >> 4, c_t = tid & 15;
  const int y_t = rb * 16 + r_t;
  const bool yok = y_t < A.wy;
  const float2 tyr = P.ty[yok ? y_t : A.wy - 1];
  {
    // IFFT along x, first pass straight from f2: butterfly (row tr, b) takes
    // IFFT columns q = b + NB s, i.e. box columns j = (u_hi - q) mod WX,
    // conjugated (inverse transform as conj FFT conj)
    using Q = Pass1<WX, 16, kTPB>;
    float2 v[Q::IT][Q::R0];
    const int uhi = -P.k0;
#pragma unroll
    for (int it = 0; it < Q::IT; ++it) {
      const int g = tid + it * kTPB;
      if (Q::TOTAL % kTPB == 0 || g < Q::TOTAL) {
        const int tr = g / Q::NB, b = g % Q::NB;
        const int y = rb * 16 + tr;
        const bool rok = y < A.wy;
        const float2* row = in + (size_t)(rok ? y : 0) * A.bxp;
        int j = (uhi - b) % WX;
        if (j < 0) j += WX;
#pragma unroll
        for (int s2 = 0; s2 < Q::R0; ++s2) {
          const bool ok = rok && j < P.bxq;
          const float2 f = ld_nt(row + (ok ? j : 0));
          v[it][s2] = ok ? conjf2(f) : make_float2(0.f, 0.f);
          j -= Q::NB;
          if (j < 0) j += WX;
        }
      }
    }
    stw.store(tww, twn<WX>(), make_float2(0.f, 0.f), tid);
    stx.store(s_tx, WX, make_float2(0.f, 0.f), tid);
    fft_pass1_regs<WX, 16, ST, kTPB>(v, buf, tid);
  }
  fft_rest<WX, 16, ST, kTPB>(buf, tww, tid);
  float emax = 0.f, pw = 0.f;
  {
    float2* brow = buf + r_t * ST;
#pragma unroll
    for (int k = 0; k < WX / 16; ++k) {
      const int q = c_t + 16 * k;
      float2 ev = make_float2(0.f, 0.f);
      if (yok) {
        ev = cmul(cmul(conjf2(brow[L::at(q)]), s_tx[q]), tyr);
        if (fld) fld[(size_t)y_t * WX + q] = ev;
      }
      brow[L::at(q)] = ev;
      if constexpr (PREC == 2) emax = fmaxf(emax, fmaxf(fabsf(ev.x), fabsf(ev.y)));
      pw = fmaf(ev.x, ev.x, fmaf(ev.y, ev.y, pw));   // field power of the block (FP32)
    }
  }
  float sE = 1.f;
  if constexpr (PREC == 2) {
    emax = wave_max(emax);
    if (lane == 0) bmax[wv] = emax;
  }
  if (A.capt) {
#pragma unroll
    for (int off = 32; off > 0; off >>= 1) pw += __shfl_xor(pw, off, 64);
    if (lane == 0) bpow[wv] = pw;
  }
  __syncthreads();
  if constexpr (PREC == 2) sE = fp16_prescale(fmaxf(fmaxf(bmax[0], bmax[1]), fmaxf(bmax[2], bmax[3])));
  floatx4 tre[MT], tim[MT];
#pragma unroll
  for (int mt = 0; mt < MT; ++mt) {
    tre[mt] = floatx4{0.f, 0.f, 0.f, 0.f};
    tim[mt] = floatx4{0.f, 0.f, 0.f, 0.f};
  }
  if constexpr (PREC == 0) {
    // T[y][m] = sum_x E[y][x] Ux[x][m] over this wave's quarter of x
    constexpr int XS = WX / 4;    // x columns per wave
    constexpr int KS = XS / 4;    // k-steps of 4
    if constexpr (KS * MT <= 16) {
#pragma unroll
      for (int s = 0; s < KS; ++s) {
        const int x = wv * XS + 4 * s + (lane >> 4);
        const float2 ev = buf[(lane & 15) * ST + L::at(x)];
#pragma unroll
        for (int mt = 0; mt < MT; ++mt) {
          tre[mt] = __builtin_amdgcn_mfma_f32_16x16x4f32(ev.x, ubp[mt][s], tre[mt], 0, 0, 0);
          tim[mt] = __builtin_amdgcn_mfma_f32_16x16x4f32(ev.y, ubp[mt][s], tim[mt], 0, 0, 0);
        }
      }
    } else {
#pragma unroll 4
      for (int s = 0; s < KS; ++s) {
        const int x = wv * XS + 4 * s + (lane >> 4);
        const float2 ev = buf[(lane & 15) * ST + L::at(x)];
#pragma unroll
        for (int mt = 0; mt < MT; ++mt) {
          const float ub = P.ux[x * gp + mt * 16 + (lane & 15)];
          tre[mt] = __builtin_amdgcn_mfma_f32_16x16x4f32(ev.x, ub, tre[mt], 0, 0, 0);
          tim[mt] = __builtin_amdgcn_mfma_f32_16x16x4f32(ev.y, ub, tim[mt], 0, 0, 0);
        }
      }
    }
  } else {
    // k-steps of 16 x values, dealt to the waves round robin; lane holds
    // x = 16 s + 4 (lane/16) + j, j = 0..3 of row lane%16
    constexpr int KT = WX / 16;
    for (int s = wv; s < KT; s += 4) {
      const int x0 = 16 * s + 4 * (lane >> 4);
      float re[4], im[4];
#pragma unroll
      for (int j = 0; j < 4; ++j) {
        const float2 ev = buf[(lane & 15) * ST + L::at(x0 + j)];
        re[j] = ev.x;
        im[j] = ev.y;
      }
      Split4<PREC> ar, ai;
      split4<PREC>(re, sE, ar);
      split4<PREC>(im, sE, ai);
#pragma unroll
      for (int mt = 0; mt < MT; ++mt) {
        Split4<PREC> u;
        table4<PREC>(P.ux_bh, P.ux_bl, P.ux_hh, P.ux_hl, x0, gp, mt * 16 + (lane & 15), u);
        tre[mt] = mfma3<PREC>(ar, u, tre[mt]);
        tim[mt] = mfma3<PREC>(ai, u, tim[mt]);
      }
    }
  }
  // C[n][m] = sum_y Uy[y][n] T[y][m]; lane holds y = rb*16 + 4*(lane/16) + r
  floatx4 cre[NPAIR], cim[NPAIR];
#pragma unroll
  for (int q = 0; q < NPAIR; ++q) {
    cre[q] = floatx4{0.f, 0.f, 0.f, 0.f};
    cim[q] = floatx4{0.f, 0.f, 0.f, 0.f};
  }
  float unscale = 1.f;
  if constexpr (PREC == 0) {
#pragma unroll
    for (int r = 0; r < 4; ++r) {
#pragma unroll
      for (int q = 0; q < NPAIR; ++q) {
        const int mt = (q == 1) ? 1 : 0;
        cre[q] = __builtin_amdgcn_mfma_f32_16x16x4f32(uap[q][r], tre[mt][r], cre[q], 0, 0, 0);
        cim[q] = __builtin_amdgcn_mfma_f32_16x16x4f32(uap[q][r], tim[mt][r], cim[q], 0, 0, 0);
      }
    }
  } else {
    float sT = 1.f;
    if constexpr (PREC == 2) {
      float tm = 0.f;
#pragma unroll
      for (int mt = 0; mt < MT; ++mt)
#pragma unroll
        for (int r = 0; r < 4; ++r) tm = fmaxf(tm, fmaxf(fabsf(tre[mt][r]), fabsf(tim[mt][r])));
      sT = fp16_prescale(wave_max(tm));
      unscale = 1.f / (sE * A.s_uh * sT * A.s_uh);   // exact: powers of two
    }
    const int y0 = rb * 16 + 4 * (lane >> 4);
    Split4<PREC> br[MT], bi[MT];
#pragma unroll
    for (int mt = 0; mt < MT; ++mt) {
      float vr[4] = {tre[mt][0], tre[mt][1], tre[mt][2], tre[mt][3]};
      float vi[4] = {tim[mt][0], tim[mt][1], tim[mt][2], tim[mt][3]};
      split4<PREC>(vr, sT, br[mt]);
      split4<PREC>(vi, sT, bi[mt]);
    }
#pragma unroll
    for (int q = 0; q < NPAIR; ++q) {
      const int nt = (q == 2) ? 1 : 0;
      const int mt = (q == 1) ? 1 : 0;
      Split4<PREC> u;
      table4<PREC>(P.uy_bh, P.uy_bl, P.uy_hh, P.uy_hl, y0, gp, nt * 16 + (lane & 15), u);
      cre[q] = mfma3<PREC>(u, br[mt], cre[q]);
      cim[q] = mfma3<PREC>(u, bi[mt], cim[q]);
    }
  }
#pragma unroll
  for (int q = 0; q < NPAIR; ++q) {
#pragma unroll
    for (int r = 0; r < 4; ++r) {
      const int n = 4 * (lane >> 4) + r, m = lane & 15;
      red[wv][q][0][n * 16 + m] = cre[q][r] * unscale;
      red[wv][q][1][n * 16 + m] = cim[q][r] * unscale;
    }
  }
  __syncthreads();
  // partial[bl][rb][p][mode]: this block's share of every coefficient, the
  // four waves summed in order
  const int pstride = A.nmodes + 1;
  float2* part = A.partial + ((size_t)(bl * A.nblk + rb) * A.npol + p) * pstride;
  if (tid == 0) part[A.nmodes] = make_float2(A.capt ? ((bpow[0] + bpow[1]) + bpow[2]) + bpow[3] : 0.f, 0.f);
  for (int i = tid; i < A.nmodes; i += kTPB) {
    const short2 mn = A.modes[i];
    const int m = mn.x, n = mn.y;
    const int q = (n >= 16) ? 2 : (m >= 16) ? 1 : 0;
    const int el = (n & 15) * 16 + (m & 15);
    part[i] = make_float2(((red[0][q][0][el] + red[1][q][0][el]) + red[2][q][0][el]) + red[3][q][0][el],
                          ((red[0][q][1][el] + red[1][q][1][el]) + red[2][q][1][el]) + red[3][q][1][el]);
  }
}

// ---------------------------------------------------------------------------
// k_norm: one workgroup per frame: coefficient (m, n) of pol p = the sum of
// the row-block partials in block order; then the FP64 power over both pols
// and the normalised coefficients.
__global__ void __launch_bounds__(kTPB) k_norm(KArgs A, int b0) {
  __shared__ double wsum[kTPB / 64];
  __shared__ double wpol[kTPB / 64][2];
  const int bl = blockIdx.x, tid = threadIdx.x;
  const int bg = b0 + bl;
  const int per = A.npol * A.nmodes;
  const int pstride = A.nmodes + 1;                 // partial: modes + the block's field power
  const int bstride = A.npol * pstride;
  float2* raw = A.coefs + (size_t)bg * per;
  const float2* part = A.partial + (size_t)bl * A.nblk * bstride;
  double s = 0.0, spol0 = 0.0, spol1 = 0.0;
  for (int i = tid; i < per; i += kTPB) {
    const int p = i / A.nmodes, md = i - p * A.nmodes;
    float re = 0.f, im = 0.f;
    // blocks summed in order, eight loads in flight at a time
    for (int rb0 = 0; rb0 < A.nblk; rb0 += 8) {
      float2 v[8];
#pragma unroll
      for (int u = 0; u < 8; ++u)
        v[u] = (rb0 + u < A.nblk) ? part[(size_t)(rb0 + u) * bstride + p * pstride + md] : make_float2(0.f, 0.f);
#pragma unroll
      for (int u = 0; u < 8; ++u) {
        re += v[u].x;
        im += v[u].y;
      }
    }
    raw[i] = make_float2(re, im);
    const double pw = (double)re * re + (double)im * im;
    s += pw;
    if (p == 0) spol0 += pw; else spol1 += pw;
  }
#pragma unroll
  for (int off = 32; off > 0; off >>= 1) {
    s += __shfl_xor(s, off, 64);
    spol0 += __shfl_xor(spol0, off, 64);
    spol1 += __shfl_xor(spol1, off, 64);
  }
  if ((tid & 63) == 0) {
    wsum[tid >> 6] = s;
    wpol[tid >> 6][0] = spol0;
    wpol[tid >> 6][1] = spol1;
  }
  __syncthreads();
  if (A.capt && tid < A.npol) {
    // captured power of pol tid: mode power and field power (blocks in order, FP64)
    double mp = 0.0, fp = 0.0;
    for (int w = 0; w < kTPB / 64; ++w) mp += wpol[w][tid];
    for (int rb = 0; rb < A.nblk; ++rb) fp += (double)part[(size_t)rb * bstride + tid * pstride + A.nmodes].x;
    A.capt[((size_t)bg * A.npol + tid) * 2 + 0] = mp;
    A.capt[((size_t)bg * A.npol + tid) * 2 + 1] = fp * A.cell;
  }
  double tot = 0.0;
#pragma unroll
  for (int w = 0; w < kTPB / 64; ++w) tot += wsum[w];
  const double inv = tot > 0.0 ? 1.0 / sqrt(tot) : 0.0;
  float2* o = A.coefs_norm + (size_t)bg * per;
  for (int i = tid; i < per; i += kTPB) {
    const float2 c = raw[i];
    o[i] = make_float2((float)(c.x * inv), (float)(c.y * inv));
  }
}

// ---------------------------------------------------------------------------
// k_hg: out[k][n] = u_n(x_k) * pitch, x_k = (k - w/2) pitch, by the normalised
// FP64 recurrence; optionally the split hi/lo tables from the same FP64 value.
__global__ void k_hg(double pitch, int w, int wpad, double waist, int G, int gp, float* __restrict__ out,
                     unsigned short* __restrict__ bh, unsigned short* __restrict__ bl, _Float16* __restrict__ hh,
                     _Float16* __restrict__ hl, double fp16_scale) {
  const int k = blockIdx.x * blockDim.x + threadIdx.x;
  if (k >= wpad) return;
  float* o = out + (size_t)k * gp;
  const double x = (k - 0.5 * w) * pitch;
  const double s = 1.4142135623730950488 * x / waist;
  const double scale = 1.1892071150027210667 / sqrt(waist) * pitch;   // 2^(1/4) w^(-1/2) p'
  double prev = 0.0;
  double cur = 0.75112554446494248286 * exp(-0.5 * s * s);             // pi^(-1/4)
  for (int n = 0; n < gp; ++n) {
    const double v = (k < w && n < G) ? cur * scale : 0.0;
    o[n] = (float)v;
    if (bh) {
      const size_t pk = ((size_t)(k >> 2) * gp + n) * 4 + (k & 3);
      const unsigned short b1 = bf16_rne((float)v);
      bh[pk] = b1;
      bl[pk] = bf16_rne((float)(v - (double)bf16_to_f32(b1)));
      const double vs = v * fp16_scale;
      const _Float16 h1 = (_Float16)vs;
      hh[pk] = h1;
      hl[pk] = (_Float16)(vs - (double)h1);
    }
    const double nxt = sqrt(2.0 / (n + 1)) * s * cur - sqrt((double)n / (n + 1)) * prev;
    prev = cur;
    cur = nxt;
  }
}

__global__ void k_zero(float2* p, size_t n) {
  size_t i = (size_t)blockIdx.x * blockDim.x + threadIdx.x;
  const size_t stride = (size_t)gridDim.x * blockDim.x;
  for (; i < n; i += stride) p[i] = make_float2(0.f, 0.f);
}

// ---------------------------------------------------------------------------
// dispatch over the supported sizes
// transforms per row-pass block and columns per column-pass block (~32-80 KB of LDS)
// row pass: TR transforms per block so that TR * N / R0 (the block size) is 256
// or 320; at N = 320, 8 transforms (160 threads, 22 KB of LDS: 7 blocks per CU)
// measured faster than 16 (320 threads, 3 blocks per CU). At N = 512 and
// 1024, 8 transforms (512 threads), so that a block writes whole 128 B t1
// tile lines (with 4 transforms: 0.726 -> 0.626 ms per 500 two-pol 1024x1024
// frames, 0.257 -> 0.243 ms per 256 one-pol 1024x1024 u16 frames). At
// N = 2048, 4 transforms (512 threads): each block then writes 64 B of every
// t1 tile line (2 transforms, 32 B pieces: 0.51 -> 0.30 ms per 64 frames with
// one tile)
template <int N> constexpr int row_tr() { return 256 / (N / FftPlan<N>::R0) > 0 ? (N == 320 ? 8 : N == 640 ? 4 : N == 2048 ? 4 : N == 512 ? 8 : N == 1024 ? 8 : 256 / (N / FftPlan<N>::R0)) : 1; }
template <int N> constexpr int col_cg() { return N >= 2048 ? 4 : N >= 1024 ? 4 : N >= 512 ? 8 : 16; }
// the spectral column pass: at 1024 rows with one mode tile 8 columns fit
// (1024-row camera: 0.253 -> 0.230 ms per 256 frames; with two mode tiles
// the larger workgroup costs occupancy and 4 stays faster)
// 8 columns per spectral workgroup at 1024 points (except with mode chunks,
// whose LDS would then allow one workgroup per CU): each workgroup reads the
// whole ys table (WY x gp) from L2, so fewer, wider workgroups read it less
// often (C5-shaped batch: 2.40 -> 2.31 ms per 1000 frames)
template <int N, int NT, bool MC = false> constexpr int cspec_cg() { return N == 1024 && !MC ? 8 : col_cg<N>(); }
// waves per spectral column workgroup: 8 from 1024 points, where the LDS
// leaves room for two workgroups per CU (16 waves instead of 8; C5-shaped
// batch 2.29 -> 2.20 ms per 1000 frames, the 1024^2 and 2048^2 cameras 3-4 %)
template <int N> constexpr int cspec_waves() { return N >= 1024 ? 8 : 4; }

template <int NX>
static hipError_t row_n(const KArgs& a, const void* frames, int u16, int b0, int nb, hipStream_t s) {
  constexpr int TR = row_tr<NX>();
  constexpr int TPB = TR * NX / FftPlan<NX>::R0;
  static_assert(TPB % 32 == 0 && TPB <= 512, "row-pass block size");
  // two row tiles per workgroup (the second tile's loads overlap the first
  // tile's transform) when that still leaves the chip well filled; one tile
  // for small batches, where latency matters more
  const int nyb = (a.ny + 2 * TR - 1) / (2 * TR);
  // one tile from 1024 points: the second tile's registers would cost a
  // workgroup per CU
  const bool two = NX < 1024 && (long)((nyb + 1) / 2) * a.npol * nb >= 4096;
  dim3 grid(two ? (nyb + 1) / 2 : nyb, a.npol, nb);
  if (u16) {
    if (two)
      hipLaunchKernelGGL((k_row<NX, TR, unsigned short, 2>), grid, dim3(TPB), 0, s, a, (const unsigned short*)frames, b0);
    else
      hipLaunchKernelGGL((k_row<NX, TR, unsigned short, 1>), grid, dim3(TPB), 0, s, a, (const unsigned short*)frames, b0);
  } else {
    if (two)
      hipLaunchKernelGGL((k_row<NX, TR, float, 2>), grid, dim3(TPB), 0, s, a, (const float*)frames, b0);
    else
      hipLaunchKernelGGL((k_row<NX, TR, float, 1>), grid, dim3(TPB), 0, s, a, (const float*)frames, b0);
  }
  return hipGetLastError();
}

template <int NY, int WY>
static hipError_t col_nw(const KArgs& a, int b0, int nb, hipStream_t s) {
  constexpr int CG = col_cg<NY>();
  dim3 grid((a.bx + CG - 1) / CG, a.npol, nb);
  hipLaunchKernelGGL((k_col<NY, WY, CG>), grid, dim3(kTPB), 0, s, a, b0);
  return hipGetLastError();
}

template <int WX, int MT>
static void fld_wm(const KArgs& a, dim3 grid, int b0, hipStream_t s) {
  if (a.prec == 1)
    hipLaunchKernelGGL((k_fld<WX, MT, 1>), grid, dim3(kTPB), 0, s, a, b0);
  else if (a.prec == 2)
    hipLaunchKernelGGL((k_fld<WX, MT, 2>), grid, dim3(kTPB), 0, s, a, b0);
  else
    hipLaunchKernelGGL((k_fld<WX, MT, 0>), grid, dim3(kTPB), 0, s, a, b0);
}

template <int WX>
static hipError_t fld_w(const KArgs& a, int b0, int nb, hipStream_t s) {
  dim3 grid(a.nblk, a.npol, nb);
  if (a.gp > kMaxGpField) return hipErrorInvalidValue;
  if (a.gp <= 16)
    fld_wm<WX, 1>(a, grid, b0, s);
  else
    fld_wm<WX, 2>(a, grid, b0, s);
  return hipGetLastError();
}

#define DH_FFT_SIZES(X) X(64) X(128) X(256) X(320) X(512) X(640) X(1024) X(2048)
#define DH_IFFT_SIZES(X) X(32) X(48) X(96) X(112) X(176) X(208) X(336) X(672)
// (FFT length, IFFT length) pairs along y: the window-radius rule at ratios up to 0.32
#define DH_COL_PAIRS(X) \
  X(64, 32) X(128, 32) X(128, 48) X(256, 48) X(256, 96) X(320, 96) X(320, 112) X(512, 96) X(512, 176) \
  X(640, 176) X(640, 208) X(1024, 176) X(1024, 336) X(2048, 336) X(2048, 672)

static bool fft_ok(int n) {
#define X(N) if (n == N) return true;
  DH_FFT_SIZES(X)
#undef X
  return false;
}
static bool ifft_ok(int n) {
#define X(N) if (n == N) return true;
  DH_IFFT_SIZES(X)
#undef X
  return false;
}
static bool pair_ok(int n, int w) {
#define X(N, W) if (n == N && w == W) return true;
  DH_COL_PAIRS(X)
#undef X
  return false;
}

void fft_radices(int n, int r[3]) {
  r[0] = r[1] = r[2] = 0;
#define X(N) if (n == N) { r[0] = FftPlan<N>::R0; r[1] = FftPlan<N>::R1; r[2] = FftPlan<N>::R2; return; }
  DH_FFT_SIZES(X)
  DH_IFFT_SIZES(X)
#undef X
}

bool sizes_supported(int nx, int ny, int wx, int wy) {
  return fft_ok(nx) && fft_ok(ny) && ifft_ok(wx) && ifft_ok(wy) && pair_ok(ny, wy);
}

bool fft_compiled(int n) { return fft_ok(n); }

hipError_t launch_row(const KArgs& a, const void* frames, int u16, int b0, int nb, hipStream_t s) {
  if (a.gx.np > 0) return launch_row_gen(a, frames, u16, b0, nb, s);
#define X(N) if (a.nx == N) return row_n<N>(a, frames, u16, b0, nb, s);
  DH_FFT_SIZES(X)
#undef X
  return hipErrorInvalidValue;
}
hipError_t launch_col(const KArgs& a, int b0, int nb, hipStream_t s) {
  if (a.gy.np > 0) return hipErrorInvalidValue;
#define X(N, W) if (a.ny == N && a.wy == W) return col_nw<N, W>(a, b0, nb, s);
  DH_COL_PAIRS(X)
#undef X
  return hipErrorInvalidValue;
}
template <int NY, int WY, int NT>
constexpr bool cspec_fits() { return ((WY + 15) / 16) * NT <= 96; }

// gp 16: one mode tile; 32: two; above: chunks of two tiles (gp a multiple of 32)
bool spectral_supported(int ny, int wy, int gp) {
  if (gp < 16 || gp > kMaxGp || (gp > 32 && gp % 32)) return false;
#define X(N, W) if (ny == N && wy == W) return gp == 16 ? cspec_fits<N, W, 1>() : cspec_fits<N, W, 2>();
  DH_COL_PAIRS(X)
#undef X
  return false;
}

int spectral_blocks(int ny, int wy, int bx, int gp) {
  if (!spectral_supported(ny, wy, gp)) {            // the generic column kernel's blocks
    const int cgg = gen_cols_per_block(ny, gp);
    return (bx + cgg - 1) / cgg;
  }
  int cg = 16;
#define X(N) if (ny == N) cg = gp == 16 ? cspec_cg<N, 1>() : gp == 32 ? cspec_cg<N, 2>() : cspec_cg<N, 2, true>();
  DH_FFT_SIZES(X)
#undef X
  return (bx + cg - 1) / cg;
}

template <int NY, int WY, int NT, bool MC>
static hipError_t cspec_nwt(const KArgs& a, int b0, int nb, hipStream_t s) {
  if constexpr (cspec_fits<NY, WY, NT>()) {
    constexpr int CG = cspec_cg<NY, NT, MC>();
    constexpr int NWV = cspec_waves<NY>();
    dim3 grid((a.bx + CG - 1) / CG, a.npol, nb);
    hipLaunchKernelGGL((k_cspec<NY, WY, CG, NT, MC, NWV>), grid, dim3(64 * NWV), 0, s, a, b0);
    return hipGetLastError();
  } else {
    return hipErrorInvalidValue;
  }
}

hipError_t launch_cspec(const KArgs& a, int b0, int nb, hipStream_t s) {
  if (a.gy.np > 0) return launch_cspec_gen(a, b0, nb, s);
  if (!spectral_supported(a.ny, a.wy, a.gp)) return hipErrorInvalidValue;
#define X(N, W)                                                                              \
  if (a.ny == N && a.wy == W)                                                                \
    return a.gp == 16 ? cspec_nwt<N, W, 1, false>(a, b0, nb, s)                              \
                      : a.gp == 32 ? cspec_nwt<N, W, 2, false>(a, b0, nb, s) : cspec_nwt<N, W, 2, true>(a, b0, nb, s);
  DH_COL_PAIRS(X)
#undef X
  return hipErrorInvalidValue;
}

hipError_t launch_fld(const KArgs& a, int b0, int nb, hipStream_t s) {
#define X(W) if (a.wx == W) return fld_w<W>(a, b0, nb, s);
  DH_IFFT_SIZES(X)
#undef X
  return hipErrorInvalidValue;
}
template <int NY>
static hipError_t spec_n(const KArgs& a, float2* spec, int nrow, int nb, hipStream_t s) {
  constexpr int CG = col_cg<NY>();
  dim3 grid((a.bx + CG - 1) / CG, a.npol, nb);
  hipLaunchKernelGGL((k_spec<NY, CG>), grid, dim3(kTPB), 0, s, a, spec, nrow);
  return hipGetLastError();
}

hipError_t launch_spec(const KArgs& a, float2* spec, int nrow, int nb, hipStream_t s) {
  if (a.gy.np > 0) return hipErrorInvalidValue;
#define X(N) if (a.ny == N) return spec_n<N>(a, spec, nrow, nb, s);
  DH_FFT_SIZES(X)
#undef X
  return hipErrorInvalidValue;
}

template <int WY>
static hipError_t gather_w(const KArgs& a, const float2* spec, int bxe, int nrow, const int* offj, const int* offi,
                           int nb, hipStream_t s) {
  constexpr int CG = 8;
  SpecRef r{spec, bxe, nrow, {offj[0], offj[1]}, {offi[0], offi[1]}};
  dim3 grid((a.bx + CG - 1) / CG, a.npol, nb);
  hipLaunchKernelGGL((k_gather<WY, CG>), grid, dim3(kTPB), 0, s, a, r);
  return hipGetLastError();
}

hipError_t launch_gather(const KArgs& a, const float2* spec, int bxe, int nrow, const int* offj, const int* offi,
                         int nb, hipStream_t s) {
#define X(W) if (a.wy == W) return gather_w<W>(a, spec, bxe, nrow, offj, offi, nb, s);
  DH_IFFT_SIZES(X)
#undef X
  return hipErrorInvalidValue;
}



hipError_t launch_norm(const KArgs& a, int b0, int nb, hipStream_t s) {
  hipLaunchKernelGGL(k_norm, dim3(nb), dim3(kTPB), 0, s, a, b0);
  return hipGetLastError();
}
hipError_t launch_zero(float2* p, size_t n, hipStream_t s) {
  if (n == 0) return hipSuccess;
  size_t blocks = (n + 255) / 256;
  if (blocks > 4096) blocks = 4096;
  hipLaunchKernelGGL(k_zero, dim3((unsigned)blocks), dim3(256), 0, s, p, n);
  return hipGetLastError();
}
hipError_t launch_hg(double pitch, int w, int wpad, double waist, int G, int gp, float* out,
                     unsigned short* bh, unsigned short* bl, _Float16* hh, _Float16* hl, double fp16_scale,
                     hipStream_t s) {
  hipLaunchKernelGGL(k_hg, dim3((wpad + 63) / 64), dim3(64), 0, s, pitch, w, wpad, waist, G, gp, out, bh, bl, hh, hl,
                     fp16_scale);
  return hipGetLastError();
}

}  // namespace dh
