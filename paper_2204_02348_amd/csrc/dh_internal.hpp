// Internal interface between the host plan (dh_api.cpp) and the gfx950
// kernels (dh_kernels.hip). Not part of the public C ABI.
#pragma once
#include <hip/hip_runtime.h>
#include <cstddef>
#include <vector>

namespace dh {

// Largest mode-group count G a plan takes, and its padded column count: the
// mode tables hold gp columns, 16 for G <= 16, else 32 ceil(G / 32) (the
// paper names LG bases of up to 100 groups; its HG basis sets no bound)
constexpr int kMaxGroups = 100;
constexpr int kMaxGp = 128;
// the field path's overlap tiles modes in at most two 16-column tiles
constexpr int kMaxGpField = 32;

// A transform length without a compiled kernel: n = r[0] r[1] ... r[np-1]
// (radices 2, 3, 4, 5, 7, 8, 11, 13, 16 and at most one prime above 13). The
// twiddles of pass s sit at table + off[s] as [r - 1][NS] (NS = r[0] ...
// r[s-1]); the roots e^{-2 pi i m / p} of a prime radix p > 16 at table +
// roots. np = 0: the length has a compiled kernel (or no plan).
constexpr int kGenMaxN = 2048;          // the compiled lengths go to 2048 too; keeps every LDS buffer <= 64 KB
constexpr int kGenMaxPasses = 12;
struct GenFft {
  int n, np;
  int r[kGenMaxPasses];
  int off[kGenMaxPasses];
  int roots;
};

// Per-polarisation plan tables (device pointers) and window geometry.
//
// "Box": the rectangle of spectrum bins that holds every bin of the Fourier
// window (mask). Box column j is row-pass bin k = k0 + j, i.e. window bin
// u = -(k0 + j); box row i is column-pass bin v' = ky0 + i, i.e. v = -(ky0 + i).
// The mask bins of the SR* term at (u, v) are read as conj(F(-u, -v)) from the
// real-input spectrum F of the frame window.
struct PolTab {
  int x0, y0;             // window origin in the frame (pixels)
  int k0, ky0;            // first row-pass bin / first column-pass bin of the box
  int bxq, byq;           // this pol's own box size (<= KArgs bx, by); IFFT column q holds box
                          // column j = (-k0 - q) mod wx if j < bxq, else none (rows alike)
  const int2* mrow;       // [by] mask interval of box row i in box columns (lo > hi: empty)
  const float2* rhox;     // [bx] sub-pixel beam-centre ramp along x
  const float2* rhoy;     // [by] same along y, times 1/(Nx Ny)
  const float2* tx;       // [wx] exp(i phi_R) along x (tilt + defocus)
  const float2* ty;       // [wy] same along y
  const float* ux;        // [wx][gp] u_m(x'_k) p'_x, zero for m >= G
  const float* uy;        // [wyp][gp] u_n(y'_l) p'_y, zero for n >= G or l >= wy
  // the same tables split as hi + lo for the precision form, packed
  // [k/4][mode][k%4] (four consecutive samples of one mode together):
  const unsigned short* ux_bh;  // bf16 hi / lo
  const unsigned short* ux_bl;
  const unsigned short* uy_bh;
  const unsigned short* uy_bl;
  const _Float16* ux_hh;        // fp16 hi / lo of the table times KArgs::s_uh
  const _Float16* ux_hl;
  const _Float16* uy_hh;
  const _Float16* uy_hl;
  // spectral path: the HG overlap, tilt/defocus, centre ramps and 1/(Nx Ny)
  // folded into two tables over the box (FP64-built, FP32):
  //   xs[j][m] = rho_x(j) sum_k tx[k] ux[k][m] e^{2 pi i u_j k / wx}, u_j = -(k0 + j)
  //   ys[i][n] = rho_y(i) sum_l ty[l] uy[l][n] e^{2 pi i v_i l / wy}, v_i = -(ky0 + i)
  // so that c_mn = sum_{j,i} mask(j,i) conj(S[j][i]) xs[j][m] ys[i][n], S the
  // column-pass spectrum at box (j, i)
  const float2* xs;       // [bx][gp]
  const float2* ys;       // [wyp][gp], zero rows i >= by
};

struct KArgs {
  int frame_w, frame_h, npol;
  int nx, ny, wx, wy, wyp;  // FFT window, IFFT window, IFFT rows rounded up to 16
  int bx, by;               // box size (max over pols)
  int bxp;                  // f2 row pitch: bx rounded up to 16
  int G, gp, nmodes;        // groups, padded group count (16 ceil(G / 16)), modes per pol
  float nxny;               // Nx * Ny
  int prec;                 // DH_PREC_FP32 / SPLIT_BF16 / SPLIT_FP16
  float s_uh;               // power-of-two prescale of the fp16 split HG tables
  PolTab pol[2];
  const short2* modes;      // [nmodes] (m, n)
  const float2* tw_nx;      // per-pass twiddle tables of each transform length (see fft_lds)
  const float2* tw_ny;
  const float2* tw_wx;
  const float2* tw_wy;
  const void* const* fptr;  // device array of frame pointers (frame b at fptr[b]) or null: contiguous frames
  float2* t1;               // [chunk][P][ny/16][bx][16] row-pass spectrum at the box columns, in
                            // tiles of 16 rows (row-pass blocks write whole tiles)
  float2* f2;               // [chunk][P][wy][bxp] column pass + crop + y-IFFT
  float2* partial;          // [chunk][nblk][P][nmodes + 1] per-row-block share of each coefficient,
                            // then the block's field power sum |E|^2 (if capt)
  double* capt;             // [max_batch][P][2] mode power, field power (FP64), or null
  double cell;              // p'_x p'_y, the field power's quadrature weight
  int nblk;                 // blocks with a partial per frame and pol: 16-row blocks of the
                            // field (wyp / 16), or column blocks of the spectral path
  int byp;                  // by rounded up to 16 (spectral path contraction length)
  float spow;               // spectral path: wx wy / (Nx Ny)^2, field power per |S|^2
  float2* coefs;            // [max_batch][P][nmodes] raw coefficients
  float2* coefs_norm;       // [max_batch][P][nmodes] power-normalised
  float2* window;           // [max_batch][P][wy][wx] or null
  float2* fields;           // [max_batch][P][wy][wx] or null
  GenFft gx, gy;            // row / column lengths without a compiled kernel (np > 0): the
                            // generic kernels run them, with tw_nx / tw_ny the generic tables
};

bool sizes_supported(int nx, int ny, int wx, int wy);    // every kernel of the field path compiled
bool fft_compiled(int n);                                // a compiled row / column / export transform
void fft_radices(int n, int r[3]);   // radices of the passes of a supported length
hipError_t launch_row(const KArgs& a, const void* frames, int u16, int b0, int nb, hipStream_t s);
hipError_t launch_col(const KArgs& a, int b0, int nb, hipStream_t s);
hipError_t launch_fld(const KArgs& a, int b0, int nb, hipStream_t s);
hipError_t launch_norm(const KArgs& a, int b0, int nb, hipStream_t s);
// spectral path: column FFT + masked window contracted with the xs / ys
// tables into per-column-block partials (replaces launch_col + launch_fld)
bool spectral_supported(int ny, int wy, int gp);
int spectral_blocks(int ny, int wy, int bx, int gp);   // column blocks per frame and pol
hipError_t launch_cspec(const KArgs& a, int b0, int nb, hipStream_t s);
hipError_t launch_zero(float2* p, size_t n, hipStream_t s);
// alignment: column FFT of an extended box stored as spec[b][p][j][i] (nrow rows
// from ky0); gather of the current window from it; batch power spectrum
hipError_t launch_spec(const KArgs& a, float2* spec, int nrow, int nb, hipStream_t s);
hipError_t launch_gather(const KArgs& a, const float2* spec, int bxe, int nrow, const int* offj, const int* offi,
                         int nb, hipStream_t s);
hipError_t launch_psum(const float2* spec, int nb, int npol, size_t plane, float* pw, hipStream_t s);
// FP64 intensity moments of n fields [wy][wx]: out[e][5] = sums of I, xI, yI,
// x^2 I, y^2 I on the coarse grid x = (k - wx/2) px, y = (l - wy/2) py
// wavelength sweep / averaging: N = I L outputs, A repetitions each; staged
// position of output o's repetition a = (w I + i) A + a, (i, w) of o by the
// output ordering (0: o = i L + w, 1: o = w I + i)
struct Comb {
  int L, I, A, out_order;
};
// sptr[s] = base + (input frame of staged position s) * fbytes for the n_out * A
// positions (avg_mode 0 sequential, 1 interlaced, 2 sequential sweep; in_order
// 0 fast, 1 slow)
hipError_t launch_fptr(const char* base, size_t fbytes, int n_out, int L, int I, int A, int avg_mode, int in_order,
                       const void** sptr, hipStream_t s);
// rot[o A + a] = exp(-i arg sum win[s(o,a)] conj(win[s(o,0)])) over `per` values (1 for a = 0)
hipError_t launch_avg_rot(const float2* win, long long per, const Comb& c, int n_out, double2* rot, hipStream_t s);
// out[o] = mean over a of rot * staged[s(o, a)] (rot null: 1), `per` values per
// position; coefficients also give out_norm (the staged normalised values for
// A = 1, else out over the FP64 norm of out)
hipError_t launch_comb_coefs(const float2* sc, const float2* scn, const double2* rot, int per, const Comb& c, int n_out,
                             float2* out, float2* out_norm, hipStream_t s);
hipError_t launch_comb_plane(const float2* in, const double2* rot, long long per, const Comb& c, int n_out, float2* out,
                             hipStream_t s);
// IFFT mode 0 field export: output frames first + z stride (z < the launch's
// frames) of the window [frame][pol][wy][wx] to fields [frame][pol][ny][nx];
// t2 [z][pol][ny][bxp] holds the y-transformed box columns of the group
struct M0Args {
  const float2* win;
  float2* t2;
  float2* fields;
  const float2* tw_nx;     // per-pass twiddles of the N_x and N_y transforms
  const float2* tw_ny;
  int nx, ny, wx, wy, bxp, npol;
  int first, stride;
  struct {
    int uhi, vhi, bxq, byq;  // box: column j is bin uhi - j, row i is bin vhi - i
    const float2* phx;       // [nx] tilt/defocus phase along x
    const float2* phy;       // [ny] the same along y, times 1/(Nx Ny)
  } pol[2];
  GenFft gx, gy;             // as in KArgs
};
hipError_t launch_m0y(const M0Args& m, int nb, hipStream_t s);
hipError_t launch_m0x(const M0Args& m, int nb, hipStream_t s);
// fields to int16 (re, im) with one FP32 scale per field: n fields of len values
hipError_t launch_q16(const float2* fields, int n, long long len, short* re, short* im, float* scale, hipStream_t s);
// generic-length kernels (dh_generic.hip): plan and twiddle table of a
// length (false: more than one prime factor above 13, or n > kGenMaxN);
// entries the table needs at most; launches as launch_row / launch_cspec /
// launch_m0y / launch_m0x, which call them for lengths with np > 0
bool gen_plan(int n, GenFft* g);
std::vector<float2> gen_twiddles(const GenFft& g);
size_t gen_twiddle_count(int n);
int gen_cols_per_block(int ny, int gp);
hipError_t launch_row_gen(const KArgs& a, const void* frames, int u16, int b0, int nb, hipStream_t s);
hipError_t launch_cspec_gen(const KArgs& a, int b0, int nb, hipStream_t s);
hipError_t launch_m0y_gen(const M0Args& m, int bx, int nb, hipStream_t s);
hipError_t launch_m0x_gen(const M0Args& m, int nb, hipStream_t s);

// basis transform of n coefficient vectors (frame x pol, rows of nin values,
// the first nused of them taken): out[e][k] = sum_{i < cnt} tt[off + i stride]
// in[e][first + i] with (first, cnt, off, stride) = rng[k], for the raw and
// the normalised coefficients
hipError_t launch_basis(const float2* in, const float2* in_norm, int nin, int nused, const int4* rng,
                        const float2* tt, int nout, float2* out, float2* out_norm, int n, hipStream_t s);
hipError_t launch_moments(const float2* fields, int n, int wx, int wy, double px, double py, double* out,
                          hipStream_t s);
// HG tables: out[k][n] in FP32 and, if the split pointers are non-null, the
// packed hi/lo tables (bf16, and fp16 of the value times fp16_scale)
hipError_t launch_hg(double pitch, int w, int wpad, double waist, int G, int gp, float* out,
                     unsigned short* bh, unsigned short* bl, _Float16* hh, _Float16* hl, double fp16_scale,
                     hipStream_t s);

// transfer-matrix metrics (FP64): A from the coefficients [B][P][M]
struct TmArgs {
  const float2* c;          // raw coefficients of the batch
  const short2* modes;      // [M] (m, n): HG mode keys (pol, m + n) when grp is null
  const int* grp;           // [M] group id of each mode (key pol * ngrp + id), or null
  int ngrp;
  int B, P, M;
  int indep;                // pol-independent rows (p B + b), cross-pol entries zero
  int rows, cols;           // B (or P B) x P M
};
// Gram X X^H (n x n, column-major) with X = A (by_rows) or A^H
hipError_t launch_tm_gram(const TmArgs& t, int by_rows, int n, double2* g, hipStream_t s);
// per row of D (A if g is null, else the rows x rows Gram in g): row power,
// and for rows < nd the diagonal power and the power sharing the row's mode key
hipError_t launch_tm_rows(const TmArgs& t, const double2* g, int nrow, int ncol, int nd, double* rowpow, double* diag,
                          double* same, hipStream_t s);
// out[i] = Re g[i][i] of an n x n complex matrix
hipError_t launch_tm_diag(const double2* g, int n, double* out, hipStream_t s);
// batch summary: the eight sums of each of n planes (see k_summ) from complex
// planes z or FP64 intensity maps, value (l, k) of plane e at e pstride + l sy
// + k sx; and map[p][l][k] (+)= the intensity summed over nb frames (plane
// b npol + p of z)
hipError_t launch_summ(const float2* z, const double* map, long long pstride, int w, int h, int sx, int sy, int n,
                       double* out, hipStream_t s);
hipError_t launch_isum(const float2* z, long long pstride, int w, int h, int sx, int sy, int nb, int npol,
                       int accumulate, double* map, hipStream_t s);
// every eigenvalue of the n x n Hermitian g (column-major, overwritten) into
// w[n] by cyclic Jacobi; info = sweeps used, -1 if it did not converge
hipError_t launch_heig(double2* g, int n, double* w, int* info, hipStream_t s);

}  // namespace dh
