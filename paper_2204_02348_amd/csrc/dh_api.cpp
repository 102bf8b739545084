// Host side of libdh: parameter validation, FP64 plan geometry and tables,
// device allocation, launch sequencing, and the C ABI of include/dh.h.
#include "dh.h"

#include <hip/hip_runtime.h>

#include <algorithm>
#include <cfloat>
#include <chrono>
#include <deque>
#include <map>
#include <cmath>
#include <complex>
#include <cstdint>
#include <cstdlib>
#include <cstring>
#include <mutex>
#include <vector>

#include "dh_internal.hpp"

namespace {

using cd = std::complex<double>;
constexpr double kPi = 3.14159265358979323846264338327950288;
constexpr double kDeg = kPi / 180.0;

bool smooth13(int n) {
  for (int f : {2, 3, 5, 7, 11, 13})
    while (n % f == 0) n /= f;
  return n == 1;
}

// IFFT (field) length for a Fourier window of radius r bins: the smallest
// multiple of 16 with prime factors <= 13 that holds floor(2r)+1 bins.
int field_len(double r) {
  const int need = (int)std::floor(2.0 * r) + 1;
  int w = 16;
  while (w < need || !smooth13(w)) w += 16;
  return w;
}

struct PolGeom {
  double ax, ay;         // cross-term position (bins): SR* at (-ax, -ay)
  int x0, y0;            // window origin
  double dx, dy;         // sub-pixel beam-centre remainder, m
  int uhi, ulo, vhi, vlo;
  std::vector<int> row_lo, row_hi;  // per box row i (v = vhi - i): mask u-range
};

struct Geom {
  int nx, ny, wx, wy, wyp, wys, bx, by, G, gp, nmodes;
  double rx, ry, pxp, pyp;
  int mode = 1;          // IFFT resolution mode
  int fx = 0, fy = 0;    // field grid: W (mode 1) or N (mode 0)
  double fpx = 0, fpy = 0;   // its pitch: N p / F
  bool spec = false;     // the plan runs the spectral path (DH_PATH_SPECTRAL)
  int byp = 16;          // by rounded up to 16
  PolGeom pol[2];
  dh::GenFft gx{}, gy{}; // row / column lengths the generic kernels run (np > 0)
};

// blocks with a coefficient partial per frame and pol: 16-row field blocks
// (field path, also used by alignment) or column blocks (spectral path)
int field_blocks(const Geom& g) { return g.wyp / 16; }
int partial_blocks(const Geom& g) {
  return g.spec ? std::max(field_blocks(g), dh::spectral_blocks(g.ny, g.wy, g.bx, g.gp)) : field_blocks(g);
}

bool inside(double u, double v, double ax, double ay, double rx, double ry) {
  const double a = (u + ax) / rx, b = (v + ay) / ry;
  return a * a + b * b <= 1.0;
}

// Tilt- and centre-dependent geometry of polarisation q: window origin,
// cross-term position, the box of bins inside the Fourier window and each box
// row's mask interval (FP64, inclusive ellipse in bins).
int derive_pol(const dh_params* p, Geom* g, int q) {
  const double pix = p->pixel_size, lam = p->wavelength;
  const int nx = g->nx, ny = g->ny;
  const int half = p->frame_w / p->pol_count;
  PolGeom& P = g->pol[q];
  P.ax = p->tilt_deg[q][0] * kDeg * nx * pix / lam;
  P.ay = p->tilt_deg[q][1] * kDeg * ny * pix / lam;
  const int ix = (int)std::floor(p->beam_centre[q][0] / pix + 0.5);
  const int iy = (int)std::floor(p->beam_centre[q][1] / pix + 0.5);
  P.x0 = q * half + half / 2 + ix - nx / 2;
  P.y0 = p->frame_h / 2 + iy - ny / 2;
  P.dx = p->beam_centre[q][0] - ix * pix;
  P.dy = p->beam_centre[q][1] - iy * pix;
  if (P.x0 < 0 || P.x0 + nx > p->frame_w || P.y0 < 0 || P.y0 + ny > p->frame_h) return DH_ERR_INVALIDDIMENSION;
  // the first and last bin inside the window on each row of a bounding range,
  // found by scanning in from both ends (the row's minimum and maximum, as a
  // full scan would give, at the cost of the bins outside only: alignment
  // trials re-derive this every time), and the box they span
  const int u_a = (int)std::floor(-P.ax - g->rx) - 1, u_b = (int)std::ceil(-P.ax + g->rx) + 1;
  const int v_a = (int)std::floor(-P.ay - g->ry) - 1, v_b = (int)std::ceil(-P.ay + g->ry) + 1;
  std::vector<int> rlo((size_t)(v_b - v_a + 1), 1), rhi((size_t)(v_b - v_a + 1), 0);
  P.ulo = u_b; P.uhi = u_a; P.vlo = v_b; P.vhi = v_a;
  for (int v = v_a; v <= v_b; ++v) {
    int lo = u_a;
    while (lo <= u_b && !inside(lo, v, P.ax, P.ay, g->rx, g->ry)) ++lo;
    if (lo > u_b) continue;
    int hi = u_b;
    while (!inside(hi, v, P.ax, P.ay, g->rx, g->ry)) --hi;   // stops at lo at the latest
    rlo[(size_t)(v - v_a)] = lo;
    rhi[(size_t)(v - v_a)] = hi;
    P.ulo = std::min(P.ulo, lo); P.uhi = std::max(P.uhi, hi);
    P.vlo = std::min(P.vlo, v); P.vhi = std::max(P.vhi, v);
  }
  if (P.uhi < P.ulo || P.vhi < P.vlo) return DH_ERR_INVALIDARGUMENT;  // empty window
  const int bxq = P.uhi - P.ulo + 1, byq = P.vhi - P.vlo + 1;
  if (bxq > g->bx || byq > g->by) return DH_ERR_INVALIDARGUMENT;
  P.row_lo.assign(byq, 1);
  P.row_hi.assign(byq, 0);
  for (int i = 0; i < byq; ++i) {
    const size_t r = (size_t)(P.vhi - i - v_a);
    P.row_lo[i] = rlo[r];
    P.row_hi[i] = rhi[r];
  }
  return DH_SUCCESS;
}

int derive(const dh_params* p, Geom* g) {
  if (!p) return DH_ERR_NULLPOINTER;
  if (p->pol_count != 1 && p->pol_count != 2) return DH_ERR_INVALIDPOLARISATION;
  if (p->frame_w <= 0 || p->frame_h <= 0 || p->frame_w % 16 || p->frame_h % 16) return DH_ERR_INVALIDDIMENSION;
  const int nx = (p->fft_w / 16) * 16, ny = (p->fft_h / 16) * 16;
  if (nx <= 0 || ny <= 0) return DH_ERR_INVALIDDIMENSION;
  if (!(p->pixel_size > 0) || !(p->wavelength > 0) || !(p->window_radius_deg > 0)) return DH_ERR_INVALIDARGUMENT;
  if (p->max_mg < 0 || p->max_mg > dh::kMaxGroups) return DH_ERR_INVALIDARGUMENT;
  if (p->max_mg > 0 && !(p->waist > 0)) return DH_ERR_INVALIDARGUMENT;
  if (p->input_dtype != DH_INPUT_F32 && p->input_dtype != DH_INPUT_U16) return DH_ERR_INVALIDARGUMENT;
  if (p->precision != DH_PREC_FP32 && p->precision != DH_PREC_SPLIT_BF16 && p->precision != DH_PREC_SPLIT_FP16)
    return DH_ERR_INVALIDARGUMENT;
  if (p->ifft_mode != 0 && p->ifft_mode != 1) return DH_ERR_INVALIDARGUMENT;
  if (p->path < DH_PATH_AUTO || p->path > DH_PATH_SPECTRAL) return DH_ERR_INVALIDARGUMENT;
  for (int q = 0; q < p->pol_count; ++q) {
    for (int a = 0; a < 2; ++a)
      if (!std::isfinite(p->tilt_deg[q][a]) || !std::isfinite(p->beam_centre[q][a])) return DH_ERR_INVALIDARGUMENT;
    if (!std::isfinite(p->defocus[q])) return DH_ERR_INVALIDARGUMENT;
  }
  const double pix = p->pixel_size, lam = p->wavelength;
  const double wmax = lam / (2.0 * pix);
  g->nx = nx;
  g->ny = ny;
  g->rx = (p->window_radius_deg * kDeg / wmax) * (nx / 2.0);
  g->ry = (p->window_radius_deg * kDeg / wmax) * (ny / 2.0);
  if (2.0 * g->rx + 1.0 >= nx || 2.0 * g->ry + 1.0 >= ny) return DH_ERR_INVALIDARGUMENT;
  g->wx = field_len(g->rx);
  g->wy = field_len(g->ry);
  g->wyp = (g->wy + 15) / 16 * 16;
  // rows of the spectral ys table: a multiple of 32 (zero past the box), the
  // K extent of the widest column workgroup's MFMA steps
  g->wys = (g->wy + 31) / 32 * 32;
  g->pxp = nx * pix / g->wx;
  g->pyp = ny * pix / g->wy;
  g->mode = p->ifft_mode;
  g->fx = g->mode ? g->wx : nx;
  g->fy = g->mode ? g->wy : ny;
  g->fpx = nx * pix / g->fx;
  g->fpy = ny * pix / g->fy;
  g->G = p->max_mg;
  // mode columns of the tables: one or two 16-column tiles, beyond that a
  // multiple of 32 (the spectral contraction's chunks of two tiles)
  g->gp = g->G <= 16 ? 16 : (g->G + 31) / 32 * 32;
  g->nmodes = g->G * (g->G + 1) / 2;
  // every window position fits a box of floor(2r)+1 bins per axis, so the
  // workspaces do not change when the tilt does (alignment)
  g->bx = (int)std::floor(2.0 * g->rx) + 1;
  g->by = (int)std::floor(2.0 * g->ry) + 1;
  if (g->bx > g->wx || g->by > g->wy) return DH_ERR_INVALIDARGUMENT;
  for (int q = 0; q < p->pol_count; ++q) {
    const int e = derive_pol(p, g, q);
    if (e != DH_SUCCESS) return e;
  }
  g->byp = (g->by + 15) / 16 * 16;
  // Lengths without a compiled kernel run on the generic kernels: the row
  // pass for N_x, the spectral column pass (and the mode-0 export) for N_y or
  // an (N_y, W_y) pair without a compiled column kernel. The field path needs
  // compiled kernels for every length.
  g->gx = dh::GenFft{};
  g->gy = dh::GenFft{};
  if (!dh::fft_compiled(nx) && !dh::gen_plan(nx, &g->gx)) return DH_ERR_INVALIDDIMENSION;
  if (g->mode == 0) {
    // IFFT mode 0: the coefficients come from spectral tables built on the FFT
    // grid, the fields (on request) from the kept window by full-size inverse
    // FFTs; with G = 0 only the window and the fields are made
    if (p->path == DH_PATH_FIELD || p->precision != DH_PREC_FP32) return DH_ERR_INVALIDARGUMENT;
    g->spec = true;
  } else {
    const bool can_spec = p->precision == DH_PREC_FP32 && !p->keep_fields && g->G > 0;
    if (p->path == DH_PATH_SPECTRAL && !can_spec) return DH_ERR_INVALIDARGUMENT;
    g->spec = p->path == DH_PATH_SPECTRAL || (p->path == DH_PATH_AUTO && can_spec);
    // the field path's overlap takes up to two mode tiles (G <= 32)
    if (g->gp > dh::kMaxGpField && !g->spec) return DH_ERR_INVALIDARGUMENT;
    if (!g->spec && !dh::sizes_supported(nx, ny, g->wx, g->wy)) return DH_ERR_INVALIDDIMENSION;
  }
  if (g->spec && !dh::spectral_supported(ny, g->wy, g->gp) && !dh::gen_plan(ny, &g->gy))
    return DH_ERR_INVALIDDIMENSION;
  return DH_SUCCESS;
}

size_t align256(size_t n) { return (n + 255) & ~size_t(255); }

// mode-0 fields are made from the kept window after the coefficients
bool exports(const Geom& g, const dh_params* p) { return g.mode == 0 && p->keep_fields; }
// frames per export group: the y-transformed columns within 256 MiB
int export_chunk(const Geom& g, const dh_params* p, int max_batch) {
  const size_t per = (size_t)p->pol_count * g.fy * ((g.bx + 15) / 16 * 16) * 8;
  const long c = (long)((256ull << 20) / (per ? per : 1));
  return (int)std::max(1L, std::min<long>(c, max_batch));
}

int env_int(const char* name, int dflt) {
  if (const char* env = std::getenv(name)) {
    const long v = std::strtol(env, nullptr, 10);
    if (v > 0) return (int)v;
  }
  return dflt;
}

int chunk_for(const Geom& g, int npol, int max_batch) {
  // Frames per launch. Larger launches amortise the partly filled last wave
  // of workgroups; whether the intermediates stay in the last-level cache was
  // measured not to matter, so a chunk is as large as a 2 GiB workspace
  // allows. DH_CHUNK_FRAMES overrides the frame count.
  const size_t per = (size_t)npol * ((size_t)g.ny + (size_t)g.wy + g.wy / 8) * ((g.bx + 15) / 16 * 16) * 8;
  long c = (long)((2ull << 30) / (per ? per : 1));
  c = env_int("DH_CHUNK_FRAMES", (int)std::min<long>(c, 1 << 30));
  if (c < 1) c = 1;
  if (c > max_batch) c = max_batch;
  return (int)c;
}

// chunks in flight at once, each on its own internal stream with its own
// workspace (DH_STREAMS overrides; 1 = everything on the caller's stream)
int streams_for(int max_batch, int chunk) {
  int n = env_int("DH_STREAMS", 2);
  const int chunks = (max_batch + chunk - 1) / chunk;
  if (n > chunks) n = chunks;
  if (n > 4) n = 4;
  return n < 1 ? 1 : n;
}

struct Layout {  // byte offsets inside one device allocation
  size_t tw_nx, tw_ny, tw_wx, tw_wy, modes, total_tables;
  size_t pol_mrow[2], pol_rhox[2], pol_rhoy[2], pol_tx[2], pol_ty[2], pol_ux[2], pol_uy[2];
  size_t pol_uxs[2][4], pol_uys[2][4];   // split tables: bf16 hi, bf16 lo, fp16 hi, fp16 lo
  size_t pol_xs[2], pol_ys[2];           // spectral path tables
  size_t pol_ex[2], pol_ey[2];           // mode-0 field export: phase tables along x and y
  size_t export_t;                       // mode-0 field export: the y-transformed box columns
  size_t t1[4], f2[4], partial[4], capt, coefs, coefs_norm, window, fields, total;
};



Layout layout(const Geom& g, const dh_params* p, int max_batch, int chunk, int nws) {
  Layout L{};
  size_t o = 0;
  auto take = [&](size_t bytes) { size_t r = o; o += align256(bytes); return r; };
  L.tw_nx = take(dh::gen_twiddle_count(g.nx) * 8); L.tw_ny = take(dh::gen_twiddle_count(g.ny) * 8);
  L.tw_wx = take(g.wx * 8); L.tw_wy = take(g.wy * 8);
  L.modes = take((g.nmodes > 0 ? g.nmodes : 1) * 4);
  for (int q = 0; q < p->pol_count; ++q) {
    L.pol_mrow[q] = take(g.by * 8);
    L.pol_rhox[q] = take(g.bx * 8);
    L.pol_rhoy[q] = take(g.by * 8);
    L.pol_tx[q] = take(g.wx * 8);
    L.pol_ty[q] = take(g.wy * 8);
  }
  L.total_tables = o;   // host-built tables end here; the HG tables (built on the GPU) follow
  for (int q = 0; q < p->pol_count; ++q) {
    L.pol_ux[q] = take((size_t)g.wx * g.gp * 4);
    L.pol_uy[q] = take((size_t)g.wyp * g.gp * 4);
    for (int t = 0; t < 4; ++t) {
      L.pol_uxs[q][t] = take((size_t)g.wx * g.gp * 2);
      L.pol_uys[q][t] = take((size_t)g.wyp * g.gp * 2);
    }
    L.pol_xs[q] = take(g.spec ? (size_t)g.bx * g.gp * 8 : 0);
    L.pol_ys[q] = take(g.spec ? (size_t)g.wys * g.gp * 8 : 0);
    L.pol_ex[q] = take(exports(g, p) ? (size_t)g.fx * 8 : 0);
    L.pol_ey[q] = take(exports(g, p) ? (size_t)g.fy * 8 : 0);
  }
  const size_t P = p->pol_count;
  const size_t nm = g.nmodes > 0 ? g.nmodes : 1;
  for (int w = 0; w < nws; ++w) {
    L.t1[w] = take((size_t)chunk * P * g.ny * g.bx * 8);
    L.f2[w] = take((size_t)chunk * P * g.wy * ((g.bx + 15) / 16 * 16) * 8);
    L.partial[w] = take((size_t)chunk * P * partial_blocks(g) * (nm + 1) * 8);
  }
  L.capt = take((size_t)max_batch * P * 2 * 8);
  L.coefs = take((size_t)max_batch * P * nm * 8);
  L.coefs_norm = take((size_t)max_batch * P * nm * 8);
  L.window = p->keep_window || exports(g, p) ? take((size_t)max_batch * P * g.wy * g.wx * 8) : 0;
  L.fields = p->keep_fields ? take((size_t)max_batch * P * g.fy * g.fx * 8) : 0;
  L.export_t = exports(g, p) ? take((size_t)export_chunk(g, p, max_batch) * P * g.fy * ((g.bx + 15) / 16 * 16) * 8)
                              : 0;
  L.total = o;
  return L;
}

struct Plan {
  dh_params params;
  Geom g;
  Layout L;
  int max_batch = 1, chunk = 1, nws = 1, last_batch = 0, last_error = 0;
  int device = 0;
  float s_uh = 1.f;
  char* mem = nullptr;
  hipStream_t last_stream = nullptr;
  dh::KArgs ka[4]{};                 // one per workspace
  hipStream_t str[4]{};              // internal streams (nws > 1)
  hipEvent_t fork = nullptr, join[4]{};
  // per-stage timing: a start and an end event around every launch, on the
  // stream the kernel runs on
  // alignment: device scratch reused across calls, and the last report
  char* amem = nullptr;
  // transfer-matrix metrics: workspace (grown on demand)
  char* tm_mem = nullptr;
  size_t tm_bytes = 0;
  unsigned lock = 0;                 // DH_ALIGN_TILT / DH_ALIGN_DEFOCUS: pol 1 takes pol 0's value
  char* q16_mem = nullptr;           // int16 fields and scales (dh_get_fields16), made on first use
  // basis transform after the HG overlap (DH_BASIS_LG / CUSTOM): c_out = T c_HG
  int basis = DH_BASIS_HG;
  int bout = 0, bin = 0, bngrp = 0;  // output modes, HG modes used, group ids
  char* bmem = nullptr;
  float2* btt = nullptr;             // T entries (see bt_entry)
  int4* brng = nullptr;              // [bout] per output mode: first HG mode, count, entry offset, entry stride
  int* bgrp = nullptr;               // [bout] group id of each output mode
  float2* bc = nullptr;              // [max(max_batch, ocap)][P][bout] raw, then normalised
  float2* bcn = nullptr;
  // outputs of batches larger than max_batch: the raw and normalised
  // coefficients (and the basis coefficients) for ocap frames, made on the
  // first such batch and grown when a larger one comes
  char* omem = nullptr;
  int ocap = 0;
  // wavelength sweep (dh_set_wavelengths) and frame averaging (dh_set_averaging)
  int nlam = 0;                      // 0: every frame at the plan's wavelength
  int in_order = 0, out_order = 0;   // DH_WL_FAST / DH_WL_SLOW
  int avg = 1, avg_mode = 0;
  std::vector<double> lams;
  std::vector<PolGeom> lam_geom;     // [nlam][P]
  struct LamTab { size_t mrow, rhox, rhoy, tx, ty, xs, ys, ex, ey; };
  std::vector<LamTab> lam_tab;       // [nlam][P] offsets in lmem
  char* lmem = nullptr;
  // staging of the input frames' results before the outputs are combined
  char* smem = nullptr;
  const void** sptr = nullptr;       // [max_batch] frame of each staged position
  float2 *sc = nullptr, *scn = nullptr, *swin = nullptr, *sfld = nullptr;
  double2* rot = nullptr;            // [max_batch] phase factor of each repetition
  int goal = DH_GOAL_CAPTURED;       // alignment goal and its transfer-matrix options
  int goal_indep = 0, goal_aa = 0;
  size_t amem_bytes = 0;
  dh_align_report rep{};
  int version = 0;                   // bumped whenever the tables are rebuilt
  std::vector<char> trial_host;      // host image of the per-pol tables of an alignment trial
  bool timing = false;
  std::vector<hipEvent_t> ev_pool;
  std::vector<int> ev_stage;         // stage of launch i (events 2i, 2i+1)
  size_t ev_used = 0;                // events used
};

hipError_t timed_event(Plan* pl, hipStream_t s, int stage, bool start) {
  if (!pl->timing) return hipSuccess;
  if (pl->ev_used == pl->ev_pool.size()) {
    hipEvent_t e;
    if (hipEventCreate(&e) != hipSuccess) return hipErrorOutOfMemory;
    pl->ev_pool.push_back(e);
  }
  if (start) pl->ev_stage.push_back(stage);
  return hipEventRecord(pl->ev_pool[pl->ev_used++], s);
}

std::mutex g_mu;
std::vector<Plan*> g_plans;

Plan* get(dh_handle h) {
  std::lock_guard<std::mutex> lk(g_mu);
  if (h < 0 || (size_t)h >= g_plans.size()) return nullptr;
  return g_plans[h];
}

template <typename T>
void put(std::vector<char>& host, size_t off, const std::vector<T>& v) {
  std::memcpy(host.data() + off, v.data(), v.size() * sizeof(T));
}

// Twiddles of the FFT passes after the first, in FP64 rounded to FP32:
// for a pass of radix R after earlier radices with product NS, entry
// (r-1)*NS + k = e^{-2 pi i k r / (NS R)}; the passes follow each other.
std::vector<float2> twiddles(int n, const dh::GenFft& gen) {
  if (gen.np > 0) return dh::gen_twiddles(gen);
  int r[3];
  dh::fft_radices(n, r);
  std::vector<float2> t;
  int ns = r[0];
  for (int s = 1; s < 3 && r[s] > 1; ++s) {
    for (int rr = 1; rr < r[s]; ++rr)
      for (int k = 0; k < ns; ++k) {
        const double a = -2.0 * kPi * (double)k * rr / ((double)ns * r[s]);
        t.push_back(make_float2((float)std::cos(a), (float)std::sin(a)));
      }
    ns *= r[s];
  }
  if (t.empty()) t.push_back(make_float2(1.f, 0.f));
  return t;
}

// Power of two that maps the largest possible HG table entry close below
// 2^14: |psi_n| <= pi^(-1/4) for every n (Cramer's bound), so
// |u_n(x) p'| <= 2^(1/4) pi^(-1/4) w^(-1/2) p'.
double hg_fp16_scale(double waist, double pitch) {
  const double bound = std::pow(2.0, 0.25) * std::pow(kPi, -0.25) / std::sqrt(waist) * pitch;
  int e;
  std::frexp(bound, &e);
  return std::ldexp(1.0, 14 - e);
}

// u_n(x'_k) p' for k < w, n < G (FP64, the normalised Hermite recurrence of
// k_hg), [k][n]
std::vector<double> hg_host(double pitch, int w, double waist, int G) {
  std::vector<double> t((size_t)w * std::max(G, 1), 0.0);
  const double scale = std::pow(2.0, 0.25) / std::sqrt(waist) * pitch;
  for (int k = 0; k < w; ++k) {
    const double s = std::sqrt(2.0) * (k - 0.5 * w) * pitch / waist;
    double prev = 0.0, cur = std::pow(kPi, -0.25) * std::exp(-0.5 * s * s);
    for (int n = 0; n < G; ++n) {
      t[(size_t)k * G + n] = cur * scale;
      const double nxt = std::sqrt(2.0 / (n + 1)) * s * cur - std::sqrt((double)n / (n + 1)) * prev;
      prev = cur;
      cur = nxt;
    }
  }
  return t;
}

// Spectral path tables (FP64, stored FP32): the inverse DFT along one axis,
// the tilt/defocus phase, the HG quadrature weights, the sub-pixel centre
// ramp (and along y the 1/(Nx Ny) of the inverse transform) folded into
//   t[j][m] = rho(j) sum_k e^{i phi(k)} u_m(x'_k) p' e^{2 pi i u_j k / W},  u_j = u_hi - j.
std::vector<float2> spectral_axis(int nbox, int npad, int gp, int G, int uhi, int w, double pitch, double tilt_bins,
                                  double defocus, double lam, double sub, double pix, int nfft, double norm,
                                  const std::vector<double>& hg) {
  std::vector<cd> ph(w), root(w);
  for (int k = 0; k < w; ++k) {
    const double x = (k - w / 2.0) * pitch;
    ph[k] = std::exp(cd(0, 2.0 * kPi * tilt_bins * (k - w / 2.0) / w + kPi * defocus * x * x / lam));
    root[k] = std::exp(cd(0, 2.0 * kPi * k / w));
  }
  std::vector<float2> t((size_t)npad * gp, make_float2(0.f, 0.f));
  std::vector<cd> acc(G);
  for (int j = 0; j < nbox; ++j) {
    const long long u = uhi - j;
    std::fill(acc.begin(), acc.end(), cd(0, 0));
    for (int k = 0; k < w; ++k) {
      long long e = (u * k) % w;
      if (e < 0) e += w;
      const cd f = ph[k] * root[(size_t)e];
      const double* h = hg.data() + (size_t)k * G;
      for (int m = 0; m < G; ++m) acc[m] += f * h[m];
    }
    const cd rho = std::exp(cd(0, 2.0 * kPi * (double)u * sub / (pix * nfft))) * norm;
    for (int m = 0; m < G; ++m) {
      const cd v = rho * acc[m];
      t[(size_t)j * gp + m] = make_float2((float)v.real(), (float)v.imag());
    }
  }
  return t;
}

// Mode-0 field export: the tilt and defocus phase along one axis of the
// F-point field grid x_k = (k - F/2) p', times norm (FP64, stored FP32):
//   e[k] = norm e^{i (2 pi a (k - F/2) / F + pi D x_k^2 / lambda)},  a the tilt in bins.
std::vector<float2> export_phase(int f, double pitch, double tilt_bins, double defocus, double lam, double norm) {
  std::vector<float2> t(f);
  for (int k = 0; k < f; ++k) {
    const double x = (k - f / 2.0) * pitch;
    const cd v = std::exp(cd(0, 2.0 * kPi * tilt_bins * (k - f / 2.0) / f + kPi * defocus * x * x / lam)) * norm;
    t[k] = make_float2((float)v.real(), (float)v.imag());
  }
  return t;
}

// Host tables of polarisation q with geometry P (its wavelength is p's):
// the window rows, the centre ramps and the tilt/defocus phases of the field
// path; with spec, the spectral path tables; with exp, the mode-0 export
// tables.
struct PolTables {
  std::vector<int2> mrow;
  std::vector<float2> rhox, rhoy, tx, ty, xs, ys, ex, ey;
};

PolTables pol_tables(const Geom& g, const PolGeom& P, const dh_params* p, int q, bool spec, bool exp) {
  PolTables t;
  const double pix = p->pixel_size, lam = p->wavelength;
  const int byq = P.vhi - P.vlo + 1;
  t.mrow.assign(g.by, make_int2(1, 0));
  for (int i = 0; i < byq; ++i)
    if (P.row_lo[i] <= P.row_hi[i]) t.mrow[i] = make_int2(P.uhi - P.row_hi[i], P.uhi - P.row_lo[i]);
  t.rhox.resize(g.bx);
  t.rhoy.resize(g.by);
  t.tx.resize(g.wx);
  t.ty.resize(g.wy);
  for (int j = 0; j < g.bx; ++j) {
    const int u = P.uhi - j;
    const cd r = std::exp(cd(0, 2.0 * kPi * u * P.dx / (pix * g.nx)));
    t.rhox[j] = make_float2((float)r.real(), (float)r.imag());
  }
  const double inv = 1.0 / ((double)g.nx * g.ny);
  for (int i = 0; i < g.by; ++i) {
    const int v = P.vhi - i;
    const cd r = std::exp(cd(0, 2.0 * kPi * v * P.dy / (pix * g.ny))) * inv;
    t.rhoy[i] = make_float2((float)r.real(), (float)r.imag());
  }
  for (int k = 0; k < g.wx; ++k) {
    const double x = (k - g.wx / 2.0) * g.pxp;
    const double ph = 2.0 * kPi * P.ax * (k - g.wx / 2.0) / g.wx + kPi * p->defocus[q] * x * x / lam;
    t.tx[k] = make_float2((float)std::cos(ph), (float)std::sin(ph));
  }
  for (int l = 0; l < g.wy; ++l) {
    const double y = (l - g.wy / 2.0) * g.pyp;
    const double ph = 2.0 * kPi * P.ay * (l - g.wy / 2.0) / g.wy + kPi * p->defocus[q] * y * y / lam;
    t.ty[l] = make_float2((float)std::cos(ph), (float)std::sin(ph));
  }
  if (spec) {
    // the overlap's quadrature runs over the field grid: the Fourier-window
    // size in IFFT mode 1, the FFT size in mode 0
    const double waist = p->waist > 0 ? p->waist : 1.0;
    const std::vector<double> hx = hg_host(g.fpx, g.fx, waist, g.G), hy = hg_host(g.fpy, g.fy, waist, g.G);
    t.xs = spectral_axis(g.bx, g.bx, g.gp, g.G, P.uhi, g.fx, g.fpx, P.ax, p->defocus[q], lam, P.dx, pix, g.nx, 1.0,
                         hx);
    t.ys = spectral_axis(g.by, g.wys, g.gp, g.G, P.vhi, g.fy, g.fpy, P.ay, p->defocus[q], lam, P.dy, pix, g.ny,
                         inv, hy);
  }
  if (exp) {
    t.ex = export_phase(g.fx, g.fpx, P.ax, p->defocus[q], lam, 1.0);
    t.ey = export_phase(g.fy, g.fpy, P.ay, p->defocus[q], lam, inv);
  }
  return t;
}

template <typename T>
bool upload(char* base, size_t off, const std::vector<T>& v) {
  return v.empty() || hipMemcpy(base + off, v.data(), v.size() * sizeof(T), hipMemcpyHostToDevice) == hipSuccess;
}

int build_spectral(Plan* pl) {
  const Geom& g = pl->g;
  if (!g.spec) return DH_SUCCESS;
  const dh_params* p = &pl->params;
  const Layout& L = pl->L;
  for (int q = 0; q < p->pol_count; ++q) {
    const PolTables t = pol_tables(g, g.pol[q], p, q, true, exports(g, p));
    if (!upload(pl->mem, L.pol_xs[q], t.xs) || !upload(pl->mem, L.pol_ys[q], t.ys) ||
        (exports(g, p) && (!upload(pl->mem, L.pol_ex[q], t.ex) || !upload(pl->mem, L.pol_ey[q], t.ey))))
      return DH_ERR_ERROR;
  }
  return DH_SUCCESS;
}

// Device tables of the current parameters. hg: also the HG tables (a new
// waist); spec: also the spectral path tables (alignment trials, which run
// the field path, skip them).
int build_tables(Plan* pl, bool hg = true, bool spec = true) {
  ++pl->version;
  const Geom& g = pl->g;
  const dh_params* p = &pl->params;
  const Layout& L = pl->L;
  std::vector<char> host(L.total_tables, 0);
  put(host, L.tw_nx, twiddles(g.nx, g.gx));
  put(host, L.tw_ny, twiddles(g.ny, g.gy));
  put(host, L.tw_wx, twiddles(g.wx, dh::GenFft{}));
  put(host, L.tw_wy, twiddles(g.wy, dh::GenFft{}));
  std::vector<short2> modes;
  for (int gg = 0; gg < g.G; ++gg)
    for (int m = gg; m >= 0; --m) modes.push_back(make_short2((short)m, (short)(gg - m)));
  put(host, L.modes, modes);
  for (int q = 0; q < p->pol_count; ++q) {
    const PolTables t = pol_tables(g, g.pol[q], p, q, false, false);
    put(host, L.pol_mrow[q], t.mrow);
    put(host, L.pol_rhox[q], t.rhox);
    put(host, L.pol_rhoy[q], t.rhoy);
    put(host, L.pol_tx[q], t.tx);
    put(host, L.pol_ty[q], t.ty);
  }
  if (hipMemcpy(pl->mem, host.data(), L.total_tables, hipMemcpyHostToDevice) != hipSuccess) return DH_ERR_ERROR;
  if (spec) {
    const int e = build_spectral(pl);
    if (e != DH_SUCCESS) return e;
  }
  if (!hg) return DH_SUCCESS;
  const double waist = p->waist > 0 ? p->waist : 1.0;
  pl->s_uh = (float)hg_fp16_scale(waist, std::max(g.pxp, g.pyp));
  for (int q = 0; q < p->pol_count; ++q) {
    char* m = pl->mem;
    if (dh::launch_hg(g.pxp, g.wx, g.wx, waist, g.G, g.gp, (float*)(m + L.pol_ux[q]),
                      (unsigned short*)(m + L.pol_uxs[q][0]), (unsigned short*)(m + L.pol_uxs[q][1]),
                      (_Float16*)(m + L.pol_uxs[q][2]), (_Float16*)(m + L.pol_uxs[q][3]), pl->s_uh, 0) != hipSuccess)
      return DH_ERR_ERROR;
    if (dh::launch_hg(g.pyp, g.wy, g.wyp, waist, g.G, g.gp, (float*)(m + L.pol_uy[q]),
                      (unsigned short*)(m + L.pol_uys[q][0]), (unsigned short*)(m + L.pol_uys[q][1]),
                      (_Float16*)(m + L.pol_uys[q][2]), (_Float16*)(m + L.pol_uys[q][3]), pl->s_uh, 0) != hipSuccess)
      return DH_ERR_ERROR;
  }
  if (hipDeviceSynchronize() != hipSuccess) return DH_ERR_ERROR;
  return DH_SUCCESS;
}

// The tables an alignment trial changes, on stream s with no host sync: the
// per-pol window tables (mask rows, centre ramps, tilt/defocus phases) in one
// upload of their contiguous range and, for a new waist (hg), the HG tables.
// The twiddles and the mode list do not depend on the trial's parameters. The
// host image lives in the plan until the next trial, which starts after this
// one's results were read back (stream synchronised).
int trial_tables(Plan* pl, bool hg, hipStream_t s) {
  ++pl->version;
  const Geom& g = pl->g;
  const dh_params* p = &pl->params;
  const Layout& L = pl->L;
  const size_t lo = L.pol_mrow[0], len = L.total_tables - lo;
  pl->trial_host.assign(L.total_tables, 0);
  for (int q = 0; q < p->pol_count; ++q) {
    const PolTables t = pol_tables(g, g.pol[q], p, q, false, false);
    put(pl->trial_host, L.pol_mrow[q], t.mrow);
    put(pl->trial_host, L.pol_rhox[q], t.rhox);
    put(pl->trial_host, L.pol_rhoy[q], t.rhoy);
    put(pl->trial_host, L.pol_tx[q], t.tx);
    put(pl->trial_host, L.pol_ty[q], t.ty);
  }
  if (hipMemcpyAsync(pl->mem + lo, pl->trial_host.data() + lo, len, hipMemcpyHostToDevice, s) != hipSuccess)
    return DH_ERR_ERROR;
  if (!hg) return DH_SUCCESS;
  const double waist = p->waist > 0 ? p->waist : 1.0;
  pl->s_uh = (float)hg_fp16_scale(waist, std::max(g.pxp, g.pyp));
  for (int q = 0; q < p->pol_count; ++q) {
    char* m = pl->mem;
    if (dh::launch_hg(g.pxp, g.wx, g.wx, waist, g.G, g.gp, (float*)(m + L.pol_ux[q]),
                      (unsigned short*)(m + L.pol_uxs[q][0]), (unsigned short*)(m + L.pol_uxs[q][1]),
                      (_Float16*)(m + L.pol_uxs[q][2]), (_Float16*)(m + L.pol_uxs[q][3]), pl->s_uh, s) != hipSuccess)
      return DH_ERR_ERROR;
    if (dh::launch_hg(g.pyp, g.wy, g.wyp, waist, g.G, g.gp, (float*)(m + L.pol_uy[q]),
                      (unsigned short*)(m + L.pol_uys[q][0]), (unsigned short*)(m + L.pol_uys[q][1]),
                      (_Float16*)(m + L.pol_uys[q][2]), (_Float16*)(m + L.pol_uys[q][3]), pl->s_uh, s) != hipSuccess)
      return DH_ERR_ERROR;
  }
  return DH_SUCCESS;
}

void fill_kargs(Plan* pl, int w) {
  const Geom& g = pl->g;
  const dh_params* p = &pl->params;
  const Layout& L = pl->L;
  dh::KArgs& a = pl->ka[w];
  char* m = pl->mem;
  a.frame_w = p->frame_w; a.frame_h = p->frame_h; a.npol = p->pol_count;
  a.nx = g.nx; a.ny = g.ny; a.wx = g.wx; a.wy = g.wy; a.wyp = g.wyp;
  a.bx = g.bx; a.by = g.by; a.bxp = (g.bx + 15) / 16 * 16; a.G = g.G; a.gp = g.gp; a.nmodes = g.nmodes;
  a.gx = g.gx; a.gy = g.gy;
  a.nxny = (float)((double)g.nx * g.ny);
  a.prec = p->precision;
  a.s_uh = pl->s_uh;
  a.capt = nullptr;
  a.cell = g.pxp * g.pyp;
  a.fptr = nullptr;
  a.byp = g.byp;
  a.spow = (float)((double)g.wx * g.wy / (((double)g.nx * g.ny) * ((double)g.nx * g.ny)));
  for (int q = 0; q < p->pol_count; ++q) {
    const PolGeom& P = g.pol[q];
    dh::PolTab& t = a.pol[q];
    t.x0 = P.x0; t.y0 = P.y0;
    t.k0 = -P.uhi; t.ky0 = -P.vhi;
    t.bxq = P.uhi - P.ulo + 1; t.byq = P.vhi - P.vlo + 1;
    t.mrow = (const int2*)(m + L.pol_mrow[q]);
    t.rhox = (const float2*)(m + L.pol_rhox[q]);
    t.rhoy = (const float2*)(m + L.pol_rhoy[q]);
    t.tx = (const float2*)(m + L.pol_tx[q]);
    t.ty = (const float2*)(m + L.pol_ty[q]);
    t.ux = (const float*)(m + L.pol_ux[q]);
    t.uy = (const float*)(m + L.pol_uy[q]);
    t.ux_bh = (const unsigned short*)(m + L.pol_uxs[q][0]);
    t.ux_bl = (const unsigned short*)(m + L.pol_uxs[q][1]);
    t.ux_hh = (const _Float16*)(m + L.pol_uxs[q][2]);
    t.ux_hl = (const _Float16*)(m + L.pol_uxs[q][3]);
    t.uy_bh = (const unsigned short*)(m + L.pol_uys[q][0]);
    t.uy_bl = (const unsigned short*)(m + L.pol_uys[q][1]);
    t.uy_hh = (const _Float16*)(m + L.pol_uys[q][2]);
    t.uy_hl = (const _Float16*)(m + L.pol_uys[q][3]);
    t.xs = (const float2*)(m + L.pol_xs[q]);
    t.ys = (const float2*)(m + L.pol_ys[q]);
  }
  a.modes = (const short2*)(m + L.modes);
  a.tw_nx = (const float2*)(m + L.tw_nx);
  a.tw_ny = (const float2*)(m + L.tw_ny);
  a.tw_wx = (const float2*)(m + L.tw_wx);
  a.tw_wy = (const float2*)(m + L.tw_wy);
  a.t1 = (float2*)(m + L.t1[w]);
  a.f2 = (float2*)(m + L.f2[w]);
  a.partial = (float2*)(m + L.partial[w]);
  a.nblk = g.spec ? dh::spectral_blocks(g.ny, g.wy, g.bx, g.gp) : field_blocks(g);
  a.coefs = pl->omem ? (float2*)pl->omem : (float2*)(m + L.coefs);
  a.coefs_norm = pl->omem ? (float2*)(pl->omem + align256((size_t)pl->ocap * p->pol_count * g.nmodes * 8))
                          : (float2*)(m + L.coefs_norm);
  a.window = p->keep_window || exports(g, p) ? (float2*)(m + L.window) : nullptr;
  // the kernels write mode-1 fields; mode-0 fields come from the export
  a.fields = p->keep_fields && g.mode == 1 ? (float2*)(m + L.fields) : nullptr;
}

int set_err(Plan* pl, int e) {
  if (pl) pl->last_error = e;
  return e;
}

// IFFT mode 0: the fields of `count` output frames (first, first + stride,
// ...) from their kept windows, with wavelength lam's tables and geometry (lam
// < 0: the plan's): the window's bins zero-padded to the N_y x N_x grid and
// inverse transformed, y first (k_m0y, into the scratch, per group of frames)
// then x (k_m0x), with the tilt/defocus phase and 1/(Nx Ny) applied.
int export_fields(Plan* pl, int first, int count, int stride, int lam, hipStream_t s) {
  const Geom& g = pl->g;
  const int P = pl->params.pol_count;
  dh::M0Args m{};
  m.win = (const float2*)(pl->mem + pl->L.window);
  m.t2 = (float2*)(pl->mem + pl->L.export_t);
  m.fields = (float2*)(pl->mem + pl->L.fields);
  m.tw_nx = pl->ka[0].tw_nx;
  m.tw_ny = pl->ka[0].tw_ny;
  m.nx = g.nx; m.ny = g.ny; m.wx = g.wx; m.wy = g.wy; m.bxp = (g.bx + 15) / 16 * 16; m.npol = P;
  m.gx = g.gx; m.gy = g.gy;
  m.stride = stride;
  for (int q = 0; q < P; ++q) {
    const PolGeom& G = lam >= 0 ? pl->lam_geom[(size_t)lam * 2 + q] : g.pol[q];
    m.pol[q].uhi = G.uhi; m.pol[q].vhi = G.vhi;
    m.pol[q].bxq = G.uhi - G.ulo + 1; m.pol[q].byq = G.vhi - G.vlo + 1;
    const char* base = lam >= 0 ? pl->lmem : pl->mem;
    m.pol[q].phx = (const float2*)(base + (lam >= 0 ? pl->lam_tab[(size_t)lam * 2 + q].ex : pl->L.pol_ex[q]));
    m.pol[q].phy = (const float2*)(base + (lam >= 0 ? pl->lam_tab[(size_t)lam * 2 + q].ey : pl->L.pol_ey[q]));
  }
  const int grp = export_chunk(g, &pl->params, pl->max_batch);
  for (int c0 = 0; c0 < count; c0 += grp) {
    m.first = first + c0 * stride;
    const int nb = std::min(grp, count - c0);
    if (dh::launch_m0y(m, nb, s) != hipSuccess || dh::launch_m0x(m, nb, s) != hipSuccess) return DH_ERR_ERROR;
  }
  return DH_SUCCESS;
}

int copy_out(Plan* pl, void* host_out, size_t bytes, const void* dev) {
  if (!host_out) return DH_SUCCESS;
  if (hipStreamSynchronize(pl->last_stream) != hipSuccess) return DH_ERR_ERROR;
  if (hipMemcpy(host_out, dev, bytes, hipMemcpyDeviceToHost) != hipSuccess) return DH_ERR_ERROR;
  return DH_SUCCESS;
}

void release(Plan* pl) {
  int dev = 0;
  (void)hipGetDevice(&dev);
  (void)hipSetDevice(pl->device);
  (void)hipDeviceSynchronize();
  for (int w = 0; w < 4; ++w) {
    if (pl->str[w]) (void)hipStreamDestroy(pl->str[w]);
    if (pl->join[w]) (void)hipEventDestroy(pl->join[w]);
  }
  if (pl->fork) (void)hipEventDestroy(pl->fork);
  for (hipEvent_t e : pl->ev_pool) (void)hipEventDestroy(e);
  if (pl->mem) (void)hipFree(pl->mem);
  if (pl->amem) (void)hipFree(pl->amem);
  if (pl->tm_mem) (void)hipFree(pl->tm_mem);
  if (pl->q16_mem) (void)hipFree(pl->q16_mem);
  if (pl->bmem) (void)hipFree(pl->bmem);
  if (pl->omem) (void)hipFree(pl->omem);
  if (pl->lmem) (void)hipFree(pl->lmem);
  if (pl->smem) (void)hipFree(pl->smem);
  (void)hipSetDevice(dev);
  delete pl;
}

}  // namespace

extern "C" {

int dh_plan_check(const dh_params* p, int max_batch, dh_plan_info* info) {
  Geom g;
  const int e = derive(p, &g);
  if (e != DH_SUCCESS) return e;
  if (max_batch < 1) max_batch = 1;
  if (info) {
    std::memset(info, 0, sizeof(*info));
    const int chunk = chunk_for(g, p->pol_count, max_batch);
    const Layout L = layout(g, p, max_batch, chunk, streams_for(max_batch, chunk));
    info->fft_w = g.nx; info->fft_h = g.ny;
    info->ifft_w = g.wx; info->ifft_h = g.wy;
    info->box_w = g.bx; info->box_h = g.by;
    info->modes = g.nmodes;
    for (int q = 0; q < p->pol_count; ++q) {
      info->x0[q] = g.pol[q].x0; info->y0[q] = g.pol[q].y0;
      info->ax[q] = g.pol[q].ax; info->ay[q] = g.pol[q].ay;
    }
    info->rx = g.rx; info->ry = g.ry;
    info->pitch_x = g.pxp; info->pitch_y = g.pyp;
    info->device_bytes = L.total;
    info->chunk = chunk;
    info->path = g.spec ? DH_PATH_SPECTRAL : DH_PATH_FIELD;
    info->field_w = g.fx; info->field_h = g.fy;
    info->field_pitch_x = g.fpx; info->field_pitch_y = g.fpy;
    info->generic = (g.gx.np > 0 ? 1 : 0) | (g.gy.np > 0 ? 2 : 0);
  }
  return DH_SUCCESS;
}

int dh_max_window_radius(const dh_params* p, int wrap, double* radius_deg) {
  if (!p || !radius_deg) return DH_ERR_NULLPOINTER;
  if (p->pol_count != 1 && p->pol_count != 2) return DH_ERR_INVALIDPOLARISATION;
  if (!(p->pixel_size > 0) || !(p->wavelength > 0)) return DH_ERR_INVALIDARGUMENT;
  // angles in degrees (paraxial, as the tilt-to-bin mapping), where the
  // window is a circle; the spectrum spans +-w_max = lambda / (2 p) along each
  // axis and repeats with period 2 w_max when it wraps
  const double wmax = p->wavelength / (2.0 * p->pixel_size) / kDeg;
  double best = HUGE_VAL;
  for (int q = 0; q < p->pol_count; ++q) {
    const double tx = p->tilt_deg[q][0], ty = p->tilt_deg[q][1];
    if (!std::isfinite(tx) || !std::isfinite(ty)) return DH_ERR_INVALIDARGUMENT;
    double w;
    if (!wrap) {
      // clear of the autocorrelation terms at the origin (radius 2w) and inside the spectrum
      w = std::min(std::hypot(tx, ty) / 3.0, std::min(wmax - std::fabs(tx), wmax - std::fabs(ty)));
    } else {
      // the same gaps from every periodic image of the origin terms and of the conjugate term
      w = HUGE_VAL;
      const double per = 2.0 * wmax;
      for (int kx = -2; kx <= 2; ++kx)
        for (int ky = -2; ky <= 2; ++ky) {
          w = std::min(w, std::hypot(tx - kx * per, ty - ky * per) / 3.0);
          w = std::min(w, std::hypot(2.0 * tx - kx * per, 2.0 * ty - ky * per) / 2.0);
        }
    }
    best = std::min(best, w);
  }
  *radius_deg = std::max(best, 0.0);
  return DH_SUCCESS;
}

int dh_plan(const dh_params* p, int max_batch, size_t hbm_budget, dh_handle* out) {
  if (!p || !out) return DH_ERR_NULLPOINTER;
  Geom g;
  int e = derive(p, &g);
  if (e != DH_SUCCESS) return e;
  if (max_batch < 1) max_batch = 1;
  Plan* pl = new Plan();
  pl->params = *p;
  pl->params.fft_w = g.nx;
  pl->params.fft_h = g.ny;
  pl->g = g;
  pl->max_batch = max_batch;
  pl->chunk = chunk_for(g, p->pol_count, max_batch);
  pl->nws = streams_for(max_batch, pl->chunk);
  pl->L = layout(g, p, max_batch, pl->chunk, pl->nws);
  if (hbm_budget && pl->L.total > hbm_budget) {
    delete pl;
    return DH_ERR_MEMORYALLOCATION;
  }
  if (hipGetDevice(&pl->device) != hipSuccess || hipMalloc(&pl->mem, pl->L.total) != hipSuccess) {
    (void)hipGetLastError();
    delete pl;
    return DH_ERR_MEMORYALLOCATION;
  }
  e = build_tables(pl);
  if (e != DH_SUCCESS) {
    (void)hipFree(pl->mem);
    delete pl;
    return e;
  }
  for (int w = 0; w < pl->nws; ++w) fill_kargs(pl, w);
  if (pl->nws > 1) {
    bool ok = hipEventCreateWithFlags(&pl->fork, hipEventDisableTiming) == hipSuccess;
    for (int w = 0; w < pl->nws && ok; ++w)
      ok = hipStreamCreateWithFlags(&pl->str[w], hipStreamNonBlocking) == hipSuccess &&
           hipEventCreateWithFlags(&pl->join[w], hipEventDisableTiming) == hipSuccess;
    if (!ok) {
      release(pl);
      return DH_ERR_ERROR;
    }
  }
  std::lock_guard<std::mutex> lk(g_mu);
  g_plans.push_back(pl);
  *out = (dh_handle)(g_plans.size() - 1);
  return DH_SUCCESS;
}

namespace {

// the path over frames [b0, b0 + nb) with arguments a on stream st
bool launch_path(Plan* pl, const dh::KArgs& a, const void* frames, int u16, int b0, int nb, hipStream_t st) {
  bool ok = timed_event(pl, st, DH_STAGE_FFT, true) == hipSuccess &&
            dh::launch_row(a, frames, u16, b0, nb, st) == hipSuccess &&
            timed_event(pl, st, DH_STAGE_FFT, false) == hipSuccess &&
            timed_event(pl, st, DH_STAGE_CROP, true) == hipSuccess &&
            (pl->g.spec ? dh::launch_cspec(a, b0, nb, st) : dh::launch_col(a, b0, nb, st)) == hipSuccess &&
            timed_event(pl, st, DH_STAGE_CROP, false) == hipSuccess;
  if (ok && !pl->g.spec && (a.G > 0 || a.fields))
    ok = timed_event(pl, st, DH_STAGE_FIELD, true) == hipSuccess && dh::launch_fld(a, b0, nb, st) == hipSuccess &&
         timed_event(pl, st, DH_STAGE_FIELD, false) == hipSuccess;
  if (ok && a.G > 0)
    ok = timed_event(pl, st, DH_STAGE_NORM, true) == hipSuccess && dh::launch_norm(a, b0, nb, st) == hipSuccess &&
         timed_event(pl, st, DH_STAGE_NORM, false) == hipSuccess;
  return ok;
}

// A run of frames [b0, b0 + n) processed with one wavelength's tables (lam
// < 0: the plan's own) into the staging buffers (staged) or the outputs.
struct Seg {
  int b0, n, lam;
  bool staged;
};

// the segments' chunks round robin over the workspaces and internal streams,
// after the caller's prior work; the caller's stream continues after all
int run_segments(Plan* pl, const void* frames, const std::vector<Seg>& segs, hipStream_t s) {
  const int u16 = pl->params.input_dtype == DH_INPUT_U16;
  int nchunks = 0;
  for (const Seg& g : segs) nchunks += (g.n + pl->chunk - 1) / pl->chunk;
  const int nws = std::max(1, std::min(pl->nws, nchunks));
  if (nws > 1) {
    if (hipEventRecord(pl->fork, s) != hipSuccess) return DH_ERR_ERROR;
    for (int w = 0; w < nws; ++w)
      if (hipStreamWaitEvent(pl->str[w], pl->fork, 0) != hipSuccess) return DH_ERR_ERROR;
  }
  int c = 0;
  for (const Seg& sg : segs) {
    for (int b0 = sg.b0; b0 < sg.b0 + sg.n; b0 += pl->chunk, ++c) {
      const int nb = std::min(pl->chunk, sg.b0 + sg.n - b0);
      const int w = c % nws;
      dh::KArgs a = pl->ka[w];
      if (sg.staged) {
        a.fptr = pl->sptr;
        a.coefs = pl->sc;
        a.coefs_norm = pl->scn;
        a.window = pl->swin;
        a.fields = pl->sfld;
      }
      if (sg.lam >= 0) {
        for (int q = 0; q < pl->params.pol_count; ++q) {
          const PolGeom& P = pl->lam_geom[(size_t)sg.lam * 2 + q];
          const Plan::LamTab& t = pl->lam_tab[(size_t)sg.lam * 2 + q];
          dh::PolTab& pt = a.pol[q];
          pt.x0 = P.x0; pt.y0 = P.y0;
          pt.k0 = -P.uhi; pt.ky0 = -P.vhi;
          pt.bxq = P.uhi - P.ulo + 1; pt.byq = P.vhi - P.vlo + 1;
          pt.mrow = (const int2*)(pl->lmem + t.mrow);
          pt.rhox = (const float2*)(pl->lmem + t.rhox);
          pt.rhoy = (const float2*)(pl->lmem + t.rhoy);
          pt.tx = (const float2*)(pl->lmem + t.tx);
          pt.ty = (const float2*)(pl->lmem + t.ty);
          if (pl->g.spec) {
            pt.xs = (const float2*)(pl->lmem + t.xs);
            pt.ys = (const float2*)(pl->lmem + t.ys);
          }
        }
      }
      if (!launch_path(pl, a, frames, u16, b0, nb, nws > 1 ? pl->str[w] : s)) return DH_ERR_ERROR;
    }
  }
  if (nws > 1) {
    for (int w = 0; w < nws; ++w)
      if (hipEventRecord(pl->join[w], pl->str[w]) != hipSuccess || hipStreamWaitEvent(s, pl->join[w], 0) != hipSuccess)
        return DH_ERR_ERROR;
  }
  return DH_SUCCESS;
}

bool sweeping(const Plan* pl) { return pl->nlam > 0 || pl->avg > 1; }

// Wavelength sweep and/or averaging: the batch's batch * avg frames are
// staged wavelength by wavelength (position (w I + i) A + a for input i at
// wavelength w, repetition a), then combined into the outputs in the output
// ordering (the repetitions phase-aligned and averaged).
int process_sweep(Plan* pl, const void* frames, int batch, hipStream_t s) {
  const Geom& g = pl->g;
  const int P = pl->params.pol_count, L = std::max(pl->nlam, 1), A = pl->avg;
  if (!pl->smem) return DH_ERR_ERROR;
  if (batch % L) return DH_ERR_INVALIDDIMENSION;
  const int I = batch / L, n_in = batch * A;
  if (n_in > pl->max_batch) return DH_ERR_INVALIDDIMENSION;
  const size_t fbytes = (size_t)pl->params.frame_w * pl->params.frame_h *
                        (pl->params.input_dtype == DH_INPUT_U16 ? 2 : 4);
  const size_t plane = (size_t)g.wy * g.wx;
  if (dh::launch_fptr((const char*)frames, fbytes, batch, L, I, A, pl->avg_mode, pl->in_order, pl->sptr, s) !=
          hipSuccess ||
      (pl->swin && dh::launch_zero(pl->swin, (size_t)n_in * P * plane, s) != hipSuccess))
    return DH_ERR_ERROR;
  std::vector<Seg> segs;
  for (int w = 0; w < L; ++w) segs.push_back({w * I * A, I * A, pl->nlam > 0 ? w : -1, true});
  int e = run_segments(pl, frames, segs, s);
  if (e != DH_SUCCESS) return e;
  const dh::KArgs& a0 = pl->ka[0];
  const dh::Comb cb{L, I, A, pl->out_order};
  if (A > 1 && dh::launch_avg_rot(pl->swin, P * plane, cb, batch, pl->rot, s) != hipSuccess) return DH_ERR_ERROR;
  const double2* rot = A > 1 ? pl->rot : nullptr;
  if (g.G > 0 && dh::launch_comb_coefs(pl->sc, pl->scn, rot, P * g.nmodes, cb, batch, a0.coefs, a0.coefs_norm, s) !=
                     hipSuccess)
    return DH_ERR_ERROR;
  if (a0.window && dh::launch_comb_plane(pl->swin, rot, P * plane, cb, batch, a0.window, s) != hipSuccess)
    return DH_ERR_ERROR;
  if (pl->sfld && dh::launch_comb_plane(pl->sfld, rot, P * plane, cb, batch, (float2*)(pl->mem + pl->L.fields), s) !=
                      hipSuccess)
    return DH_ERR_ERROR;
  return DH_SUCCESS;
}

}  // namespace

namespace {
// Coefficient outputs for a batch larger than the plan's max_batch (the
// paper sizes its buffers by the batch count it is given): the raw and
// normalised coefficients, and the basis coefficients when a basis is set,
// move to an allocation for `batch` frames, made once and grown only when a
// larger batch comes. Not while the stream is being captured (no allocation
// there), nor for plans that keep windows or fields, sweep or average (their
// buffers stay at max_batch).
int grow_outputs(Plan* pl, int batch, hipStream_t s) {
  if (batch <= pl->max_batch || batch <= pl->ocap) return DH_SUCCESS;
  const dh_params& p = pl->params;
  if (p.keep_window || p.keep_fields || sweeping(pl)) return DH_ERR_INVALIDDIMENSION;
  hipStreamCaptureStatus cs = hipStreamCaptureStatusNone;
  if (hipStreamIsCapturing(s, &cs) != hipSuccess || cs != hipStreamCaptureStatusNone) return DH_ERR_INVALIDDIMENSION;
  const size_t P = p.pol_count, nm = pl->g.nmodes;
  const size_t cb = align256((size_t)batch * P * nm * 8), bb = align256((size_t)batch * P * pl->bout * 8);
  // work in flight may still write the old outputs
  if (hipDeviceSynchronize() != hipSuccess) return DH_ERR_ERROR;
  char* mem = nullptr;
  if (hipMalloc(&mem, 2 * cb + 2 * bb + 256) != hipSuccess) {
    (void)hipGetLastError();
    return DH_ERR_MEMORYALLOCATION;
  }
  if (pl->omem) (void)hipFree(pl->omem);
  pl->omem = mem;
  pl->ocap = batch;
  for (int w = 0; w < pl->nws; ++w) fill_kargs(pl, w);
  if (pl->basis != DH_BASIS_HG) {
    pl->bc = (float2*)(mem + 2 * cb);
    pl->bcn = (float2*)(mem + 2 * cb + bb);
  }
  return DH_SUCCESS;
}
}  // namespace

int dh_process_batch(dh_handle h, const void* frames, int batch, void* stream) {
  Plan* pl = get(h);
  if (!pl) return DH_ERR_INVALIDHANDLE;
  if (!frames) return set_err(pl, DH_ERR_NULLPOINTER);
  if (batch < 1) batch = 1;
  hipStream_t s = (hipStream_t)stream;
  if (batch > pl->max_batch) {
    const int e = grow_outputs(pl, batch, s);
    if (e != DH_SUCCESS) return set_err(pl, e);
  }
  const Geom& g = pl->g;
  const int P = pl->params.pol_count;
  if (sweeping(pl)) {
    const int e = process_sweep(pl, frames, batch, s);
    if (e != DH_SUCCESS) return set_err(pl, e);
  } else {
    const dh::KArgs& a0 = pl->ka[0];
    if (a0.window && dh::launch_zero(a0.window, (size_t)batch * a0.npol * a0.wy * a0.wx, s) != hipSuccess)
      return set_err(pl, DH_ERR_ERROR);
    if (run_segments(pl, frames, {{0, batch, -1, false}}, s) != DH_SUCCESS) return set_err(pl, DH_ERR_ERROR);
  }
  if (pl->basis != DH_BASIS_HG &&
      dh::launch_basis(pl->ka[0].coefs, pl->ka[0].coefs_norm, g.nmodes, pl->bin, pl->brng, pl->btt, pl->bout, pl->bc, pl->bcn,
                       batch * P, s) != hipSuccess)
    return set_err(pl, DH_ERR_ERROR);
  if (exports(g, &pl->params)) {
    // each output's fields from its window, with its wavelength's tables
    const int L = std::max(pl->nlam, 1), I = batch / L;
    for (int w = 0; w < L; ++w) {
      const bool fast = pl->nlam > 0 && pl->out_order == DH_WL_FAST;
      const int first = pl->nlam > 0 ? (fast ? w : w * I) : 0, count = pl->nlam > 0 ? I : batch;
      if (export_fields(pl, first, count, fast ? L : 1, pl->nlam > 0 ? w : -1, s) != DH_SUCCESS)
        return set_err(pl, DH_ERR_ERROR);
    }
  }
  pl->last_batch = batch;
  pl->last_stream = s;
  return set_err(pl, DH_SUCCESS);
}

int dh_mode_coefs(dh_handle h, dh_c64* host_out, const dh_c64** dev_out, int* batch, int* modes, int* pols,
                  int normalised) {
  Plan* pl = get(h);
  if (!pl) {
    if (batch) *batch = 0;
    if (modes) *modes = 0;
    if (pols) *pols = 0;
    if (dev_out) *dev_out = nullptr;
    return DH_ERR_INVALIDHANDLE;
  }
  const bool tr = pl->basis != DH_BASIS_HG;
  const int nm = tr ? pl->bout : pl->g.nmodes;
  if (batch) *batch = pl->last_batch;
  if (modes) *modes = nm;
  if (pols) *pols = pl->params.pol_count;
  const float2* src = tr ? (normalised ? pl->bcn : pl->bc) : (normalised ? pl->ka[0].coefs_norm : pl->ka[0].coefs);
  if (dev_out) *dev_out = nm > 0 ? (const dh_c64*)src : nullptr;
  if (nm == 0) return set_err(pl, DH_SUCCESS);
  const size_t bytes = (size_t)pl->last_batch * pl->params.pol_count * nm * sizeof(dh_c64);
  return set_err(pl, copy_out(pl, host_out, bytes, src));
}

// the plan's field buffer (mode 1: written by the kernels; mode 0: by the export)
static const float2* field_buffer(Plan* pl) {
  return pl->params.keep_fields ? (const float2*)(pl->mem + pl->L.fields) : nullptr;
}

static int get_plane(dh_handle h, bool win, dh_c64* host_out, const dh_c64** dev_out, int* batch, int* pols,
                     int* width, int* height) {
  Plan* pl = get(h);
  if (!pl) return DH_ERR_INVALIDHANDLE;
  const float2* src = win ? pl->ka[0].window : field_buffer(pl);
  const int w = win ? pl->g.wx : pl->g.fx, hgt = win ? pl->g.wy : pl->g.fy;
  if (batch) *batch = pl->last_batch;
  if (pols) *pols = pl->params.pol_count;
  if (width) *width = w;
  if (height) *height = hgt;
  if (dev_out) *dev_out = (const dh_c64*)src;
  if (!src) return set_err(pl, DH_ERR_ERROR);
  const size_t bytes = (size_t)pl->last_batch * pl->params.pol_count * w * hgt * sizeof(dh_c64);
  return set_err(pl, copy_out(pl, host_out, bytes, src));
}

int dh_get_window(dh_handle h, dh_c64* host_out, const dh_c64** dev_out, int* batch, int* pols, int* width,
                  int* height) {
  return get_plane(h, true, host_out, dev_out, batch, pols, width, height);
}

int dh_get_fields(dh_handle h, dh_c64* host_out, const dh_c64** dev_out, int* batch, int* pols, int* width,
                  int* height) {
  return get_plane(h, false, host_out, dev_out, batch, pols, width, height);
}

int dh_get_field_axes(dh_handle h, double* x, double* y, int* width, int* height) {
  Plan* pl = get(h);
  if (!pl) return DH_ERR_INVALIDHANDLE;
  const Geom& g = pl->g;
  if (width) *width = g.fx;
  if (height) *height = g.fy;
  for (int k = 0; x && k < g.fx; ++k) x[k] = (k - 0.5 * g.fx) * g.fpx;
  for (int l = 0; y && l < g.fy; ++l) y[l] = (l - 0.5 * g.fy) * g.fpy;
  return set_err(pl, DH_SUCCESS);
}

// Batch summary ("Analysis parameter types", digHoloBatchGetSummary). The
// eight sums of every plane (k_summ) are turned into the seven parameters on
// the host in FP64: with axis values (k + cx) dx and (l + cy) dy, dA = |dx dy|
// the axis cell, total power S dA, the centres of mass (cx + sum(k I)/S) dx
// and (cy + sum(l I)/S) dy, sqrt(max I) and its index l W + k, the effective
// area (S dA)^2 / (sum I^2 dA), and the wrap-aware y centre
// (cy + H arg(sum I e^{2 pi i l/H}) / (2 pi)) dy, the angle in [0, 2 pi). An
// all-zero plane gives zeros.
extern "C" int dh_batch_summary(dh_handle h, int plane, const void* frames, int batch, void* stream, float* params,
                                double* x_axis, double* y_axis, float* total_intensity, int* total_count, int* pols,
                                int* width, int* height) {
  Plan* pl = get(h);
  if (!pl) return DH_ERR_INVALIDHANDLE;
  if (plane != 0 && plane != 1) return set_err(pl, DH_ERR_INVALIDARGUMENT);
  const Geom& g = pl->g;
  const dh_params& p = pl->params;
  const int P = p.pol_count;
  const int W = plane == 0 ? g.nx / 2 + 1 : g.fx, H = plane == 0 ? g.ny : g.fy;
  if (plane == 1) batch = pl->last_batch;
  else if (batch < 1) batch = 1;
  const int total = batch + 1;
  if (total_count) *total_count = total;
  if (pols) *pols = P;
  if (width) *width = W;
  if (height) *height = H;
  // axes: degrees of paraxial angle (Fourier plane) or metres from the beam
  // centre (field plane, the values dh_get_field_axes gives): value (k + cx) dx
  double dx, dy, cx, cy;
  if (plane == 0) {
    dx = p.wavelength / (g.nx * p.pixel_size) / kDeg;
    dy = p.wavelength / (g.ny * p.pixel_size) / kDeg;
    cx = 0.0;
    cy = -(double)(g.ny / 2);
  } else {
    dx = g.fpx;
    dy = g.fpy;
    cx = -0.5 * g.fx;
    cy = -0.5 * g.fy;
  }
  for (int k = 0; x_axis && k < W; ++k) x_axis[k] = (k + cx) * dx;
  for (int l = 0; y_axis && l < H; ++l) y_axis[l] = (l + cy) * dy;
  if (!params && !total_intensity) return set_err(pl, DH_SUCCESS);
  const float2* fld = field_buffer(pl);
  if (plane == 1 && (!fld || pl->last_batch < 1)) return set_err(pl, DH_ERR_ERROR);
  if (plane == 0 && !frames) return set_err(pl, DH_ERR_NULLPOINTER);
  // the Fourier plane takes the compiled column transform of N_y
  if (plane == 0 && pl->g.gy.np > 0) return set_err(pl, DH_ERR_INVALIDDIMENSION);
  hipStream_t s = plane == 1 ? pl->last_stream : (hipStream_t)stream;
  // scratch: the sums, the summed intensity, and (Fourier plane) the half
  // plane of a group of frames: row pass over columns 0..Nx/2, column FFT
  const int bxe = g.nx / 2 + 1;
  const size_t per = (size_t)P * g.ny * bxe * 8;
  int grp = plane == 0 ? (int)std::max<size_t>(1, std::min<size_t>(batch, (256ull << 20) / per)) : 0;
  const size_t sb = align256((size_t)(batch + 1) * P * 8 * 8), mb = align256((size_t)P * W * H * 8);
  const size_t tb = align256((size_t)grp * per);
  char* mem = nullptr;
  if (hipMalloc(&mem, sb + mb + 2 * tb) != hipSuccess) {
    (void)hipGetLastError();
    return set_err(pl, DH_ERR_MEMORYALLOCATION);
  }
  double* sums = (double*)mem;
  double* map = (double*)(mem + sb);
  bool ok = true;
  if (plane == 1) {
    ok = dh::launch_summ(fld, nullptr, (long long)W * H, W, H, 1, W, batch * P, sums, s) == hipSuccess &&
         dh::launch_isum(fld, (long long)W * H, W, H, 1, W, batch, P, 0, map, s) == hipSuccess;
  } else {
    dh::KArgs ke = pl->ka[0];
    ke.bx = bxe;
    ke.t1 = (float2*)(mem + sb + mb);
    ke.fptr = nullptr;
    for (int q = 0; q < P; ++q) {
      ke.pol[q].k0 = 0;
      ke.pol[q].ky0 = -(g.ny / 2);
    }
    float2* spec = (float2*)(mem + sb + mb + tb);
    const int u16 = p.input_dtype == DH_INPUT_U16;
    for (int b0 = 0; ok && b0 < batch; b0 += grp) {
      const int nb = std::min(grp, batch - b0);
      ok = dh::launch_row(ke, frames, u16, b0, nb, s) == hipSuccess &&
           dh::launch_spec(ke, spec, g.ny, nb, s) == hipSuccess &&
           dh::launch_summ(spec, nullptr, (long long)bxe * g.ny, W, H, g.ny, 1, nb * P, sums + (size_t)b0 * P * 8,
                           s) == hipSuccess &&
           dh::launch_isum(spec, (long long)bxe * g.ny, W, H, g.ny, 1, nb, P, b0 > 0, map, s) == hipSuccess;
    }
  }
  ok = ok && dh::launch_summ(nullptr, map, (long long)W * H, W, H, 1, W, P, sums + (size_t)batch * P * 8, s) ==
                 hipSuccess;
  std::vector<double> hs((size_t)(batch + 1) * P * 8), hm(total_intensity ? (size_t)P * W * H : 0);
  ok = ok && hipMemcpyAsync(hs.data(), sums, hs.size() * 8, hipMemcpyDeviceToHost, s) == hipSuccess &&
       (!total_intensity || hipMemcpyAsync(hm.data(), map, hm.size() * 8, hipMemcpyDeviceToHost, s) == hipSuccess);
  const bool synced = hipStreamSynchronize(s) == hipSuccess;
  (void)hipFree(mem);
  if (!ok || !synced) return set_err(pl, DH_ERR_ERROR);
  const double da = std::fabs(dx * dy);
  for (int e = 0; e <= batch && params; ++e)
    for (int q = 0; q < P; ++q) {
      const double* t = &hs[((size_t)e * P + q) * 8];
      double v[DH_ANALYSIS_COUNT] = {0, 0, 0, 0, 0, 0, 0};
      int idx = 0;
      if (t[0] > 0.0) {
        v[DH_ANALYSIS_TOTALPOWER] = t[0] * da;
        v[DH_ANALYSIS_COMX] = (cx + t[1] / t[0]) * dx;
        v[DH_ANALYSIS_COMY] = (cy + t[2] / t[0]) * dy;
        v[DH_ANALYSIS_MAXABS] = std::sqrt(t[6]);
        idx = (int)t[7];
        v[DH_ANALYSIS_AEFF] = (t[0] * da) * (t[0] * da) / (t[3] * da);
        double ang = std::atan2(t[5], t[4]);
        if (ang < 0.0) ang += 2.0 * M_PI;
        if (ang >= 2.0 * M_PI) ang = 0.0;
        v[DH_ANALYSIS_COMYWRAP] = (cy + H * ang / (2.0 * M_PI)) * dy;
      }
      for (int k = 0; k < DH_ANALYSIS_COUNT; ++k) {
        float* o = params + ((size_t)k * P + q) * total + e;
        if (k == DH_ANALYSIS_MAXABSIDX)
          std::memcpy(o, &idx, sizeof(int));
        else
          *o = (float)v[k];
      }
    }
  for (size_t i = 0; i < hm.size(); ++i) total_intensity[i] = (float)hm[i];
  return set_err(pl, DH_SUCCESS);
}

int dh_get_params(dh_handle h, dh_params* out) {
  Plan* pl = get(h);
  if (!pl) return DH_ERR_INVALIDHANDLE;
  if (!out) return set_err(pl, DH_ERR_NULLPOINTER);
  *out = pl->params;
  return DH_SUCCESS;
}

int dh_get_plan_info(dh_handle h, dh_plan_info* out) {
  Plan* pl = get(h);
  if (!pl) return DH_ERR_INVALIDHANDLE;
  if (!out) return set_err(pl, DH_ERR_NULLPOINTER);
  const int e = dh_plan_check(&pl->params, pl->max_batch, out);
  if (e != DH_SUCCESS) return set_err(pl, e);
  // what the plan was built with (the environment may have changed since)
  out->chunk = pl->chunk;
  out->device_bytes = pl->L.total;
  return set_err(pl, DH_SUCCESS);
}

int dh_set_stage_timing(dh_handle h, int enabled) {
  Plan* pl = get(h);
  if (!pl) return DH_ERR_INVALIDHANDLE;
  if (hipDeviceSynchronize() != hipSuccess) return set_err(pl, DH_ERR_ERROR);
  pl->timing = enabled != 0;
  pl->ev_used = 0;
  pl->ev_stage.clear();
  return set_err(pl, DH_SUCCESS);
}

int dh_stage_times(dh_handle h, double* ms, int* launches) {
  Plan* pl = get(h);
  if (!pl) return DH_ERR_INVALIDHANDLE;
  if (!ms || !launches) return set_err(pl, DH_ERR_NULLPOINTER);
  for (int k = 0; k < DH_STAGE_COUNT; ++k) {
    ms[k] = 0.0;
    launches[k] = 0;
  }
  for (size_t i = 0; i < pl->ev_stage.size(); ++i) {
    float t = 0.f;
    if (hipEventSynchronize(pl->ev_pool[2 * i + 1]) != hipSuccess ||
        hipEventElapsedTime(&t, pl->ev_pool[2 * i], pl->ev_pool[2 * i + 1]) != hipSuccess)
      return set_err(pl, DH_ERR_ERROR);
    ms[pl->ev_stage[i]] += t;
    launches[pl->ev_stage[i]] += 1;
  }
  pl->ev_used = 0;
  pl->ev_stage.clear();
  return set_err(pl, DH_SUCCESS);
}

int dh_last_error(dh_handle h) {
  Plan* pl = get(h);
  return pl ? pl->last_error : DH_ERR_INVALIDHANDLE;
}

int dh_destroy(dh_handle h) {
  Plan* pl;
  {
    std::lock_guard<std::mutex> lk(g_mu);
    if (h < 0 || (size_t)h >= g_plans.size() || !g_plans[h]) return DH_ERR_INVALIDHANDLE;
    pl = g_plans[h];
    g_plans[h] = nullptr;
  }
  release(pl);
  return DH_SUCCESS;
}

}  // extern "C"

// ---------------------------------------------------------------------------
// Alignment (digHoloAutoAlign): snap + tweak of tilt, defocus and waist.
//
// Goal: captured power, 10 log10(sum |c|^2 / sum |E|^2 p'x p'y) over the
// batch and both polarisations: the share of the reconstructed field's power
// that the HG basis holds (0 dB when the field is exactly a combination of the
// modes; our reading of the paper's insertion-loss goal for one batch).
// The row pass and the column FFT run once over an extended box that covers
// every window position within the search margin; each trial re-runs only the
// window gather, the IFFTs and the overlap from the stored spectrum.
namespace {

double db10(double x) {
  if (!(x > 0.0)) return -HUGE_VAL;
  if (std::isinf(x)) return HUGE_VAL;
  return 10.0 * std::log10(x);
}

// The nine metrics of the transfer matrix of the B frames whose raw
// coefficients are in ka[0].coefs, on stream s (synchronises it). IL is the
// Gram matrix's trace over n (the sum of the s_k^2); only MDL needs the
// eigenvalues, and with eig = false (a goal other than MDL) the eigen-solver
// is skipped and out[MDL] is NaN.
int tm_compute(Plan* pl, int B, int pol_independent, int mul_conj_trans, hipStream_t s, double* out,
               bool eig = true) {
  const int P = pl->params.pol_count, M = pl->g.nmodes;
  if (B < 1 || M < 1) return DH_ERR_ERROR;
  const int MC = pl->basis != DH_BASIS_HG ? pl->bout : M;   // columns per pol of the matrix
  dh::TmArgs t{};
  t.grp = nullptr;
  t.c = pl->ka[0].coefs;
  t.modes = pl->ka[0].modes;
  t.B = B; t.P = P; t.M = M;
  if (pl->basis != DH_BASIS_HG) {
    // the matrix of the current basis: its coefficients made from the HG ones
    if (dh::launch_basis(pl->ka[0].coefs, pl->ka[0].coefs_norm, M, pl->bin, pl->brng, pl->btt, pl->bout, pl->bc, pl->bcn,
                         B * P, s) != hipSuccess)
      return DH_ERR_ERROR;
    t.c = pl->bc;
    t.M = pl->bout;
    t.grp = pl->bgrp;
    t.ngrp = pl->bngrp;
  }
  t.indep = pol_independent ? 1 : 0;
  t.rows = t.indep ? P * B : B;
  t.cols = P * MC;
  // singular values: eigenvalues of the smaller Gram matrix
  const int byrows = t.rows <= t.cols;
  const int n = byrows ? t.rows : t.cols;
  // the matrix of the diagonal metrics: A (rows x cols) or A A^H (rows x rows)
  const bool aa = mul_conj_trans != 0;
  const bool extra = aa && !byrows;            // A A^H besides the Gram of the SVD
  const int ncol = aa ? t.rows : t.cols;
  const int nd = std::min(t.rows, ncol);
  size_t o = 0;
  auto take = [&](size_t bytes) { size_t r = o; o += align256(bytes); return r; };
  const size_t og = take((size_t)n * n * 16), od = extra ? take((size_t)t.rows * t.rows * 16) : 0;
  // the results, one block for one copy to the host: eigenvalues [n], the
  // Gram's diagonal [n], row powers [rows], diagonal powers [nd], same-group
  // powers [nd], the solver's info
  const size_t nres = 2 * (size_t)n + t.rows + 2 * (size_t)nd + 1;
  const size_t ores = take(nres * 8);
  const size_t oe = ores, ogd = oe + (size_t)n * 8, orow = ogd + (size_t)n * 8;
  const size_t odg = orow + (size_t)t.rows * 8, osm = odg + (size_t)nd * 8, oi = osm + (size_t)nd * 8;
  if (o > pl->tm_bytes) {
    if (pl->tm_mem) (void)hipFree(pl->tm_mem);
    pl->tm_mem = nullptr;
    pl->tm_bytes = 0;
    if (hipMalloc(&pl->tm_mem, o) != hipSuccess) {
      (void)hipGetLastError();
      return DH_ERR_MEMORYALLOCATION;
    }
    pl->tm_bytes = o;
  }
  char* m = pl->tm_mem;
  double2* g = (double2*)(m + og);
  double2* gd = extra ? (double2*)(m + od) : g;
  // the row statistics read the Gram matrix before the eigen-solver overwrites it
  if (dh::launch_tm_gram(t, byrows, n, g, s) != hipSuccess ||
      (extra && dh::launch_tm_gram(t, 1, t.rows, gd, s) != hipSuccess) ||
      dh::launch_tm_rows(t, aa ? gd : nullptr, t.rows, ncol, nd, (double*)(m + orow), (double*)(m + odg),
                         (double*)(m + osm), s) != hipSuccess)
    return DH_ERR_ERROR;
  // the Gram's diagonal, read before the eigen-solver overwrites the matrix
  if (dh::launch_tm_diag(g, n, (double*)(m + ogd), s) != hipSuccess) return DH_ERR_ERROR;
  if (eig && dh::launch_heig(g, n, (double*)(m + oe), (int*)(m + oi), s) != hipSuccess) return DH_ERR_ERROR;
  std::vector<double> res(nres);
  if (hipMemcpyAsync(res.data(), m + ores, nres * 8, hipMemcpyDeviceToHost, s) != hipSuccess ||
      hipStreamSynchronize(s) != hipSuccess)
    return DH_ERR_ERROR;
  int info = 0;                          // the eigen-solver's status: -1 if the matrix was not finite
  if (eig) std::memcpy(&info, &res[nres - 1], sizeof(info));
  if (info < 0) return DH_ERR_ERROR;
  const double* eigv = res.data();
  const double* gdiag = eigv + n;
  const double* rowp = gdiag + n;
  const double* dg = rowp + t.rows;
  const double* sm = dg + nd;
  // IL = sum s_k^2 / n = trace / n; MDL from s^2 = the Gram's eigenvalues
  // (rounding can leave tiny negatives)
  double trace = 0.0;
  for (int i = 0; i < n; ++i) trace += gdiag[i];
  out[DH_METRIC_IL] = db10(trace / n);
  if (eig) {
    double smin = HUGE_VAL, smax = 0.0;
    for (int i = 0; i < n; ++i) {
      const double v = std::max(eigv[i], 0.0);
      smin = std::min(smin, v);
      smax = std::max(smax, v);
    }
    out[DH_METRIC_MDL] = smax > 0.0 ? db10(smin / smax) : -HUGE_VAL;
  } else {
    out[DH_METRIC_MDL] = std::nan("");
  }
  double total = 0.0, dsum = 0.0, ssame = 0.0, dmax = 0.0, dmin = HUGE_VAL, rmax = -1.0, rmin = HUGE_VAL;
  for (int i = 0; i < t.rows; ++i) total += rowp[i];
  for (int i = 0; i < nd; ++i) {
    dsum += dg[i];
    ssame += sm[i];
    dmax = std::max(dmax, dg[i]);
    dmin = std::min(dmin, dg[i]);
    const double off = rowp[i] - dg[i];
    const double r = off > 0.0 ? dg[i] / off : HUGE_VAL;
    rmax = std::max(rmax, r);
    rmin = std::min(rmin, r);
  }
  out[DH_METRIC_DIAG] = db10(dsum / nd);
  out[DH_METRIC_SNRAVG] = total > dsum ? db10(dsum / (total - dsum)) : HUGE_VAL;
  out[DH_METRIC_DIAGBEST] = db10(dmax);
  out[DH_METRIC_DIAGWORST] = db10(dmin);
  out[DH_METRIC_SNRBEST] = db10(rmax);
  out[DH_METRIC_SNRWORST] = db10(rmin);
  out[DH_METRIC_SNRMG] = total > ssame ? db10(ssame / (total - ssame)) : HUGE_VAL;
  return DH_SUCCESS;
}

struct AlignCtx {
  Plan* pl;
  hipStream_t s;
  int batch;
  const void* frames;
  int u16;
  int bxe, bye;
  int k0e[2], ky0e[2];
  int ox[2] = {0, 0}, oy[2] = {0, 0};   // window origins the stored spectrum was made at
  float2* t1e;
  float2* spec;
  double* capt;
  float2* fields = nullptr;             // set: trials also write the fields here
  int evals = 0;
};

// the extended row pass and column FFT of the batch at the plan's current
// window origins, stored as the resident spectrum
bool align_fft(AlignCtx& c) {
  Plan* pl = c.pl;
  dh::KArgs ke = pl->ka[0];
  ke.bx = c.bxe;
  ke.t1 = c.t1e;
  for (int q = 0; q < pl->params.pol_count; ++q) {
    ke.pol[q].k0 = c.k0e[q];
    ke.pol[q].ky0 = c.ky0e[q];
    c.ox[q] = pl->g.pol[q].x0;
    c.oy[q] = pl->g.pol[q].y0;
  }
  return dh::launch_row(ke, c.frames, c.u16, 0, c.batch, c.s) == hipSuccess &&
         dh::launch_spec(ke, c.spec, c.bye, c.batch, c.s) == hipSuccess;
}

// one trial with the plan's current parameters: per-pol mode and field power
// summed over the batch (FP64), or false if the window left the stored region
bool align_eval(AlignCtx& c, bool hg, double mp[2], double fp[2], bool readback = true) {
  Plan* pl = c.pl;
  Geom& g = pl->g;
  const int np = pl->params.pol_count;
  int offj[2] = {0, 0}, offi[2] = {0, 0};
  for (int q = 0; q < np; ++q) {
    if (derive_pol(&pl->params, &g, q) != DH_SUCCESS) return false;
    offj[q] = -g.pol[q].uhi - c.k0e[q];
    offi[q] = -g.pol[q].vhi - c.ky0e[q];
    if (offj[q] < 0 || offj[q] + g.bx > c.bxe || offi[q] < 0 || offi[q] + g.by > c.bye) return false;
  }
  // on a failure past this point the stream is drained first, so that no
  // pending upload of this trial lands after the caller's restoring rebuild
  auto fail = [&]() {
    (void)hipStreamSynchronize(c.s);
    return false;
  };
  if (trial_tables(pl, hg, c.s) != DH_SUCCESS) return fail();
  for (int w = 0; w < pl->nws; ++w) fill_kargs(pl, w);
  // a beam centre that moved the window by whole pixels needs the spectrum anew
  bool moved = false;
  for (int q = 0; q < np; ++q) moved |= g.pol[q].x0 != c.ox[q] || g.pol[q].y0 != c.oy[q];
  if (moved && !align_fft(c)) return fail();
  dh::KArgs k = pl->ka[0];
  k.capt = c.capt;
  k.fields = c.fields;
  k.nblk = field_blocks(g);      // trials run the field path
  const size_t per_frame = (size_t)np * c.bxe * c.bye;
  for (int b0 = 0; b0 < c.batch; b0 += pl->chunk) {
    const int nb = std::min(pl->chunk, c.batch - b0);
    if (dh::launch_gather(k, c.spec + b0 * per_frame, c.bxe, c.bye, offj, offi, nb, c.s) != hipSuccess ||
        dh::launch_fld(k, b0, nb, c.s) != hipSuccess || dh::launch_norm(k, b0, nb, c.s) != hipSuccess)
      return fail();
  }
  if (!readback) {   // the caller reads the trial's coefficients on the same stream
    ++c.evals;
    return true;
  }
  std::vector<double> h((size_t)c.batch * np * 2);
  if (hipMemcpyAsync(h.data(), c.capt, h.size() * 8, hipMemcpyDeviceToHost, c.s) != hipSuccess ||
      hipStreamSynchronize(c.s) != hipSuccess)
    return false;
  for (int q = 0; q < 2; ++q) mp[q] = fp[q] = 0.0;
  for (int b = 0; b < c.batch; ++b)
    for (int q = 0; q < np; ++q) {
      mp[q] += h[((size_t)b * np + q) * 2];
      fp[q] += h[((size_t)b * np + q) * 2 + 1];
    }
  ++c.evals;
  return true;
}

double db(double m, double f) { return (m > 0 && f > 0) ? 10.0 * std::log10(m / f) : -300.0; }

// The snap's first guess of the tilt from scratch (the paper's snap discards
// the current alignment and looks for the off-axis term in Fourier space):
// the power spectrum of each pol's whole FFT window summed over the first nb
// frames; bins inside the zero-order region (the ellipse of twice the window
// radius around the origin) are left out; the brightest other bin and its
// mirror are the two cross terms, and the one whose tilt (minus its bin) lies
// nearer the starting tilt is taken (from a zero start: positive x tilt, then
// positive y); its position is refined to the centroid of the power above the
// mean of the bins left in, over the window-radius ellipse around the
// brightest bin, with bin offsets taken periodically. tilt[q] in degrees.
// back to the parameters an alignment started from (its error paths): the
// geometry derived again, the tables rebuilt and the kernel arguments refilled
void restore(Plan* pl, const dh_params& start) {
  pl->params = start;
  for (int q = 0; q < start.pol_count; ++q) (void)derive_pol(&pl->params, &pl->g, q);
  (void)build_tables(pl);
  for (int w = 0; w < pl->nws; ++w) fill_kargs(pl, w);
}

constexpr int kSnapFrames = 32;   // frames the whole-plane snap sums

int snap_plane(Plan* pl, const void* frames, int nb, hipStream_t s, double tilt[2][2]) {
  const Geom& g = pl->g;
  const dh_params& p = pl->params;
  const int np = p.pol_count, nx = g.nx, ny = g.ny;
  const size_t plane = (size_t)nx * ny;
  const size_t tb = align256((size_t)nb * np * plane * 8), pb = align256((size_t)np * plane * 4);
  char* mem = nullptr;
  if (hipMalloc(&mem, 2 * tb + pb) != hipSuccess) {
    (void)hipGetLastError();
    return DH_ERR_MEMORYALLOCATION;
  }
  dh::KArgs ke = pl->ka[0];
  ke.bx = nx;
  ke.t1 = (float2*)mem;
  for (int q = 0; q < np; ++q) {
    ke.pol[q].k0 = 0;
    ke.pol[q].ky0 = 0;
  }
  float2* spec = (float2*)(mem + tb);
  float* pw = (float*)(mem + 2 * tb);
  std::vector<float> hp((size_t)np * plane);
  const bool ok = dh::launch_row(ke, frames, p.input_dtype == DH_INPUT_U16, 0, nb, s) == hipSuccess &&
                  dh::launch_spec(ke, spec, ny, nb, s) == hipSuccess &&
                  dh::launch_psum(spec, nb, np, plane, pw, s) == hipSuccess &&
                  hipMemcpyAsync(hp.data(), pw, hp.size() * 4, hipMemcpyDeviceToHost, s) == hipSuccess &&
                  hipStreamSynchronize(s) == hipSuccess;
  if (!ok) (void)hipStreamSynchronize(s);          // nothing still uses mem or hp when they go
  (void)hipFree(mem);
  if (!ok) {
    (void)hipGetLastError();
    return DH_ERR_ERROR;
  }
  const double binx = p.wavelength / (nx * p.pixel_size) / kDeg, biny = p.wavelength / (ny * p.pixel_size) / kDeg;
  auto sgn = [](int k, int n) { return k < n / 2 ? k : k - n; };        // signed bin of index k
  auto idx = [](int k, int n) { return ((k % n) + n) % n; };            // index of signed bin k
  for (int q = 0; q < np; ++q) {
    const float* m = hp.data() + (size_t)q * plane;                      // m[j * ny + i]: bin (j, i)
    double mean = 0.0;
    long cnt = 0;
    int pj = -1, pi = -1;
    float best = -1.f;
    for (int j = 0; j < nx; ++j)
      for (int i = 0; i < ny; ++i) {
        if (inside(sgn(j, nx), sgn(i, ny), 0.0, 0.0, 2.0 * g.rx, 2.0 * g.ry)) continue;
        const float v = m[(size_t)j * ny + i];
        mean += v;
        ++cnt;
        if (v > best) { best = v; pj = j; pi = i; }
      }
    if (pj < 0) return DH_ERR_INVALIDARGUMENT;
    mean /= (double)cnt;
    // the two cross terms: at bin b (tilt -b) and at -b (tilt b)
    const int bu = sgn(pj, nx), bv = sgn(pi, ny);
    const double t0x = p.tilt_deg[q][0], t0y = p.tilt_deg[q][1];
    const double d1 = std::hypot(-bu * binx - t0x, -bv * biny - t0y), d2 = std::hypot(bu * binx - t0x, bv * biny - t0y);
    bool first;
    if (d1 != d2) first = d1 < d2;
    else first = (-bu > 0) || (-bu == 0 && -bv > 0);
    const int cu = first ? bu : -bu, cv = first ? bv : -bv;            // the chosen term's bin
    const int hx = (int)std::ceil(g.rx), hy = (int)std::ceil(g.ry);
    double sw = 0.0, su = 0.0, sv = 0.0;
    for (int du = -hx; du <= hx; ++du)
      for (int dv = -hy; dv <= hy; ++dv) {
        if (!inside(du, dv, 0.0, 0.0, g.rx, g.ry)) continue;
        const double w = std::max(0.0, (double)m[(size_t)idx(cu + du, nx) * ny + idx(cv + dv, ny)] - mean);
        sw += w; su += w * du; sv += w * dv;
      }
    const double uc = cu + (sw > 0 ? su / sw : 0.0), vc = cv + (sw > 0 ? sv / sw : 0.0);
    tilt[q][0] = -uc * binx;
    tilt[q][1] = -vc * biny;
  }
  return DH_SUCCESS;
}

}  // namespace

extern "C" float dh_autoalign(dh_handle h, const void* frames, int batch, int mode, unsigned what, float tol,
                              void* stream) {
  Plan* pl = get(h);
  if (!pl) return -FLT_MAX;
  if (!frames) return (set_err(pl, DH_ERR_NULLPOINTER), -FLT_MAX);
  if (batch < 1) batch = 1;
  if (batch > pl->max_batch) return (set_err(pl, DH_ERR_INVALIDDIMENSION), -FLT_MAX);
  if (sweeping(pl) || mode < DH_ALIGN_FULL || mode > DH_ALIGN_ESTIMATE ||
      (what & ~(DH_ALIGN_TILT | DH_ALIGN_DEFOCUS | DH_ALIGN_WAIST | DH_ALIGN_CENTRE)) ||
      (mode != DH_ALIGN_ESTIMATE && pl->g.G == 0) || !(tol >= 0.f) ||
      pl->g.gp > dh::kMaxGpField)      // the trials run the field path's overlap (G <= 32)
    return (set_err(pl, DH_ERR_INVALIDARGUMENT), -FLT_MAX);
  // the snaps and trials run compiled kernels for every length
  if (pl->g.gx.np > 0 || pl->g.gy.np > 0 || !dh::sizes_supported(pl->g.nx, pl->g.ny, pl->g.wx, pl->g.wy))
    return (set_err(pl, DH_ERR_INVALIDDIMENSION), -FLT_MAX);
  hipStream_t s = (hipStream_t)stream;
  if (hipDeviceSynchronize() != hipSuccess) return (set_err(pl, DH_ERR_ERROR), -FLT_MAX);
  dh_params& P = pl->params;
  Geom& g = pl->g;
  const int np = P.pol_count;
  const double pix = P.pixel_size, lam = P.wavelength;
  const double binx = lam / (g.nx * pix) / kDeg, biny = lam / (g.ny * pix) / kDeg;   // one bin in degrees
  const dh_params start = P;
  dh_align_report rep{};
  // snap from scratch: the tilt of the off-axis term in the whole Fourier
  // plane, around which the stored spectrum is then made
  if (mode != DH_ALIGN_TWEAK && (what & DH_ALIGN_TILT)) {
    double t[2][2] = {{0.0, 0.0}, {0.0, 0.0}};
    const int e = snap_plane(pl, frames, std::min(batch, kSnapFrames), s, t);
    if (e != DH_SUCCESS) return (set_err(pl, e), -FLT_MAX);
    for (int q = 0; q < np; ++q)
      for (int a = 0; a < 2; ++a) P.tilt_deg[q][a] = rep.plane_tilt_deg[q][a] = t[q][a];
    for (int q = 0; q < np; ++q)
      if (derive_pol(&P, &g, q) != DH_SUCCESS)
        return (restore(pl, start), set_err(pl, DH_ERR_INVALIDARGUMENT), -FLT_MAX);
  }
  // search margin around the starting tilt: 0.6 w_c, within the spectrum
  const double mdeg = 0.6 * P.window_radius_deg;
  AlignCtx c{pl, s, batch, frames, P.input_dtype == DH_INPUT_U16};
  c.bxe = c.bye = 0;
  double tlo[2][2], thi[2][2];
  for (int q = 0; q < np; ++q) {
    const double ax = P.tilt_deg[q][0] / binx, ay = P.tilt_deg[q][1] / biny;
    const double mx = mdeg / binx, my = mdeg / biny;
    c.k0e[q] = (int)std::floor(ax - mx - g.rx) - 2;
    c.ky0e[q] = (int)std::floor(ay - my - g.ry) - 2;
    c.bxe = std::max(c.bxe, (int)std::ceil(ax + mx + g.rx) + 2 - c.k0e[q] + 1);
    c.bye = std::max(c.bye, (int)std::ceil(ay + my + g.ry) + 2 - c.ky0e[q] + 1);
    tlo[q][0] = P.tilt_deg[q][0] - mdeg; thi[q][0] = P.tilt_deg[q][0] + mdeg;
    tlo[q][1] = P.tilt_deg[q][1] - mdeg; thi[q][1] = P.tilt_deg[q][1] + mdeg;
  }
  if (c.bxe >= g.nx || c.bye >= g.ny) return (restore(pl, start), set_err(pl, DH_ERR_INVALIDARGUMENT), -FLT_MAX);
  // beam-centre search range: an eighth of the FFT window around the start,
  // and centres whose window stays inside the frame (the window's centre pixel
  // is the centre rounded to the nearest pixel, offset from the half-frame's)
  const double cmx = (g.nx / 8) * pix, cmy = (g.ny / 8) * pix;
  auto clamp_centre = [&](int q, int a, double v) {
    const double c0 = start.beam_centre[q][a], m = a ? cmy : cmx;
    const int half = P.frame_w / np;
    const int base = a ? P.frame_h / 2 - g.ny / 2 : q * half + half / 2 - g.nx / 2;   // origin at pixel 0
    const int n = a ? g.ny : g.nx, extent = a ? P.frame_h : P.frame_w;
    const double lo = (-base - 0.5) * pix, hi = (extent - n - base + 0.499) * pix;
    return std::min(std::min(c0 + m, hi), std::max(std::max(c0 - m, lo), v));
  };
  // the snap estimates centre and waist from the fields (with modes to fit)
  const bool snap_field =
      mode != DH_ALIGN_TWEAK && (what & (DH_ALIGN_CENTRE | DH_ALIGN_WAIST | DH_ALIGN_DEFOCUS)) && g.G > 0;
  // scratch: extended row pass, stored spectrum, power map, captured power,
  // and for the field snap the fields and their moments
  const size_t t1b = align256((size_t)batch * np * c.bxe * g.ny * 8);
  const size_t spb = align256((size_t)batch * np * c.bxe * c.bye * 8);
  const size_t pwb = align256((size_t)np * c.bxe * c.bye * 4);
  const size_t cpb = align256((size_t)batch * np * 2 * 8);
  const size_t fdb = snap_field ? align256((size_t)batch * np * g.wx * g.wy * 8) : 0;
  const size_t mob = snap_field ? align256((size_t)batch * np * 5 * 8) : 0;
  const size_t need = t1b + spb + pwb + cpb + fdb + mob;
  if (need > pl->amem_bytes) {
    if (pl->amem) (void)hipFree(pl->amem);
    pl->amem = nullptr;
    pl->amem_bytes = 0;
    if (hipMalloc(&pl->amem, need) != hipSuccess) {
      (void)hipGetLastError();
      return (restore(pl, start), set_err(pl, DH_ERR_MEMORYALLOCATION), -FLT_MAX);
    }
    pl->amem_bytes = need;
  }
  c.t1e = (float2*)pl->amem;
  c.spec = (float2*)(pl->amem + t1b);
  float* pw = (float*)(pl->amem + t1b + spb);
  c.capt = (double*)(pl->amem + t1b + spb + pwb);
  float2* fdev = (float2*)(pl->amem + t1b + spb + pwb + cpb);
  double* mdev = (double*)(pl->amem + t1b + spb + pwb + cpb + fdb);
  if (!align_fft(c)) return (restore(pl, start), set_err(pl, DH_ERR_ERROR), -FLT_MAX);
  // the batch power spectrum over the stored box (tilt and defocus snaps)
  const size_t plane = (size_t)c.bxe * c.bye;
  std::vector<float> hp;
  if (mode != DH_ALIGN_TWEAK && (what & (DH_ALIGN_TILT | DH_ALIGN_DEFOCUS))) {
    hp.resize(np * plane);
    if (dh::launch_psum(c.spec, batch, np, plane, pw, s) != hipSuccess ||
        hipMemcpyAsync(hp.data(), pw, hp.size() * 4, hipMemcpyDeviceToHost, s) != hipSuccess ||
        hipStreamSynchronize(s) != hipSuccess)
      return (restore(pl, start), set_err(pl, DH_ERR_ERROR), -FLT_MAX);
  }
  // snap: tilt at the centroid of the batch power spectrum above its mean
  if (mode != DH_ALIGN_TWEAK && (what & DH_ALIGN_TILT)) {
    for (int q = 0; q < np; ++q) {
      const float* m = hp.data() + q * plane;
      double mean = 0.0;
      for (size_t e = 0; e < plane; ++e) mean += m[e];
      mean /= (double)plane;
      double sw = 0.0, sj = 0.0, si = 0.0;
      for (int j = 0; j < c.bxe; ++j)
        for (int i = 0; i < c.bye; ++i) {
          const double w = std::max(0.0, (double)m[(size_t)j * c.bye + i] - mean);
          sw += w; sj += w * j; si += w * i;
        }
      if (sw > 0) {
        P.tilt_deg[q][0] = std::min(thi[q][0], std::max(tlo[q][0], (c.k0e[q] + sj / sw) * binx));
        P.tilt_deg[q][1] = std::min(thi[q][1], std::max(tlo[q][1], (c.ky0e[q] + si / sw) * biny));
      }
      rep.snap_tilt_deg[q][0] = P.tilt_deg[q][0];
      rep.snap_tilt_deg[q][1] = P.tilt_deg[q][1];
    }
  }
  // locked parameters take the first polarisation's value
  if (np > 1) {
    if (pl->lock & DH_ALIGN_TILT) for (int a = 0; a < 2; ++a) P.tilt_deg[1][a] = P.tilt_deg[0][a];
    if (pl->lock & DH_ALIGN_DEFOCUS) P.defocus[1] = P.defocus[0];
  }
  double mp[2] = {0.0, 0.0}, fp[2] = {0.0, 0.0};
  if (snap_field) {
    // snap of the beam centre (intensity centroid of the reconstructed fields)
    // and of the waist (pooled central second moment, read as the power spread
    // evenly over the modes of G groups: <x^2> = <y^2> = w^2 (2G + 1) / 12)
    c.fields = fdev;
    const bool ok = align_eval(c, true, mp, fp);
    c.fields = nullptr;
    std::vector<double> hm((size_t)batch * np * 5);
    if (!ok || dh::launch_moments(fdev, batch * np, g.wx, g.wy, g.pxp, g.pyp, mdev, s) != hipSuccess ||
        hipMemcpyAsync(hm.data(), mdev, hm.size() * 8, hipMemcpyDeviceToHost, s) != hipSuccess ||
        hipStreamSynchronize(s) != hipSuccess)
      return (restore(pl, start), set_err(pl, DH_ERR_ERROR), -FLT_MAX);
    double mom[2][5] = {};
    for (int b = 0; b < batch; ++b)
      for (int q = 0; q < np; ++q)
        for (int t = 0; t < 5; ++t) mom[q][t] += hm[((size_t)b * np + q) * 5 + t];
    double mxx = 0.0, myy = 0.0, tot = 0.0;
    for (int q = 0; q < np; ++q) {
      const double* m = mom[q];
      if (!(m[0] > 0.0)) continue;
      if (what & DH_ALIGN_CENTRE) {
        P.beam_centre[q][0] = clamp_centre(q, 0, P.beam_centre[q][0] + m[1] / m[0]);
        P.beam_centre[q][1] = clamp_centre(q, 1, P.beam_centre[q][1] + m[2] / m[0]);
      }
      mxx += m[3] - m[1] * m[1] / m[0];
      myy += m[4] - m[2] * m[2] / m[0];
      tot += m[0];
    }
    if ((what & DH_ALIGN_WAIST) && tot > 0.0 && mxx + myy > 0.0)
      P.waist = std::min(4.0 * start.waist, std::max(0.25 * start.waist,
                                                     std::sqrt(6.0 * (mxx + myy) / tot / (2 * g.G + 1))));
    for (int q = 0; q < np; ++q) {
      rep.snap_centre[q][0] = P.beam_centre[q][0];
      rep.snap_centre[q][1] = P.beam_centre[q][1];
    }
    rep.snap_waist = P.waist;
    if (what & DH_ALIGN_DEFOCUS) {
      // defocus magnitude per pol (reading 30): the spread of the window's
      // power in angle beyond what the modes of G groups hold at the waist,
      // over the spread of the field's intensity in space; the sign (and
      // the start value) by one trial each, kept per pol by its captured power
      double dmag[2] = {0.0, 0.0};
      for (int q = 0; q < np; ++q) {
        const double* m = mom[q];
        const double sx = m[0] > 0.0 ? (m[3] - m[1] * m[1] / m[0]) / m[0] : 0.0;
        const double sy = m[0] > 0.0 ? (m[4] - m[2] * m[2] / m[0]) / m[0] : 0.0;
        const double ax = P.tilt_deg[q][0] / binx, ay = P.tilt_deg[q][1] / biny;
        const float* hq = hp.data() + (size_t)q * plane;
        double w0 = 0.0, wt = 0.0, ws = 0.0, wtt = 0.0, wss = 0.0;
        for (int j = 0; j < c.bxe; ++j)
          for (int i = 0; i < c.bye; ++i) {
            const double t = c.k0e[q] + j, u = c.ky0e[q] + i;     // tilt bins of the stored (mirror) term
            if (!inside(-t, -u, ax, ay, g.rx, g.ry)) continue;
            const double w = hq[(size_t)j * c.bye + i];
            w0 += w; wt += w * t; ws += w * u; wtt += w * t * t; wss += w * u * u;
          }
        if (!(w0 > 0.0) || !(sx + sy > 0.0)) continue;
        const double kx = 2.0 * kPi / (g.nx * pix), ky = 2.0 * kPi / (g.ny * pix);
        const double k2 = kx * kx * (wtt / w0 - (wt / w0) * (wt / w0)) + ky * ky * (wss / w0 - (ws / w0) * (ws / w0));
        const double k2s = 2.0 * (2 * g.G + 1) / (3.0 * P.waist * P.waist);
        const double a2 = std::max(0.0, (k2 - k2s) / (sx + sy));
        dmag[q] = std::sqrt(a2) * lam / (2.0 * kPi);
      }
      double best[2] = {-HUGE_VAL, -HUGE_VAL}, keep[2] = {P.defocus[0], np > 1 ? P.defocus[1] : 0.0};
      const double d0[2] = {P.defocus[0], np > 1 ? P.defocus[1] : 0.0};
      for (int k = 0; k < 3; ++k) {
        for (int q = 0; q < np; ++q) P.defocus[q] = k == 0 ? d0[q] : (k == 1 ? dmag[q] : -dmag[q]);
        // the first trial also builds the HG tables of the snapped waist
        if (!align_eval(c, k == 0, mp, fp)) return (restore(pl, start), set_err(pl, DH_ERR_ERROR), -FLT_MAX);
        for (int q = 0; q < np; ++q) {
          const double v = db(mp[q], fp[q]);
          if (v > best[q]) { best[q] = v; keep[q] = P.defocus[q]; }
        }
      }
      for (int q = 0; q < np; ++q) {
        P.defocus[q] = keep[q];
        rep.snap_defocus[q] = dmag[q];
      }
      if (np > 1 && (pl->lock & DH_ALIGN_DEFOCUS)) P.defocus[1] = P.defocus[0];
    }
  }
  if (pl->g.G == 0) {  // estimate only, nothing to evaluate
    for (int q = 0; q < np; ++q) derive_pol(&P, &g, q);
    if (build_tables(pl, false) != DH_SUCCESS) return (set_err(pl, DH_ERR_ERROR), -FLT_MAX);
    rep.goal = pl->goal;
    pl->rep = rep;
    set_err(pl, DH_SUCCESS);
    return 0.f;
  }
  // goal: captured power (per pol and joint), or one transfer-matrix metric
  // of the batch's coefficients (joint only)
  const bool metric_goal = pl->goal >= 0;
  auto captured = [&]() { return db(mp[0] + (np > 1 ? mp[1] : 0.0), fp[0] + (np > 1 ? fp[1] : 0.0)); };
  // a metric goal reads the trial's coefficients in tm_compute; the captured
  // powers are read back only where they are used (capt)
  auto eval_goal = [&](bool hg, double& gv, bool capt = false) -> bool {
    if (!align_eval(c, hg, mp, fp, !metric_goal || capt)) return false;
    if (!metric_goal) {
      gv = captured();
      return true;
    }
    double m[DH_METRIC_COUNT];
    if (tm_compute(pl, c.batch, pl->goal_indep, pl->goal_aa, s, m, pl->goal == DH_METRIC_MDL) != DH_SUCCESS) {
      (void)hipStreamSynchronize(s);   // the trial's uploads land before any restoring rebuild
      return false;
    }
    gv = std::max(-1000.0, std::min(1000.0, m[pl->goal]));   // finite for the parabola
    return true;
  };
  double goal;
  if (!eval_goal(true, goal)) return (restore(pl, start), set_err(pl, DH_ERR_ERROR), -FLT_MAX);
  double best_pol[2] = {db(mp[0], fp[0]), np > 1 ? db(mp[1], fp[1]) : 0.0};
  rep.start_goal_db = goal;
  // tweak: coordinate search, a parabola through three trials per coordinate.
  // A coordinate is one parameter kind along one axis and takes one of three
  // forms: every pol its own value, each on its own captured power (captured
  // goal: a pol's power depends only on its own tilt, defocus and centre);
  // one pol's value on the joint goal (metric goals couple the pols); or one
  // value shared by all pols on the joint goal (the waist, locked parameters).
  if (mode != DH_ALIGN_ESTIMATE) {
    enum { TILT, DEFOCUS, WAIST, CENTRE };
    enum { PER_POL = -2, SHARED = -1 };
    struct Coord { int kind; int axis; int pol; double h; };
    std::vector<Coord> coords;
    auto add = [&](int kind, int axis, double h, bool locked) {
      if (kind == WAIST || (locked && np > 1)) coords.push_back({kind, axis, SHARED, h});
      else if (!metric_goal) coords.push_back({kind, axis, PER_POL, h});
      else for (int q = 0; q < np; ++q) coords.push_back({kind, axis, q, h});
    };
    const bool lt = pl->lock & DH_ALIGN_TILT, ld = pl->lock & DH_ALIGN_DEFOCUS;
    if (what & DH_ALIGN_TILT) { add(TILT, 0, 0.5 * binx, lt); add(TILT, 1, 0.5 * biny, lt); }
    if (what & DH_ALIGN_CENTRE) { add(CENTRE, 0, 0.5 * pix, false); add(CENTRE, 1, 0.5 * pix, false); }
    if (what & DH_ALIGN_DEFOCUS) add(DEFOCUS, 0, 0.02, ld);
    if (what & DH_ALIGN_WAIST) add(WAIST, 0, 0.03 * P.waist, false);
    auto get = [&](const Coord& k, int q) -> double& {
      switch (k.kind) {
        case TILT: return P.tilt_deg[q][k.axis];
        case DEFOCUS: return P.defocus[q];
        case CENTRE: return P.beam_centre[q][k.axis];
        default: return P.waist;
      }
    };
    auto clampv = [&](const Coord& k, int q, double v) {
      if (k.kind == TILT) return std::min(thi[q][k.axis], std::max(tlo[q][k.axis], v));
      if (k.kind == CENTRE) return clamp_centre(q, k.axis, v);
      if (k.kind == WAIST) return std::max(0.25 * start.waist, v);
      return v;
    };
    for (int sweep = 0; sweep < 60 && !coords.empty(); ++sweep) {
      const double goal0 = goal;
      for (Coord& k : coords) {
        const bool joint = k.pol != PER_POL;
        const int nv = joint ? 1 : np;                       // values this coordinate moves
        auto pol_of = [&](int i) { return joint ? std::max(k.pol, 0) : i; };
        auto set = [&](int i, double v) {
          if (k.pol == SHARED) for (int q = 0; q < np; ++q) get(k, q) = v;
          else get(k, pol_of(i)) = v;
        };
        const bool hg = k.kind == WAIST;
        double x0[2], f0[2], fm[2], fpl[2], last[2];
        for (int i = 0; i < nv; ++i) x0[i] = get(k, pol_of(i));
        auto trial = [&](const double* v, double* out) -> bool {
          for (int i = 0; i < nv; ++i) set(i, last[i] = v[i]);
          if (joint) return eval_goal(hg, out[0]);
          if (!align_eval(c, false, mp, fp)) return false;
          for (int q = 0; q < nv; ++q) out[q] = db(mp[q], fp[q]);
          return true;
        };
        for (int i = 0; i < nv; ++i) f0[i] = joint ? goal : best_pol[i];
        double vp[2], vm[2];
        for (int i = 0; i < nv; ++i) {
          vp[i] = clampv(k, pol_of(i), x0[i] + k.h);
          vm[i] = clampv(k, pol_of(i), x0[i] - k.h);
        }
        bool okp = trial(vp, fpl), okm = trial(vm, fm);
        double vn[2], fn[2];
        for (int i = 0; i < nv; ++i) {
          if (!okp) fpl[i] = -1e300;
          if (!okm) fm[i] = -1e300;
          const double cv = fpl[i] + fm[i] - 2.0 * f0[i];
          double d;
          if (okp && okm && cv < 0) d = 0.5 * k.h * (fm[i] - fpl[i]) / cv;
          else d = (fpl[i] > fm[i]) ? 2.0 * k.h : -2.0 * k.h;
          d = std::max(-2.0 * k.h, std::min(2.0 * k.h, d));
          vn[i] = clampv(k, pol_of(i), x0[i] + d);
        }
        const bool okn = trial(vn, fn);
        // keep the best of the four trials per value; the step grows when the
        // best trial is the far one and shrinks when no trial beat the centre
        bool moved = false, far = false, stale = false;
        for (int i = 0; i < nv; ++i) {
          double bv = x0[i], bf = f0[i];
          if (okp && fpl[i] > bf) { bv = vp[i]; bf = fpl[i]; }
          if (okm && fm[i] > bf) { bv = vm[i]; bf = fm[i]; }
          if (okn && fn[i] > bf) { bv = vn[i]; bf = fn[i]; }
          set(i, bv);
          if (joint) goal = bf; else best_pol[i] = bf;
          moved |= bv != x0[i];
          far |= std::fabs(bv - x0[i]) > 1.5 * k.h;
          stale |= !(okn && bv == last[i]);
        }
        k.h *= far ? 2.0 : moved ? 1.0 : 0.5;
        if (!joint) {
          // the kept per-pol values come from different trials: the joint goal anew
          if (!align_eval(c, false, mp, fp)) return (restore(pl, start), set_err(pl, DH_ERR_ERROR), -FLT_MAX);
          goal = captured();
        } else {
          // the HG tables of a waist step must not be left at a rejected
          // trial; per-pol powers follow every shared step
          if (stale && (hg || !metric_goal)) {
            double gv;
            if (!eval_goal(hg, gv)) return (restore(pl, start), set_err(pl, DH_ERR_ERROR), -FLT_MAX);
          }
          if (!metric_goal) for (int q = 0; q < np; ++q) best_pol[q] = db(mp[q], fp[q]);
        }
      }
      rep.sweeps = sweep + 1;
      if (sweep >= 1 && goal - goal0 < tol) break;
    }
  }
  // leave the plan at the final parameters with complete tables; all the
  // metrics of the final coefficients go in the report
  if (!eval_goal(true, goal, true) || build_spectral(pl) != DH_SUCCESS ||
      tm_compute(pl, c.batch, pl->goal_indep, pl->goal_aa, s, rep.metrics) != DH_SUCCESS)
    return (restore(pl, start), set_err(pl, DH_ERR_ERROR), -FLT_MAX);
  for (int w = 0; w < pl->nws; ++w) fill_kargs(pl, w);
  rep.goal = pl->goal;
  rep.goal_db = goal;
  rep.captured = std::pow(10.0, captured() / 10.0);
  rep.evaluations = c.evals;
  pl->rep = rep;
  pl->last_batch = batch;
  pl->last_stream = s;
  set_err(pl, DH_SUCCESS);
  return (float)goal;
}

extern "C" int dh_transfer_metrics(dh_handle h, int pol_independent, int mul_conj_trans, double* out) {
  Plan* pl = get(h);
  if (!pl) return DH_ERR_INVALIDHANDLE;
  if (!out) return set_err(pl, DH_ERR_NULLPOINTER);
  return set_err(pl, tm_compute(pl, pl->last_batch, pol_independent, mul_conj_trans, pl->last_stream, out));
}

extern "C" int dh_hermitian_eigenvalues(const double* a_host, int n, double* w_host, void* stream) {
  if (!a_host || !w_host) return DH_ERR_NULLPOINTER;
  if (n < 1 || n > 2048) return DH_ERR_INVALIDDIMENSION;
  hipStream_t s = (hipStream_t)stream;
  const size_t mb = align256((size_t)n * n * 16), wb = align256((size_t)n * 8);
  char* mem = nullptr;
  if (hipMalloc(&mem, mb + wb + 256) != hipSuccess) {
    (void)hipGetLastError();
    return DH_ERR_MEMORYALLOCATION;
  }
  std::vector<double> w(n);
  int info = -1;
  const bool ok = hipMemcpyAsync(mem, a_host, (size_t)n * n * 16, hipMemcpyHostToDevice, s) == hipSuccess &&
                  dh::launch_heig((double2*)mem, n, (double*)(mem + mb), (int*)(mem + mb + wb), s) == hipSuccess &&
                  hipMemcpyAsync(w.data(), mem + mb, (size_t)n * 8, hipMemcpyDeviceToHost, s) == hipSuccess &&
                  hipMemcpyAsync(&info, mem + mb + wb, sizeof(int), hipMemcpyDeviceToHost, s) == hipSuccess &&
                  hipStreamSynchronize(s) == hipSuccess;
  if (!ok) (void)hipStreamSynchronize(s);          // nothing still reads mem when it is freed
  (void)hipFree(mem);
  if (!ok) {
    (void)hipGetLastError();
    return DH_ERR_ERROR;
  }
  if (info < 0) return DH_ERR_ERROR;
  std::memcpy(w_host, w.data(), (size_t)n * 8);     // ascending, as the kernel writes them
  return DH_SUCCESS;
}

// ---------------------------------------------------------------------------
// dh_hermitian_eigenvalues_noalloc: the same eigen step with the working copy
// of the matrix in a fixed device array instead of an allocation. Every GPU
// the library runs on holds its own copy of `scratch` (the matrix, up to
// DH_NOALLOC_EIG_MAX_N rows, then the solver's info word) until the process
// ends; host code reaches it only through the device address that
// hipGetSymbolAddress returns on that device, looked up once per device on
// the first call there. Calls on one GPU share the array: calls that overlap
// on one GPU race. The matrix copy and the info word are rewritten by every
// call, so nothing has to start at zero.
namespace {
constexpr size_t kNoAllocMat = (size_t)DH_NOALLOC_EIG_MAX_N * DH_NOALLOC_EIG_MAX_N;
__device__ __align__(256) double2 scratch[kNoAllocMat + 16];

std::mutex g_scratch_mu;
std::map<int, double2*> g_scratch_ptr;     // device ordinal -> device address of scratch

// scratch's device address on the current device (looked up on first use)
double2* scratch_on_device() {
  int dev = -1;
  if (hipGetDevice(&dev) != hipSuccess) return nullptr;
  std::lock_guard<std::mutex> lk(g_scratch_mu);
  auto it = g_scratch_ptr.find(dev);
  if (it != g_scratch_ptr.end()) return it->second;
  void* ptr = nullptr;
  if (hipGetSymbolAddress(&ptr, HIP_SYMBOL(scratch)) != hipSuccess || !ptr) {
    (void)hipGetLastError();
    return nullptr;
  }
  g_scratch_ptr[dev] = (double2*)ptr;
  return (double2*)ptr;
}
}  // namespace

extern "C" int dh_hermitian_eigenvalues_noalloc(const double* a_dev, int n, double* w_dev, void* stream) {
  if (!a_dev || !w_dev) return DH_ERR_NULLPOINTER;
  if (n < 1 || n > DH_NOALLOC_EIG_MAX_N) return DH_ERR_INVALIDDIMENSION;
  double2* sp = scratch_on_device();
  if (!sp) return DH_ERR_ERROR;
  hipStream_t s = (hipStream_t)stream;
  int* info_dev = (int*)(sp + kNoAllocMat);
  int info = -1;
  const bool ok = hipMemcpyAsync(sp, a_dev, (size_t)n * n * 16, hipMemcpyDeviceToDevice, s) == hipSuccess &&
                  dh::launch_heig(sp, n, w_dev, info_dev, s) == hipSuccess &&
                  hipMemcpyAsync(&info, info_dev, sizeof(int), hipMemcpyDeviceToHost, s) == hipSuccess &&
                  hipStreamSynchronize(s) == hipSuccess;
  if (!ok) {
    (void)hipGetLastError();
    return DH_ERR_ERROR;
  }
  return info < 0 ? DH_ERR_ERROR : DH_SUCCESS;
}

extern "C" int dh_set_align_goal(dh_handle h, int goal, int pol_independent, int mul_conj_trans) {
  Plan* pl = get(h);
  if (!pl) return DH_ERR_INVALIDHANDLE;
  if (goal < DH_GOAL_CAPTURED || goal >= DH_METRIC_COUNT) return set_err(pl, DH_ERR_INVALIDARGUMENT);
  pl->goal = goal;
  pl->goal_indep = pol_independent != 0;
  pl->goal_aa = mul_conj_trans != 0;
  return set_err(pl, DH_SUCCESS);
}

namespace {
// HG -> LG coefficient transform. LG mode (p, l) of group N = 2p + |l| is a
// combination of the HG modes of the same group only ("Basis types": both
// bases hold the same modes per group), so T is block diagonal: block N is
// (N+1) x (N+1), rows in LG order (l = N, N-2, ..., -N), columns HG(N-k, k)
// in the plan's mode order (m = N - k descending):
//   T = (-1)^p i^k b(n, m, k),  n = p + max(l, 0), m = p + max(-l, 0),
//   b = sqrt((N-k)! k! / (2^N n! m!)) [t^k] (1 - t)^n (1 + t)^m,
// the mode-converter expansion of LG in HG, conjugated (T = <LG|HG>). The
// polynomial coefficient is an alternating sum of binomial products up to
// C(N, k) (< 2^97 for N < 100), summed exactly in 128-bit integers.
// Returns the blocks one after another, block N row-major.
std::vector<cd> lg_blocks(int G) {
  std::vector<cd> t;
  auto binom = [](int n, int k) -> __int128 {
    if (k < 0 || k > n) return 0;
    __int128 r = 1;
    for (int i = 1; i <= k; ++i) r = r * (n - k + i) / i;
    return r;
  };
  static const cd ik[4] = {cd(1, 0), cd(0, 1), cd(-1, 0), cd(0, -1)};
  for (int N = 0; N < G; ++N) {
    for (int r = 0; r <= N; ++r) {
      const int l = N - 2 * r, p = (N - std::abs(l)) / 2;
      const int n = p + std::max(l, 0), m = p + std::max(-l, 0);
      for (int k = 0; k <= N; ++k) {
        __int128 poly = 0;
        for (int a = 0; a <= k; ++a) poly += (a & 1 ? -1 : 1) * binom(n, a) * binom(m, k - a);
        const double b = std::exp(0.5 * (std::lgamma(N - k + 1.0) + std::lgamma(k + 1.0) - N * std::log(2.0) -
                                         std::lgamma(n + 1.0) - std::lgamma(m + 1.0))) * (double)poly;
        t.push_back(((p & 1) ? -1.0 : 1.0) * ik[k & 3] * b);
      }
    }
  }
  return t;
}
}  // namespace

extern "C" int dh_set_basis(dh_handle h, int type, int modes_out, int modes_in, const dh_c64* transform) {
  Plan* pl = get(h);
  if (!pl) return DH_ERR_INVALIDHANDLE;
  if (type < DH_BASIS_HG || type > DH_BASIS_CUSTOM) return set_err(pl, DH_ERR_INVALIDARGUMENT);
  const int M = pl->g.nmodes, G = pl->g.G, P = pl->params.pol_count;
  int mout = 0, mused = 0, ngrp = 0;
  // the transform as entries and, per output mode k, the range of HG modes it
  // takes: out[k] = sum_{i < cnt} e[off + i stride] c[first + i]
  std::vector<float2> tt;
  std::vector<int4> rng;
  std::vector<int> grp;
  if (type == DH_BASIS_LG) {
    if (M == 0) return set_err(pl, DH_ERR_INVALIDDIMENSION);
    mout = mused = M;
    ngrp = G;
    const std::vector<cd> t = lg_blocks(G);
    tt.resize(t.size());
    size_t off = 0;
    int base = 0;
    for (int N = 0; N < G; ++N) {
      // block N stored transposed, [HG k][LG r], so the threads of one group read consecutive entries
      for (int r = 0; r <= N; ++r) {
        for (int k = 0; k <= N; ++k) {
          const cd v = t[off + (size_t)r * (N + 1) + k];
          tt[off + (size_t)k * (N + 1) + r] = make_float2((float)v.real(), (float)v.imag());
        }
        rng.push_back(make_int4(base, N + 1, (int)(off + r), N + 1));
        grp.push_back(N);
      }
      off += (size_t)(N + 1) * (N + 1);
      base += N + 1;
    }
  } else if (type == DH_BASIS_CUSTOM) {
    if (M == 0 || modes_out < 1 || modes_in < 1 || modes_out > 65536) return set_err(pl, DH_ERR_INVALIDDIMENSION);
    if (!transform) return set_err(pl, DH_ERR_NULLPOINTER);
    mout = modes_out;
    mused = std::min(modes_in, M);
    if ((size_t)mout * mused > (size_t)INT32_MAX) return set_err(pl, DH_ERR_INVALIDDIMENSION);
    ngrp = mout;                     // no group structure: every output mode its own
    // dense, stored transposed [j][k] (consecutive output modes side by side)
    tt.resize((size_t)mout * mused);
    for (int k = 0; k < mout; ++k) {
      for (int j = 0; j < mused; ++j) {
        const dh_c64& v = transform[(size_t)k * modes_in + j];
        tt[(size_t)j * mout + k] = make_float2((float)v.re, (float)v.im);
      }
      rng.push_back(make_int4(0, mused, k, mout));
      grp.push_back(k);
    }
  }
  // work in flight may still read the old tables
  if (hipDeviceSynchronize() != hipSuccess) return set_err(pl, DH_ERR_ERROR);
  if (pl->bmem) (void)hipFree(pl->bmem);
  pl->bmem = nullptr;
  pl->btt = nullptr; pl->brng = nullptr; pl->bgrp = nullptr; pl->bc = pl->bcn = nullptr;
  pl->basis = DH_BASIS_HG;
  pl->bout = pl->bin = pl->bngrp = 0;
  ++pl->version;
  if (type == DH_BASIS_HG) return set_err(pl, DH_SUCCESS);
  const size_t ott = 0, orn = align256(tt.size() * 8), ogr = orn + align256((size_t)mout * 16);
  const size_t cap = (size_t)std::max(pl->max_batch, pl->ocap);
  const size_t oc = ogr + align256((size_t)mout * 4), ocn = oc + align256(cap * P * mout * 8);
  const size_t total = ocn + align256(cap * P * mout * 8);
  if (hipMalloc(&pl->bmem, total) != hipSuccess) {
    (void)hipGetLastError();
    pl->bmem = nullptr;
    return set_err(pl, DH_ERR_MEMORYALLOCATION);
  }
  if (hipMemcpy(pl->bmem + ott, tt.data(), tt.size() * 8, hipMemcpyHostToDevice) != hipSuccess ||
      hipMemcpy(pl->bmem + orn, rng.data(), rng.size() * 16, hipMemcpyHostToDevice) != hipSuccess ||
      hipMemcpy(pl->bmem + ogr, grp.data(), grp.size() * 4, hipMemcpyHostToDevice) != hipSuccess) {
    (void)hipFree(pl->bmem);
    pl->bmem = nullptr;
    return set_err(pl, DH_ERR_ERROR);
  }
  pl->btt = (float2*)(pl->bmem + ott);
  pl->brng = (int4*)(pl->bmem + orn);
  pl->bgrp = (int*)(pl->bmem + ogr);
  pl->bc = (float2*)(pl->bmem + oc);
  pl->bcn = (float2*)(pl->bmem + ocn);
  pl->basis = type;
  pl->bout = mout;
  pl->bin = mused;
  pl->bngrp = ngrp;
  return set_err(pl, DH_SUCCESS);
}

namespace {
// staging buffers of a sweep or averaged batch (freed when neither is set)
int ensure_staging(Plan* pl) {
  if (pl->smem) (void)hipFree(pl->smem);
  pl->smem = nullptr;
  pl->sptr = nullptr;
  pl->sc = pl->scn = pl->swin = pl->sfld = nullptr;
  pl->rot = nullptr;
  if (!sweeping(pl)) return DH_SUCCESS;
  const Geom& g = pl->g;
  const dh_params* p = &pl->params;
  const size_t B = pl->max_batch, P = p->pol_count, nm = std::max(g.nmodes, 1);
  const size_t plane = B * P * g.wy * g.wx * 8;
  const bool win = pl->avg > 1 || p->keep_window || exports(g, p), fld = p->keep_fields && g.mode == 1;
  size_t o = 0;
  auto take = [&](size_t n) { size_t r = o; o += align256(n); return r; };
  const size_t o_ptr = take(B * 8), o_c = take(B * P * nm * 8), o_cn = take(B * P * nm * 8);
  const size_t o_w = win ? take(plane) : 0, o_f = fld ? take(plane) : 0, o_r = take(B * 16);
  if (hipMalloc(&pl->smem, o) != hipSuccess) {
    (void)hipGetLastError();
    pl->smem = nullptr;
    return DH_ERR_MEMORYALLOCATION;
  }
  pl->sptr = (const void**)(pl->smem + o_ptr);
  pl->sc = (float2*)(pl->smem + o_c);
  pl->scn = (float2*)(pl->smem + o_cn);
  pl->swin = win ? (float2*)(pl->smem + o_w) : nullptr;
  pl->sfld = fld ? (float2*)(pl->smem + o_f) : nullptr;
  pl->rot = (double2*)(pl->smem + o_r);
  return DH_SUCCESS;
}
}  // namespace

extern "C" int dh_set_wavelengths(dh_handle h, const double* lambdas, int count, int in_order, int out_order) {
  Plan* pl = get(h);
  if (!pl) return DH_ERR_INVALIDHANDLE;
  if (count < 0 || count > 4096) return set_err(pl, DH_ERR_INVALIDDIMENSION);
  if (count > 0 && !lambdas) return set_err(pl, DH_ERR_NULLPOINTER);
  if ((in_order != DH_WL_FAST && in_order != DH_WL_SLOW) || (out_order != DH_WL_FAST && out_order != DH_WL_SLOW))
    return set_err(pl, DH_ERR_INVALIDARGUMENT);
  const Geom& g = pl->g;
  const dh_params* p = &pl->params;
  const int P = p->pol_count;
  // every wavelength's window must lie in the spectrum with the plan's box
  std::vector<PolGeom> geo((size_t)count * 2);
  for (int w = 0; w < count; ++w) {
    if (!(lambdas[w] > 0.0) || !std::isfinite(lambdas[w])) return set_err(pl, DH_ERR_INVALIDARGUMENT);
    dh_params pw = *p;
    pw.wavelength = lambdas[w];
    Geom gw = g;
    for (int q = 0; q < P; ++q) {
      const int e = derive_pol(&pw, &gw, q);
      if (e != DH_SUCCESS) return set_err(pl, e);
      geo[(size_t)w * 2 + q] = gw.pol[q];
    }
  }
  if (hipDeviceSynchronize() != hipSuccess) return set_err(pl, DH_ERR_ERROR);
  if (pl->lmem) (void)hipFree(pl->lmem);
  pl->lmem = nullptr;
  pl->nlam = 0;
  pl->lams.clear();
  pl->lam_geom.clear();
  pl->lam_tab.clear();
  if (count > 0) {
    const bool exp = exports(g, p);
    std::vector<Plan::LamTab> tab((size_t)count * 2);
    size_t o = 0;
    auto take = [&](size_t n) { size_t r = o; o += align256(n); return r; };
    for (int w = 0; w < count; ++w)
      for (int q = 0; q < P; ++q) {
        Plan::LamTab& t = tab[(size_t)w * 2 + q];
        t.mrow = take(g.by * 8); t.rhox = take(g.bx * 8); t.rhoy = take(g.by * 8);
        t.tx = take(g.wx * 8); t.ty = take(g.wy * 8);
        t.xs = g.spec ? take((size_t)g.bx * g.gp * 8) : 0;
        t.ys = g.spec ? take((size_t)g.wys * g.gp * 8) : 0;
        t.ex = exp ? take((size_t)g.fx * 8) : 0;
        t.ey = exp ? take((size_t)g.fy * 8) : 0;
      }
    if (hipMalloc(&pl->lmem, o) != hipSuccess) {
      (void)hipGetLastError();
      pl->lmem = nullptr;
      return set_err(pl, DH_ERR_MEMORYALLOCATION);
    }
    for (int w = 0; w < count; ++w) {
      dh_params pw = *p;
      pw.wavelength = lambdas[w];
      for (int q = 0; q < P; ++q) {
        const Plan::LamTab& t = tab[(size_t)w * 2 + q];
        const PolTables v = pol_tables(g, geo[(size_t)w * 2 + q], &pw, q, g.spec, exp);
        if (!upload(pl->lmem, t.mrow, v.mrow) || !upload(pl->lmem, t.rhox, v.rhox) ||
            !upload(pl->lmem, t.rhoy, v.rhoy) || !upload(pl->lmem, t.tx, v.tx) || !upload(pl->lmem, t.ty, v.ty) ||
            (g.spec && (!upload(pl->lmem, t.xs, v.xs) || !upload(pl->lmem, t.ys, v.ys))) ||
            (exp && (!upload(pl->lmem, t.ex, v.ex) || !upload(pl->lmem, t.ey, v.ey)))) {
          (void)hipFree(pl->lmem);
          pl->lmem = nullptr;
          return set_err(pl, DH_ERR_ERROR);
        }
      }
    }
    pl->nlam = count;
    pl->lams.assign(lambdas, lambdas + count);
    pl->lam_geom = geo;
    pl->lam_tab = tab;
  }
  pl->in_order = in_order;
  pl->out_order = out_order;
  const int e = ensure_staging(pl);
  if (e != DH_SUCCESS) {   // no staging: back to single-wavelength processing
    if (pl->lmem) (void)hipFree(pl->lmem);
    pl->lmem = nullptr;
    pl->nlam = 0;
    pl->lams.clear();
    pl->lam_geom.clear();
    pl->lam_tab.clear();
    (void)ensure_staging(pl);
  }
  return set_err(pl, e);
}

extern "C" int dh_set_averaging(dh_handle h, int count, int mode) {
  Plan* pl = get(h);
  if (!pl) return DH_ERR_INVALIDHANDLE;
  if (count < 1 || count > 4096) return set_err(pl, DH_ERR_INVALIDDIMENSION);
  if (mode < DH_AVG_SEQUENTIAL || mode > DH_AVG_SEQUENTIAL_SWEEP) return set_err(pl, DH_ERR_INVALIDARGUMENT);
  if (hipDeviceSynchronize() != hipSuccess) return set_err(pl, DH_ERR_ERROR);
  const int old = pl->avg;
  pl->avg = count;
  pl->avg_mode = mode;
  const int e = ensure_staging(pl);
  if (e != DH_SUCCESS) {   // no staging: averaging stays as it was
    pl->avg = old;
    (void)ensure_staging(pl);
  }
  return set_err(pl, e);
}

extern "C" int dh_fields_to_int16(const dh_c64* fields, int n_fields, long long field_len, short* re, short* im,
                                  float* scale, void* stream) {
  if (n_fields < 0 || field_len < 1) return DH_ERR_INVALIDARGUMENT;
  if (n_fields == 0) return DH_SUCCESS;
  if (!fields || !re || !im || !scale) return DH_ERR_NULLPOINTER;
  return dh::launch_q16((const float2*)fields, n_fields, field_len, re, im, scale, (hipStream_t)stream) == hipSuccess
             ? DH_SUCCESS
             : DH_ERR_ERROR;
}

extern "C" int dh_get_fields16(dh_handle h, short* re_host, short* im_host, float* scale_host, const short** re_dev,
                               const short** im_dev, const float** scale_dev, int* batch, int* pols, int* width,
                               int* height) {
  Plan* pl = get(h);
  if (!pl) return DH_ERR_INVALIDHANDLE;
  const Geom& g = pl->g;
  const int P = pl->params.pol_count;
  if (batch) *batch = pl->last_batch;
  if (pols) *pols = P;
  if (width) *width = g.fx;
  if (height) *height = g.fy;
  const float2* src = field_buffer(pl);
  if (!src || pl->last_batch < 1) return set_err(pl, DH_ERR_ERROR);
  const size_t n = (size_t)pl->max_batch * P, len = (size_t)g.fx * g.fy;
  const size_t o_im = align256(n * len * 2), o_sc = o_im + align256(n * len * 2);
  if (!pl->q16_mem && hipMalloc(&pl->q16_mem, o_sc + align256(n * 4)) != hipSuccess) {
    (void)hipGetLastError();
    pl->q16_mem = nullptr;
    return set_err(pl, DH_ERR_MEMORYALLOCATION);
  }
  short* re = (short*)pl->q16_mem;
  short* im = (short*)(pl->q16_mem + o_im);
  float* sc = (float*)(pl->q16_mem + o_sc);
  if (re_dev) *re_dev = re;
  if (im_dev) *im_dev = im;
  if (scale_dev) *scale_dev = sc;
  const int nf = pl->last_batch * P;
  hipStream_t s = pl->last_stream;
  if (dh::launch_q16(src, nf, (long long)len, re, im, sc, s) != hipSuccess) return set_err(pl, DH_ERR_ERROR);
  if (re_host && hipMemcpyAsync(re_host, re, (size_t)nf * len * 2, hipMemcpyDeviceToHost, s) != hipSuccess)
    return set_err(pl, DH_ERR_ERROR);
  if (im_host && hipMemcpyAsync(im_host, im, (size_t)nf * len * 2, hipMemcpyDeviceToHost, s) != hipSuccess)
    return set_err(pl, DH_ERR_ERROR);
  if (scale_host && hipMemcpyAsync(scale_host, sc, (size_t)nf * 4, hipMemcpyDeviceToHost, s) != hipSuccess)
    return set_err(pl, DH_ERR_ERROR);
  if (hipStreamSynchronize(s) != hipSuccess) return set_err(pl, DH_ERR_ERROR);
  return set_err(pl, DH_SUCCESS);
}

extern "C" int dh_set_pol_lock(dh_handle h, unsigned lock) {
  Plan* pl = get(h);
  if (!pl) return DH_ERR_INVALIDHANDLE;
  if (lock & ~(DH_ALIGN_TILT | DH_ALIGN_DEFOCUS | DH_ALIGN_WAIST)) return set_err(pl, DH_ERR_INVALIDARGUMENT);
  pl->lock = lock & (DH_ALIGN_TILT | DH_ALIGN_DEFOCUS);   // the waist is always one for both pols
  return set_err(pl, DH_SUCCESS);
}

extern "C" int dh_get_align_report(dh_handle h, dh_align_report* out) {
  Plan* pl = get(h);
  if (!pl) return DH_ERR_INVALIDHANDLE;
  if (!out) return set_err(pl, DH_ERR_NULLPOINTER);
  *out = pl->rep;
  return DH_SUCCESS;
}

// ---------------------------------------------------------------------------
// Serving: continuous batching of frames from several cameras.
//
// Each camera is a resident plan (tables, HG bases, alignment state stay on
// the device). Its "lanes" are independent in-flight batch slots: a HIP
// stream, a workspace for up to max_batch frames, a device array of frame
// pointers and pinned result buffers. As many lanes are made as the HBM budget
// allows (at least one, at most four per camera). A request waits in its
// camera's queue until a lane of that camera is free; the lane then takes
// every waiting request (up to max_batch) as one batch, so batches grow with
// the load and requests that arrive while others are on the GPU join the next
// free lane. Lanes of all cameras run concurrently on the device. The launch
// sequence of a batch is captured once per (lane, batch size) as a hipGraph
// and replayed (batches of up to 16 requests; larger ones launch directly).
namespace {

using Clock = std::chrono::steady_clock;

struct Req {
  const void* frame;
  dh_c64* out;
  int idx;
};

struct Lane {
  int version = -1;              // plan version the arguments and graphs were made for
  size_t off[8] = {0, 0, 0, 0, 0, 0, 0, 0};
  hipStream_t s = nullptr;
  hipEvent_t done = nullptr;
  char* mem = nullptr;
  const void** hptr = nullptr;   // pinned host copy of the frame pointers
  float2* hres = nullptr;        // pinned host results
  dh::KArgs k{};
  std::vector<Req> batch;
  bool busy = false;
  std::map<int, hipGraphExec_t> graphs;
};

struct Camera {
  Plan* pl = nullptr;
  std::deque<Req> pending;
  std::vector<Lane> lanes;
  size_t lane_bytes = 0;
  int per_result = 0;            // complex values per request: pols x modes
  int basis = DH_BASIS_HG;       // the plan's basis when the server was made
  int bout = 0;
};

struct Server {
  std::vector<Camera> cams;
  int max_batch = 1;
  bool graphs = true, normalised = true;
  Clock::time_point t0;
  double* t_done = nullptr;      // replay: completion time per request index
  long long batches = 0, frames = 0;
  int last_error = 0;
};

std::mutex g_smu;
std::vector<Server*> g_servers;

Server* sget(dh_server h) {
  std::lock_guard<std::mutex> lk(g_smu);
  if (h < 0 || (size_t)h >= g_servers.size()) return nullptr;
  return g_servers[h];
}

size_t lane_layout(const Plan* pl, int mb, size_t off[8]) {
  const Geom& g = pl->g;
  const size_t P = pl->params.pol_count, nm = g.nmodes > 0 ? g.nmodes : 1;
  size_t o = 0;
  auto take = [&](size_t bytes) { size_t r = o; o += align256(bytes); return r; };
  off[0] = take((size_t)mb * P * g.ny * g.bx * 8);                  // t1
  off[1] = take(g.spec ? 0 : (size_t)mb * P * g.wy * ((g.bx + 15) / 16 * 16) * 8);  // f2
  const int nblk = g.spec ? dh::spectral_blocks(g.ny, g.wy, g.bx, g.gp) : field_blocks(g);
  off[2] = take((size_t)mb * P * nblk * (nm + 1) * 8);               // partial
  off[3] = take((size_t)mb * P * nm * 8);                            // coefs
  off[4] = take((size_t)mb * P * nm * 8);                            // coefs_norm
  off[5] = take((size_t)mb * 8);                                     // frame pointers
  const size_t nb = pl->basis != DH_BASIS_HG ? pl->bout : 0;
  off[6] = take((size_t)mb * P * nb * 8);                            // basis coefs
  off[7] = take((size_t)mb * P * nb * 8);                            // basis coefs, normalised
  return o;
}

void free_lane(Lane& L) {
  for (auto& kv : L.graphs) (void)hipGraphExecDestroy(kv.second);
  L.graphs.clear();
  if (L.s) (void)hipStreamDestroy(L.s);
  if (L.done) (void)hipEventDestroy(L.done);
  if (L.mem) (void)hipFree(L.mem);
  if (L.hptr) (void)hipHostFree(L.hptr);
  if (L.hres) (void)hipHostFree(L.hres);
  L = Lane();
}

int make_lane(Server* S, Camera& C, Lane& L) {
  size_t off[8];
  lane_layout(C.pl, S->max_batch, off);
  if (hipStreamCreateWithFlags(&L.s, hipStreamNonBlocking) != hipSuccess ||
      hipEventCreateWithFlags(&L.done, hipEventDisableTiming) != hipSuccess ||
      hipMalloc(&L.mem, C.lane_bytes) != hipSuccess ||
      hipHostMalloc((void**)&L.hptr, (size_t)S->max_batch * sizeof(void*), hipHostMallocDefault) != hipSuccess ||
      hipHostMalloc((void**)&L.hres, (size_t)S->max_batch * C.per_result * 8, hipHostMallocDefault) != hipSuccess) {
    (void)hipGetLastError();
    free_lane(L);
    return DH_ERR_MEMORYALLOCATION;
  }
  for (int i = 0; i < 8; ++i) L.off[i] = off[i];
  return DH_SUCCESS;
}

// the plan's current tables with the lane's own buffers; graphs made for an
// older version of the plan are dropped
void lane_args(const Camera& C, Lane& L) {
  if (L.version == C.pl->version) return;
  for (auto& kv : L.graphs) (void)hipGraphExecDestroy(kv.second);
  L.graphs.clear();
  L.k = C.pl->ka[0];
  L.k.t1 = (float2*)(L.mem + L.off[0]);
  L.k.f2 = (float2*)(L.mem + L.off[1]);
  L.k.partial = (float2*)(L.mem + L.off[2]);
  L.k.coefs = (float2*)(L.mem + L.off[3]);
  L.k.coefs_norm = (float2*)(L.mem + L.off[4]);
  L.k.fptr = (const void* const*)(L.mem + L.off[5]);
  L.k.window = nullptr;
  L.k.fields = nullptr;
  L.k.capt = nullptr;
  L.version = C.pl->version;
}

constexpr int kGraphBatches = 16;   // largest batch launched as a captured graph

hipError_t record_batch(const Camera& C, const Lane& L, int n) {
  const Plan* pl = C.pl;
  const int u16 = pl->params.input_dtype == DH_INPUT_U16;
  const bool spec = pl->g.spec;
  hipError_t e = dh::launch_row(L.k, nullptr, u16, 0, n, L.s);
  if (e == hipSuccess) e = spec ? dh::launch_cspec(L.k, 0, n, L.s) : dh::launch_col(L.k, 0, n, L.s);
  if (e == hipSuccess && !spec && L.k.G > 0) e = dh::launch_fld(L.k, 0, n, L.s);
  if (e == hipSuccess && L.k.G > 0) e = dh::launch_norm(L.k, 0, n, L.s);
  if (e == hipSuccess && C.basis != DH_BASIS_HG)
    e = dh::launch_basis(L.k.coefs, L.k.coefs_norm, pl->g.nmodes, pl->bin, pl->brng, pl->btt, pl->bout,
                         (float2*)(L.mem + L.off[6]), (float2*)(L.mem + L.off[7]), n * pl->params.pol_count, L.s);
  return e;
}

int launch_lane(Server* S, Camera& C, Lane& L) {
  // the lanes were sized for the basis the plan had when the server was made;
  // sweeps and averaging are not served
  if (C.pl->basis != C.basis || (C.basis != DH_BASIS_HG && C.pl->bout != C.bout) || sweeping(C.pl))
    return DH_ERR_ERROR;
  lane_args(C, L);
  const int n = (int)std::min<size_t>(C.pending.size(), (size_t)S->max_batch);
  L.batch.assign(C.pending.begin(), C.pending.begin() + n);
  C.pending.erase(C.pending.begin(), C.pending.begin() + n);
  for (int i = 0; i < n; ++i) L.hptr[i] = L.batch[i].frame;
  if (hipMemcpyAsync((void*)L.k.fptr, L.hptr, (size_t)n * sizeof(void*), hipMemcpyHostToDevice, L.s) != hipSuccess)
    return DH_ERR_ERROR;
  // graphs replay the small batches, where launch latency is a large part of
  // a request's time; a larger batch is launched directly (its kernels run far
  // longer than the few launches take), so a lane holds at most kGraphBatches
  // graphs and a burst of large batches never waits for a capture
  if (S->graphs && n <= kGraphBatches) {
    auto it = L.graphs.find(n);
    if (it == L.graphs.end()) {
      hipGraph_t gr = nullptr;
      hipGraphExec_t ex = nullptr;
      if (hipStreamBeginCapture(L.s, hipStreamCaptureModeThreadLocal) != hipSuccess) return DH_ERR_ERROR;
      const hipError_t rec = record_batch(C, L, n);
      const hipError_t end = hipStreamEndCapture(L.s, &gr);
      if (rec != hipSuccess || end != hipSuccess || hipGraphInstantiate(&ex, gr, nullptr, nullptr, 0) != hipSuccess) {
        if (gr) (void)hipGraphDestroy(gr);
        return DH_ERR_ERROR;
      }
      (void)hipGraphDestroy(gr);
      it = L.graphs.emplace(n, ex).first;
    }
    if (hipGraphLaunch(it->second, L.s) != hipSuccess) return DH_ERR_ERROR;
  } else if (record_batch(C, L, n) != hipSuccess) {
    return DH_ERR_ERROR;
  }
  const float2* res = C.basis != DH_BASIS_HG
                          ? (const float2*)(L.mem + L.off[S->normalised ? 7 : 6])
                          : (S->normalised ? L.k.coefs_norm : L.k.coefs);
  if (C.per_result > 0 &&
      hipMemcpyAsync(L.hres, res, (size_t)n * C.per_result * 8, hipMemcpyDeviceToHost, L.s) != hipSuccess)
    return DH_ERR_ERROR;
  if (hipEventRecord(L.done, L.s) != hipSuccess) return DH_ERR_ERROR;
  L.busy = true;
  ++S->batches;
  S->frames += n;
  return DH_SUCCESS;
}

// one scheduling round: retire finished batches, start new ones
int serve_round(Server* S, int* completed) {
  int done = 0;
  for (Camera& C : S->cams) {
    for (Lane& L : C.lanes) {
      if (!L.busy) continue;
      const hipError_t q = hipEventQuery(L.done);
      if (q == hipErrorNotReady) continue;
      if (q != hipSuccess) return DH_ERR_ERROR;
      const double t = std::chrono::duration<double>(Clock::now() - S->t0).count();
      for (size_t i = 0; i < L.batch.size(); ++i) {
        const Req& r = L.batch[i];
        if (r.out) std::memcpy(r.out, L.hres + i * C.per_result, (size_t)C.per_result * 8);
        if (S->t_done && r.idx >= 0) S->t_done[r.idx] = t;
      }
      done += (int)L.batch.size();
      L.batch.clear();
      L.busy = false;
    }
    for (Lane& L : C.lanes) {
      if (C.pending.empty()) break;
      if (!L.busy) {
        const int e = launch_lane(S, C, L);
        if (e != DH_SUCCESS) return e;
      }
    }
  }
  if (completed) *completed = done;
  return DH_SUCCESS;
}

}  // namespace

extern "C" {

int dh_serve_create(const dh_handle* plans, int ncam, int max_batch, size_t hbm_budget, int use_graphs,
                    int normalised, dh_server* out) {
  if (!plans || !out) return DH_ERR_NULLPOINTER;
  if (ncam < 1 || max_batch < 1) return DH_ERR_INVALIDDIMENSION;
  Server* S = new Server();
  S->max_batch = max_batch;
  S->graphs = use_graphs != 0;
  S->normalised = normalised != 0;
  S->cams.resize(ncam);
  size_t total = 0;
  for (int c = 0; c < ncam; ++c) {
    Camera& C = S->cams[c];
    C.pl = get(plans[c]);
    if (!C.pl) {
      delete S;
      return DH_ERR_INVALIDHANDLE;
    }
    if (sweeping(C.pl)) {   // each request is one frame at the plan's wavelength
      delete S;
      return DH_ERR_INVALIDARGUMENT;
    }
    size_t off[8];
    C.lane_bytes = lane_layout(C.pl, max_batch, off);
    C.basis = C.pl->basis;
    C.bout = C.pl->bout;
    C.per_result = C.pl->params.pol_count * (C.basis != DH_BASIS_HG ? C.bout : C.pl->g.nmodes);
    total += C.lane_bytes;
  }
  if (hbm_budget && total > hbm_budget) {  // not even one lane per camera fits
    delete S;
    return DH_ERR_MEMORYALLOCATION;
  }
  // lanes round robin over the cameras while the budget allows
  int err = DH_SUCCESS;
  size_t used = 0;
  for (int round = 0; round < 4 && err == DH_SUCCESS; ++round)
    for (Camera& C : S->cams) {
      if (round > 0 && hbm_budget && used + C.lane_bytes > hbm_budget) continue;
      C.lanes.emplace_back();
      err = make_lane(S, C, C.lanes.back());
      if (err != DH_SUCCESS) {
        C.lanes.pop_back();
        if (round > 0) err = DH_SUCCESS;  // extra lanes are optional
        break;
      }
      used += C.lane_bytes;
    }
  if (err != DH_SUCCESS) {
    for (Camera& C : S->cams)
      for (Lane& L : C.lanes) free_lane(L);
    delete S;
    return err;
  }
  S->t0 = Clock::now();
  std::lock_guard<std::mutex> lk(g_smu);
  g_servers.push_back(S);
  *out = (dh_server)(g_servers.size() - 1);
  return DH_SUCCESS;
}

int dh_serve_info(dh_server h, int camera, int* lanes, size_t* lane_bytes, int* per_result) {
  Server* S = sget(h);
  if (!S) return DH_ERR_INVALIDHANDLE;
  if (camera < 0 || camera >= (int)S->cams.size()) return DH_ERR_INVALIDARGUMENT;
  const Camera& C = S->cams[camera];
  if (lanes) *lanes = (int)C.lanes.size();
  if (lane_bytes) *lane_bytes = C.lane_bytes;
  if (per_result) *per_result = C.per_result;
  return DH_SUCCESS;
}

int dh_serve_submit(dh_server h, int camera, const void* frame, dh_c64* result) {
  Server* S = sget(h);
  if (!S) return DH_ERR_INVALIDHANDLE;
  if (camera < 0 || camera >= (int)S->cams.size()) return DH_ERR_INVALIDARGUMENT;
  if (!frame) return DH_ERR_NULLPOINTER;
  S->cams[camera].pending.push_back(Req{frame, result, -1});
  return DH_SUCCESS;
}

int dh_serve_progress(dh_server h, int* completed) {
  Server* S = sget(h);
  if (!S) return DH_ERR_INVALIDHANDLE;
  return serve_round(S, completed);
}

int dh_serve_replay(dh_server h, int n, const double* t_arrival, const int* camera, const void* const* frames,
                    dh_c64* const* results, double* t_done, double* t_start) {
  Server* S = sget(h);
  if (!S) return DH_ERR_INVALIDHANDLE;
  if (!t_arrival || !camera || !frames || !t_done) return DH_ERR_NULLPOINTER;
  for (int i = 0; i < n; ++i)
    if (camera[i] < 0 || camera[i] >= (int)S->cams.size() || !frames[i] || (i && t_arrival[i] < t_arrival[i - 1]))
      return DH_ERR_INVALIDARGUMENT;
  S->t0 = Clock::now();
  S->t_done = t_done;
  int next = 0, finished = 0, err = DH_SUCCESS;
  while (finished < n) {
    const double now = std::chrono::duration<double>(Clock::now() - S->t0).count();
    while (next < n && t_arrival[next] <= now) {
      S->cams[camera[next]].pending.push_back(Req{frames[next], results ? results[next] : nullptr, next});
      ++next;
    }
    int done = 0;
    err = serve_round(S, &done);
    if (err != DH_SUCCESS) break;
    finished += done;
  }
  S->t_done = nullptr;
  if (t_start) *t_start = 0.0;
  if (err != DH_SUCCESS) {
    (void)hipDeviceSynchronize();
    for (Camera& C : S->cams) {
      C.pending.clear();
      for (Lane& L : C.lanes) {
        L.busy = false;
        L.batch.clear();
      }
    }
  }
  return err;
}

int dh_serve_stats(dh_server h, long long* batches, long long* frames) {
  Server* S = sget(h);
  if (!S) return DH_ERR_INVALIDHANDLE;
  if (batches) *batches = S->batches;
  if (frames) *frames = S->frames;
  return DH_SUCCESS;
}

int dh_serve_destroy(dh_server h) {
  Server* S;
  {
    std::lock_guard<std::mutex> lk(g_smu);
    if (h < 0 || (size_t)h >= g_servers.size() || !g_servers[h]) return DH_ERR_INVALIDHANDLE;
    S = g_servers[h];
    g_servers[h] = nullptr;
  }
  (void)hipDeviceSynchronize();
  for (Camera& C : S->cams)
    for (Lane& L : C.lanes) free_lane(L);
  delete S;
  return DH_SUCCESS;
}

}  // extern "C"
