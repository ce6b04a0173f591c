// Host side of the C ABI declared in include/ell.h: grid/level construction,
// the V-cycle schedule and the preconditioned CG driver for one MI355X.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <array>
#include <chrono>
#include <map>
#include <mutex>
#include <type_traits>
#include <cmath>
#include <cstdarg>
#include <cstdio>
#include <cstring>
#include <string>
#include <vector>

#include "ell.h"
#include "ell_kernels.hpp"

using namespace ell;

namespace {

thread_local std::string g_err;

int fail(int code, const char *fmt, ...) {
  char buf[512];
  va_list ap;
  va_start(ap, fmt);
  vsnprintf(buf, sizeof(buf), fmt, ap);
  va_end(ap);
  g_err = buf;
  return code;
}

#define HIPCHK(expr)                                                                    \
  do {                                                                                  \
    hipError_t e_ = (expr);                                                             \
    if (e_ != hipSuccess)                                                               \
      return fail(ELL_ERR_HIP, "%s failed: %s", #expr, hipGetErrorString(e_));          \
  } while (0)

#define CHK(expr)                \
  do {                           \
    int rc_ = (expr);            \
    if (rc_ != ELL_OK) return rc_; \
  } while (0)

int check_launch(const char *what) {
  hipError_t e = hipGetLastError();
  if (e != hipSuccess) return fail(ELL_ERR_HIP, "launch of %s failed: %s", what, hipGetErrorString(e));
  return ELL_OK;
}

inline int blocks8(long long threads) {
  long long b = (threads + kBlock - 1) / kBlock;
  if (b < 1) b = 1;
  b = (b + 7) / 8 * 8;
  return (int)b;
}

// blocks of 64 columns x kSeg k-segments covering `cols` columns
inline int seg_blocks(long long cols) { return blocks8((cols + kSegCols - 1) / kSegCols * kBlock); }

// blocks of the CG operator kernels: (4 / nseg) chunks of 64 slots per block
inline int stencil_blocks(long long slots, int nseg) {
  const long long per = (long long)kSegCols * (4 / nseg);
  return blocks8((slots + per - 1) / per * kBlock);
}

// Grid of a flat vector kernel over n2 element pairs: a fixed function of n2,
// so reductions over it are reproducible.
inline int flat_blocks(long long n2) {
  long long b = (n2 + kBlock * 4 - 1) / (kBlock * 4);
  if (b > 2048) b = 2048;
  if (b < 8) b = 8;
  return (int)((b + 7) / 8 * 8);
}

// Blocks of a vector kernel inside a grouped (batched) launch: a fixed chunk of
// kBatchChunk double2 per thread, so that blocks of grids of every size cost
// the same and the blocks of one launch spread evenly over the XCDs.
constexpr int kBatchChunk = 16;
inline int batch_flat_blocks(long long n2) {
  const long long b = (n2 + (long long)kBlock * kBatchChunk - 1) / ((long long)kBlock * kBatchChunk);
  return (int)std::max<long long>(b, 1);
}

// k-segments of the tiled CG operator step: enough blocks to occupy the chip
// on thin grids, few enough that the two extra levels a segment reads at its
// ends stay a small fraction.
inline int apply_segments(int nz) { return nz >= 64 ? 4 : (nz >= 32 ? 2 : 1); }
inline long long tile_blocks(const Geo &G, int nseg) {
  return G.has_x && G.has_y ? (long long)tile_count(G.hx2, G.ny) * nseg : 0;
}

// Blocks whose partial sums one grid's reduction buffer must hold.
inline long long partial_blocks(const Geo &G0, long long n0) {
  long long b = std::max<long long>(seg_blocks(2LL * G0.H), flat_blocks(n0 / 2));
  b = std::max<long long>(b, batch_flat_blocks(n0 / 2));
  b = std::max<long long>(b, 2LL * ((G0.hx2 + kSTX - 1) / kSTX) * (G0.ny / 2));  // fused dots
  // fused forms of the per-column sweep: one slot per block of either colour
  b = std::max<long long>(b, blocks8(((long long)G0.ncol0 + kSegCols - 1) / kSegCols * kBlock) +
                                 blocks8(((long long)G0.ncol1 + kSegCols - 1) / kSegCols * kBlock));
  return std::max<long long>(b, blocks8(tile_blocks(G0, 4) * kBlock));
}

bool can_halve(int n) { return n % 2 == 0 && ((n / 2) % 2 == 0 || n / 2 == 1); }

int standard_depth(int nx, int ny) {
  int L = 1;
  while (can_halve(nx) && can_halve(ny)) {
    nx /= 2;
    ny /= 2;
    ++L;
  }
  return L;
}

// Round to the nearest bfloat16 (ties to even), returned as float.
float round_bf16(float x) {
  uint32_t u;
  std::memcpy(&u, &x, 4);
  if ((u & 0x7f800000u) == 0x7f800000u) return x;
  uint32_t lsb = (u >> 16) & 1u;
  u += 0x7fffu + lsb;
  u &= 0xffff0000u;
  float r;
  std::memcpy(&r, &u, 4);
  return r;
}

struct Prof {
  int cap = 0;
  int n = 0;
  bool paused = false;  // launches made while paused record nothing
  std::vector<hipEvent_t> ev;
};

struct Level {
  Geo geo;
  double hx, hy;
  void *tab = nullptr;  // device table, element type of the V-cycle
  void *b = nullptr;    // levels >= 1: right-hand side (split)
  void *u = nullptr;    // levels >= 1: correction (split)
  // grids with horizontally varying vertical coefficients (split layout, FP64):
  // each column's faces T_{k-1/2} (zero at k = 0) and the factors 1/p_k and
  // T_{k+1/2}/p_k of its column elimination
  double *tz3 = nullptr, *ip3 = nullptr, *cf3 = nullptr;
  float *tz3f = nullptr, *ip3f = nullptr, *cf3f = nullptr;  // FP32 copies (mixed-precision grids)
};

}  // namespace

struct ell_grid {
  ell_grid_desc d;
  std::vector<double> dz, lam;
  int L = 0;
  int prec = ELL_FP64;
  size_t esz = 8;
  std::vector<Level> lev;
  long long n0 = 0;          // split elements of level 0 (2*cs)
  double *us = nullptr, *r = nullptr, *z = nullptr, *p = nullptr, *q = nullptr;
  double *p2 = nullptr;                 // second and third search-direction buffers (p_K
  double *p3 = nullptr;                 //   lives in {p, p2, p3}[K mod 3])
  void *b32 = nullptr, *z32 = nullptr;  // FP32 preconditioner: level-0 b and z
  void *ybuf = nullptr;                 // rho != 1: forward-sweep values
  double *vol0 = nullptr;               // level-0 cell volumes (FP64, nz)
  const double *tab64_0 = nullptr;      // level-0 FP64 table of the CG operator
  int stencil_seg = 1;                  // k-segments of the CG operator kernels
  int apply_tile = 0;                   // the CG operator step uses the LDS-tiled kernel
  int apply_nseg = 1;                   // its k-segments
  int smooth_tile = 0;                  // FP64 half-sweeps use the LDS-tiled kernel
  int fused_dot = 0;                    // the last post-smoothing half-sweeps form the CG dots
  int fused_update = 0;                 // the first pre-smoothing pair updates the CG residual
  int fused_prolong = 0;                // the first post-smoothing sweep applies the finest correction
  int tiled_ends = 0;                   // a solve's start and end run on the operator step's LDS tiles
  int coarse_tail = 0;                  // the coarsest level's sweeps in one cooperative launch
  int coarse_pair = 0;                  // the coarsest level's sweep pairs one launch each
  double *partial = nullptr;
  long long partial_cap = 0;
  PcgState *st = nullptr;
  PcgState *st_host = nullptr;          // pinned
  Prof prof[ELL_K_COUNT];
  std::vector<void *> allocs;
  bool varying = false;       // per-column vertical coefficients (Level::tz3, ip3, cf3)
  bool batch_layout = false;  // coarse levels use 4 or 8 k-segments (grouped launches)
  void *gdev = nullptr;       // device copy of the grid descriptor (batched kernels)
  int busy = 0;               // a batch request is using the grid
};

namespace {

int dalloc(ell_grid *g, void **p, size_t bytes) {
  if (bytes == 0) bytes = 256;
  hipError_t e = hipMalloc(p, bytes);
  if (e != hipSuccess) {
    *p = nullptr;
    (void)hipGetLastError();
    return fail(ELL_ERR_OOM, "hipMalloc(%zu) failed: %s", bytes, hipGetErrorString(e));
  }
  g->allocs.push_back(*p);
  HIPCHK(hipMemset(*p, 0, bytes));
  return ELL_OK;
}

// Layout tuning (process-wide; read when a grid is created).  Each k-plane of
// a colour array is padded so that the planes a column walk touches in
// parallel do not all start at the same offset modulo the HBM channel
// interleave; the two colour arrays are offset from each other likewise.
int g_plane_pad = 64;
int g_colour_pad = 256;
int g_stencil_seg = 1;  // k-segments of the CG operator kernels (1, 2 or 4)
int g_apply_tile = 1;   // 1: LDS-tiled CG operator step where both horizontal directions exist
int g_batch_graph = 1;  // 1: batch engines replay each grouped step from a captured graph
int g_smooth_tile = 1;  // 1: FP64 half-sweeps stage the other colour in LDS tiles
int g_fused_dot = 1;    // 1: the last post-smoothing half-sweeps form the CG dots
int g_fused_update = 1; // 1: the first pre-smoothing pair updates the CG residual
int g_fused_prolong = 1;  // 1: the first post-smoothing sweep applies the finest correction
int g_tiled_ends = 1;     // 1: a solve's start and end on LDS tiles where both horizontal directions exist
int g_coarse_pair = 1;    // 1: each coarsest-level sweep pair in one launch (k_coarse_pair) where it applies
int g_coarse_tail = 0;    // 1: the coarsest level's sweeps in one cooperative launch where it applies
                          //    (off by default: measured slower than one launch per half-sweep)

// Smoother segments per column: enough lanes to occupy the chip on small
// levels, four (the register-resident optimum) on large ones; the finest
// level uses eight for 64 <= nz <= 128, else four.
int smoother_segments(long long cols_per_colour, int nz, bool finest) {
  // finest level: 8 segments where a kernel instance covers them (nz in
  // [64, 128]); measured 1% faster than 4 at 512^2 x 128
  if (finest) return (nz >= 64 && seg_len(nz, 8) <= 16) ? 8 : 4;
  int ns = 4;
  {
    if (cols_per_colour < 4096) ns = 16;
    else if (cols_per_colour < 16384) ns = 8;
  }
  while (ns > 4 && seg_len(nz, ns) < 8) ns /= 2;  // keep at least 8 levels per lane
  return ns;
}

int batch_coarse_segments(long long cols_per_colour, int nz) {
  const int L8 = seg_len(nz, 8);
  return cols_per_colour < 16384 && L8 >= 8 && L8 <= 16 ? 8 : 4;
}

Geo make_geo(int nx, int ny, int nz, bool finest = false, bool uniform_seg = false) {
  Geo G;
  G.nx = nx;
  G.ny = ny;
  G.nz = nz;
  long long ncols = (long long)nx * ny;
  G.H = (int)((ncols + 1) / 2);
  G.ncol0 = (int)((ncols + 1) / 2);
  G.ncol1 = (int)(ncols / 2);
  G.hx2 = nx > 1 ? nx / 2 : 0;
  G.has_x = nx > 1;
  G.has_y = ny > 1;
  G.P = nz + 1;
  G.S = (int)(((long long)G.H + 63) / 64 * 64 + g_plane_pad);
  G.cs = (long long)nz * G.S + g_colour_pad;
  // batch grids: the finest level as a single grid; on coarse levels the
  // grouped launches come in two block shapes, four segments, or eight on
  // the small (latency-bound) levels where a segment holds 8..16 levels
  G.nseg = uniform_seg && !finest ? batch_coarse_segments(G.H, nz) : smoother_segments(G.H, nz, finest);
  return G;
}

int validate(const ell_grid_desc *d, int *levels) {
  if (!d) return fail(ELL_ERR_INVALID, "descriptor is NULL");
  if (d->nx < 1 || d->ny < 1 || d->nz < 1) return fail(ELL_ERR_INVALID, "sizes must be >= 1");
  if ((d->nx > 1 && d->nx % 2) || (d->ny > 1 && d->ny % 2))
    return fail(ELL_ERR_INVALID, "nx and ny must each be even or 1 (red/black colouring)");
  if ((long long)d->nx * d->ny > (1LL << 30) || (long long)d->nx * d->ny * d->nz > (1LL << 36))
    return fail(ELL_ERR_INVALID, "grid too large");
  if (!(d->hx > 0) || !(d->hy > 0) || !std::isfinite(d->hx) || !std::isfinite(d->hy))
    return fail(ELL_ERR_INVALID, "hx and hy must be positive");
  if (!(d->omega2 >= 0) || !std::isfinite(d->omega2)) return fail(ELL_ERR_INVALID, "omega2 must be >= 0");
  if (!d->dz || !d->lambda2) return fail(ELL_ERR_INVALID, "dz and lambda2 are required");
  for (int k = 0; k < d->nz; ++k) {
    if (!(d->dz[k] > 0) || !std::isfinite(d->dz[k])) return fail(ELL_ERR_INVALID, "dz[%d] must be positive", k);
    if (!(d->lambda2[k] > 0) || !std::isfinite(d->lambda2[k]))
      return fail(ELL_ERR_INVALID, "lambda2[%d] must be positive", k);
  }
  if (d->nu_pre < 0 || d->nu_post < 0 || d->nu_coarse < 0 || d->nu_pre > 64 || d->nu_post > 64 ||
      d->nu_coarse > 1024)
    return fail(ELL_ERR_INVALID, "sweep counts out of range");
  if (!(d->rho > 0 && d->rho < 2)) return fail(ELL_ERR_INVALID, "rho must lie in (0, 2)");
  if (d->prolong != 0 && d->prolong != 1) return fail(ELL_ERR_INVALID, "prolong must be 0 or 1");
  if (d->precision < ELL_FP64 || d->precision > ELL_FP32_BF16COEF)
    return fail(ELL_ERR_INVALID, "unknown precision");
  const int Ls = standard_depth(d->nx, d->ny);
  int L = d->n_levels <= 0 ? Ls : d->n_levels;
  if (L > Ls) return fail(ELL_ERR_INVALID, "n_levels %d exceeds the possible depth %d", d->n_levels, Ls);
  *levels = L;
  return ELL_OK;
}

// Products of the recurrence multipliers over each of the nseg k-segments of
// a column: pf[k] = prod_{i=start..k} Tz[i] ip[i] (forward),
// qb[k] = prod_{i=k..end-1} cf[i] (backward), in the table's precision.
template <typename T>
void segment_products(int nz, int nseg, const T *Tz, const T *ip, const T *cf, T *pf, T *qb) {
  const int Ls = seg_len(nz, nseg);
  for (int s0 = 0; s0 < nz; s0 += Ls) {
    const int e = std::min(s0 + Ls, nz);
    T acc = T(1);
    for (int k = s0; k < e; ++k) {
      acc = acc * (Tz[k] * ip[k]);
      pf[k] = acc;
    }
    acc = T(1);
    for (int k = e - 1; k >= s0; --k) {
      acc = acc * cf[k];
      qb[k] = acc;
    }
  }
}

// Coefficients of level l in FP64: V, Tx, Ty, Tz (nz+1), and the Thomas
// factors 1/p_k and T_{k+1/2}/p_k of the column matrix
//   diag s_k + T_{k-1/2} + T_{k+1/2}, off-diagonals -T_{k+-1/2},
// with the pivot written p_k = T_{k+1/2} + e_k, e_0 = s_0,
// e_k = s_k + T_{k-1/2} e_{k-1} / (T_{k-1/2} + e_{k-1}); s_k = V_k + 2Tx_k + 2Ty_k
// is the part of the diagonal that the vertical couplings do not cancel.
// Face coefficients: omega^2 * area / distance; vertical faces combine the two
// half-cell resistances dz/(2 lambda^2) in series (Sec. 3.1).
// The stencil part of level l's table (slots TV..TZ, each P = nz+1 long, at t)
// from a descriptor; dz and lam: its nz thicknesses and lambda^2 values.
void stencil_coeffs(const ell_grid_desc &d, const double *dz, const double *lam, int l, double *t) {
  const int nz = d.nz, P = nz + 1;
  const int nx = d.nx >> l, ny = d.ny >> l;
  const double hx = d.hx * (double)(1 << l), hy = d.hy * (double)(1 << l);
  const double w2 = d.omega2;
  double *V = &t[TV * P], *Tx = &t[TX * P], *Ty = &t[TY * P], *Tz = &t[TZ * P];
  for (int k = 0; k < nz; ++k) {
    V[k] = hx * hy * dz[k];
    Tx[k] = nx > 1 ? w2 * hy * dz[k] / hx : 0.0;
    Ty[k] = ny > 1 ? w2 * hx * dz[k] / hy : 0.0;
  }
  V[nz] = Tx[nz] = Ty[nz] = 0.0;
  Tz[0] = 0.0;
  Tz[nz] = 0.0;
  for (int k = 1; k < nz; ++k) {
    const double res = dz[k - 1] / (2.0 * lam[k - 1]) + dz[k] / (2.0 * lam[k]);
    Tz[k] = w2 * hx * hy / res;
  }
}

void level_table64(const ell_grid *g, int l, std::vector<double> &t) {
  const int nz = g->d.nz, P = nz + 1;
  t.assign((size_t)TSLOTS * P, 0.0);
  stencil_coeffs(g->d, g->dz.data(), g->lam.data(), l, t.data());
  const double *V = &t[TV * P], *Tx = &t[TX * P], *Ty = &t[TY * P], *Tz = &t[TZ * P];
  double *ip = &t[TIP * P], *cf = &t[TCF * P];
  double e = 0.0;
  for (int k = 0; k < nz; ++k) {
    const double s = (V[k] + 2.0 * Tx[k]) + 2.0 * Ty[k];
    e = k == 0 ? s : s + Tz[k] * e / (Tz[k] + e);
    const double p = Tz[k + 1] + e;
    ip[k] = 1.0 / p;
    cf[k] = Tz[k + 1] / p;
  }
  segment_products(nz, g->lev[l].geo.nseg, Tz, ip, cf, &t[TPF * P], &t[TQB * P]);
}

// FP32 tables: either the FP64 values rounded once, or (BF16 mode) the
// stencil coefficients rounded to bfloat16 and the Thomas factors recomputed
// in FP32 from those rounded coefficients.
void level_table32(const ell_grid *g, int l, const std::vector<double> &t64, std::vector<float> &t) {
  const int nz = g->d.nz, P = nz + 1;
  t.assign((size_t)TSLOTS * P, 0.0f);
  for (size_t i = 0; i < t64.size(); ++i) t[i] = (float)t64[i];
  if (g->prec != ELL_FP32_BF16COEF) {
    segment_products(nz, g->lev[l].geo.nseg, &t[TZ * P], &t[TIP * P], &t[TCF * P], &t[TPF * P],
                     &t[TQB * P]);
    return;
  }
  for (int s = TV; s <= TZ; ++s)
    for (int k = 0; k < P; ++k) t[s * P + k] = round_bf16(t[s * P + k]);
  float *V = &t[TV * P], *Tx = &t[TX * P], *Ty = &t[TY * P], *Tz = &t[TZ * P];
  float *ip = &t[TIP * P], *cf = &t[TCF * P];
  float e = 0.0f;
  for (int k = 0; k < nz; ++k) {
    const float s = (V[k] + 2.0f * Tx[k]) + 2.0f * Ty[k];
    e = k == 0 ? s : s + Tz[k] * e / (Tz[k] + e);
    const float p = Tz[k + 1] + e;
    ip[k] = 1.0f / p;
    cf[k] = Tz[k + 1] / p;
  }
  segment_products(nz, g->lev[l].geo.nseg, Tz, ip, cf, &t[TPF * P], &t[TQB * P]);
}

size_t grid_bytes(const ell_grid_desc *d, int L) {
  const size_t es = d->precision == ELL_FP64 ? 8 : 4;
  const Geo g0 = make_geo(d->nx, d->ny, d->nz);
  const size_t n0 = 2 * (size_t)g0.cs;
  size_t bytes = 7 * n0 * 8;                           // u, r, z, p (x3), q (FP64)
  if (d->precision != ELL_FP64) bytes += 2 * n0 * 4;   // b32, z32
  if (d->rho != 1.0) bytes += (size_t)g0.cs * es;      // ybuf
  for (int l = 0; l < L; ++l) {
    const Geo G = make_geo(d->nx >> l, d->ny >> l, d->nz);
    bytes += (size_t)TSLOTS * G.P * es;
    if (l > 0) bytes += 2 * 2 * (size_t)G.cs * es;
  }
  const long long nb = partial_blocks(g0, n0);
  bytes += (size_t)nb * 2 * 8 + sizeof(PcgState) + (size_t)d->nz * 8;
  return bytes;
}

// Per-column vertical coefficients of every level (horizontally varying
// lambda^2): level 0's faces by the harmonic rule of level_table64 in each
// column, T_{k-1/2} = omega^2 hx hy / (dz_{k-1}/(2 lambda^2_{k-1}) +
// dz_k/(2 lambda^2_k)); a coarse column's face is the sum of its four
// children's, ((0,0) + (1,0)) + ((0,1) + (1,1)) (parallel faces).  Each
// column's Thomas elimination in excess form with the level's shared excess
// s_k = V_k + 2 Tx_k + 2 Ty_k gives 1/p_k and T_{k+1/2}/p_k.  Uploaded in the
// split layout of the level.
int build_varying(ell_grid *g, const double *lam3) {
  const ell_grid_desc &d = g->d;
  const int nz = d.nz;
  std::vector<double> fz, fzc, t64, tz_s, ip_s, cf_s;
  {
    const size_t plane = (size_t)d.nx * d.ny;
    fz.assign((size_t)(nz + 1) * plane, 0.0);
    for (int k = 1; k < nz; ++k)
      for (size_t c = 0; c < plane; ++c) {
        const double res = g->dz[k - 1] / (2.0 * lam3[(size_t)(k - 1) * plane + c]) +
                           g->dz[k] / (2.0 * lam3[(size_t)k * plane + c]);
        fz[(size_t)k * plane + c] = d.omega2 * d.hx * d.hy / res;
      }
  }
  for (int l = 0; l < g->L; ++l) {
    Level &Lv = g->lev[l];
    const Geo &G = Lv.geo;
    const int nx = G.nx, ny = G.ny;
    if (l > 0) {  // sum the children of the previous level's faces
      const int fx = nx * 2, fy = ny * 2;
      fzc.assign((size_t)(nz + 1) * nx * ny, 0.0);
      for (int k = 0; k <= nz; ++k)
        for (int J = 0; J < ny; ++J)
          for (int I = 0; I < nx; ++I) {
            const double *f = &fz[(size_t)k * fx * fy];
            const double a = f[(size_t)(2 * J) * fx + 2 * I] + f[(size_t)(2 * J) * fx + 2 * I + 1];
            const double b = f[(size_t)(2 * J + 1) * fx + 2 * I] + f[(size_t)(2 * J + 1) * fx + 2 * I + 1];
            fzc[((size_t)k * ny + J) * nx + I] = a + b;
          }
      fz.swap(fzc);
    }
    const size_t plane = (size_t)nx * ny;
    level_table64(g, l, t64);
    const int P = nz + 1;
    const size_t ne = 2 * (size_t)G.cs;
    tz_s.assign(ne, 0.0);
    ip_s.assign(ne, 0.0);
    cf_s.assign(ne, 0.0);
    for (int j = 0; j < ny; ++j)
      for (int i = 0; i < nx; ++i) {
        const int c = (i + j) & 1;
        const long long m = nx > 1 ? (long long)j * G.hx2 + (i >> 1) : (j >> 1);
        const size_t col = (size_t)j * nx + i;
        double e = 0.0;
        for (int k = 0; k < nz; ++k) {
          const double s = (t64[TV * P + k] + 2.0 * t64[TX * P + k]) + 2.0 * t64[TY * P + k];
          const double tb = fz[(size_t)k * plane + col], ta = fz[(size_t)(k + 1) * plane + col];
          e = k == 0 ? s : s + tb * e / (tb + e);
          const double p = ta + e;
          const size_t o = (size_t)c * G.cs + (size_t)k * G.S + m;
          tz_s[o] = tb;
          ip_s[o] = 1.0 / p;
          cf_s[o] = ta / p;
        }
      }
    void *tmp;
    const std::vector<double> *src[3] = {&tz_s, &ip_s, &cf_s};
    double **dst[3] = {&Lv.tz3, &Lv.ip3, &Lv.cf3};
    float **dstf[3] = {&Lv.tz3f, &Lv.ip3f, &Lv.cf3f};
    std::vector<float> f32;
    for (int a = 0; a < 3; ++a) {
      CHK(dalloc(g, &tmp, ne * 8));
      *dst[a] = (double *)tmp;
      if (hipMemcpy(tmp, src[a]->data(), ne * 8, hipMemcpyHostToDevice) != hipSuccess)
        return fail(ELL_ERR_HIP, "coefficient upload failed");
      if (g->prec != ELL_FP64) {  // the FP64 values rounded once, as level_table32 rounds the tables
        f32.assign(src[a]->begin(), src[a]->end());
        CHK(dalloc(g, &tmp, ne * 4));
        *dstf[a] = (float *)tmp;
        if (hipMemcpy(tmp, f32.data(), ne * 4, hipMemcpyHostToDevice) != hipSuccess)
          return fail(ELL_ERR_HIP, "coefficient upload failed");
      }
    }
  }
  return ELL_OK;
}

// ------------------------------------------------------------------------
// profiling helpers
// ------------------------------------------------------------------------
struct ProfScope {
  Prof *p;
  hipStream_t s;
  bool on;
  ProfScope(ell_grid *g, int fam, hipStream_t st, bool enabled = true) : p(&g->prof[fam]), s(st) {
    on = enabled && !p->paused && p->cap > 0 && p->n < p->cap;
    if (on) (void)hipEventRecord(p->ev[2 * p->n], s);
  }
  ~ProfScope() {
    if (on) {
      (void)hipEventRecord(p->ev[2 * p->n + 1], s);
      p->n++;
    }
  }
};

// ------------------------------------------------------------------------
// kernel launchers (element type R = double or float)
// ------------------------------------------------------------------------
template <typename R, bool FINE, bool HXY>
void smooth_dispatch(int nb, hipStream_t s, const Geo &G, const R *tab, int c, bool zero, bool rho1,
                     const R *bo, const R *uo, R *own, R *yb, R rho, const int *done) {
  if (zero && rho1) k_smooth<R, true, true, FINE, HXY><<<nb, kBlock, 0, s>>>(G, tab, c, bo, uo, own, yb, rho, done);
  else if (zero) k_smooth<R, true, false, FINE, HXY><<<nb, kBlock, 0, s>>>(G, tab, c, bo, uo, own, yb, rho, done);
  else if (rho1) k_smooth<R, false, true, FINE, HXY><<<nb, kBlock, 0, s>>>(G, tab, c, bo, uo, own, yb, rho, done);
  else k_smooth<R, false, false, FINE, HXY><<<nb, kBlock, 0, s>>>(G, tab, c, bo, uo, own, yb, rho, done);
}

template <typename R, typename TB, bool FINE, int SEG, int NSEG>
void seg_dispatch3(int nb, hipStream_t s, const Geo &G, const R *tab, int c, bool zero, bool rho1,
                   const TB *bo, const R *uo, R *own, R rho, const int *done) {
  constexpr int T = NSEG * 64;
  if (zero && rho1)
    k_smooth_seg<R, true, true, FINE, SEG, NSEG, TB><<<nb, T, 0, s>>>(G, tab, c, bo, uo, own, rho, done);
  else if (zero)
    k_smooth_seg<R, true, false, FINE, SEG, NSEG, TB><<<nb, T, 0, s>>>(G, tab, c, bo, uo, own, rho, done);
  else if (rho1)
    k_smooth_seg<R, false, true, FINE, SEG, NSEG, TB><<<nb, T, 0, s>>>(G, tab, c, bo, uo, own, rho, done);
  else
    k_smooth_seg<R, false, false, FINE, SEG, NSEG, TB><<<nb, T, 0, s>>>(G, tab, c, bo, uo, own, rho, done);
}

// returns false if no instantiation covers (nseg, segment length)
template <typename R, typename TB>
bool seg_dispatch(bool fine, int nb, hipStream_t s, const Geo &G, const R *tab, int c, bool zero, bool rho1,
                  const TB *bo, const R *uo, R *own, R rho, const int *done) {
  const int Ls = seg_len(G.nz, G.nseg);
  if (fine) {
    if (G.nseg == 8) {
      if (Ls > 16) return false;
      seg_dispatch3<R, TB, true, 16, 8>(nb, s, G, tab, c, zero, rho1, bo, uo, own, rho, done);
      return true;
    }
    if (G.nseg != 4) return false;
    if (Ls <= 16) seg_dispatch3<R, TB, true, 16, 4>(nb, s, G, tab, c, zero, rho1, bo, uo, own, rho, done);
    else if (Ls <= 32) seg_dispatch3<R, TB, true, 32, 4>(nb, s, G, tab, c, zero, rho1, bo, uo, own, rho, done);
    else if (Ls <= 64) seg_dispatch3<R, TB, true, 64, 4>(nb, s, G, tab, c, zero, rho1, bo, uo, own, rho, done);
    else return false;
    return true;
  }
  if constexpr (!std::is_same<R, TB>::value) {
    return false;  // mixed element types only on the finest level
  } else {
    switch (G.nseg) {
      case 4:
        if (Ls <= 16) seg_dispatch3<R, TB, false, 16, 4>(nb, s, G, tab, c, zero, rho1, bo, uo, own, rho, done);
        else if (Ls <= 32) seg_dispatch3<R, TB, false, 32, 4>(nb, s, G, tab, c, zero, rho1, bo, uo, own, rho, done);
        else if (Ls <= 64) seg_dispatch3<R, TB, false, 64, 4>(nb, s, G, tab, c, zero, rho1, bo, uo, own, rho, done);
        else return false;
        return true;
      case 8:
        if (Ls <= 8) seg_dispatch3<R, TB, false, 8, 8>(nb, s, G, tab, c, zero, rho1, bo, uo, own, rho, done);
        else if (Ls <= 16) seg_dispatch3<R, TB, false, 16, 8>(nb, s, G, tab, c, zero, rho1, bo, uo, own, rho, done);
        else if (Ls <= 32) seg_dispatch3<R, TB, false, 32, 8>(nb, s, G, tab, c, zero, rho1, bo, uo, own, rho, done);
        else return false;
        return true;
      case 16:
        if (Ls <= 8) seg_dispatch3<R, TB, false, 8, 16>(nb, s, G, tab, c, zero, rho1, bo, uo, own, rho, done);
        else if (Ls <= 16) seg_dispatch3<R, TB, false, 16, 16>(nb, s, G, tab, c, zero, rho1, bo, uo, own, rho, done);
        else return false;
        return true;
    }
    return false;
  }
}

// The LDS-tiled half-sweep applies to level l (after a first sweep).
bool tile_ok(const ell_grid *g, int l) {
  const Geo &G = g->lev[l].geo;
  const int Ls = seg_len(G.nz, G.nseg);
  // pairs of columns load as one vector: even half-width, plane and colour strides
  return g->d.rho == 1.0 && G.has_x && G.has_y && g->smooth_tile && !g->varying && G.hx2 % 2 == 0 &&
         G.ny % 2 == 0 && G.S % 2 == 0 && G.cs % 2 == 0 &&
         ((G.nseg == 16 && Ls <= 8) || (G.nseg == 8 && Ls <= 16) || (G.nseg == 4 && Ls <= 32));
}

// Blocks (tiles of 32 x 2 columns of one colour) of a tiled half-sweep.
inline int smooth_tiles(const Geo &G) { return ((G.hx2 + kSTX - 1) / kSTX) * (G.ny / 2); }

// The per-column-coefficient sweep (k_smooth_seg3) of one colour of a level:
// one block per 64 columns, sixteen k-segments on small (latency-bound)
// levels, eight on large ones.
struct Seg3Shape {
  int nbs;     // blocks (each writes a partial slot in the fused forms)
  bool small;  // sixteen segments
  int Ls;      // levels per segment
};
inline Seg3Shape seg3_shape(const Geo &G, int c) {
  const int ncol = c ? G.ncol1 : G.ncol0;
  Seg3Shape sh;
  sh.nbs = blocks8(((long long)ncol + kSegCols - 1) / kSegCols * kBlock);
  sh.small = G.H < 16384 && seg_len(G.nz, 16) <= 16;
  sh.Ls = seg_len(G.nz, sh.small ? 16 : 8);
  return sh;
}

// Where the per-column sweep applies: a grid with per-column coefficients,
// rho = 1, both horizontal directions, at most 256 levels.
bool seg3_ok(const ell_grid *g, int l) {
  const Geo &G = g->lev[l].geo;
  return g->varying && g->d.rho == 1.0 && G.has_x && G.has_y && G.nz <= 256;
}

int dot_colour_slots(const ell_grid *g, int c);

template <typename R, typename TB, typename F, bool Z, bool FN, int DOT = 0, bool UPD = false>
void seg3_launch(hipStream_t s, const Geo &G, const R *tab, int c, const TB *bo, const R *uo, R *own,
                 const int *done, const F *t3, const F *i3, const F *c3, double *partial = nullptr, int pbase = 0,
                 double *rw = nullptr, const double *qo = nullptr, const PcgState *st = nullptr) {
  const Seg3Shape sh = seg3_shape(G, c);
  auto go = [&](auto seg, auto nseg, auto ch) {
    constexpr int SEG = decltype(seg)::value, NSEG = decltype(nseg)::value, CH = decltype(ch)::value;
    k_smooth_seg3<R, TB, F, Z, FN, SEG, NSEG, CH, DOT, UPD><<<sh.nbs, NSEG * 64, 0, s>>>(
        G, tab, c, bo, uo, own, done, t3, i3, c3, partial, pbase, rw, qo, st);
  };
  using I4 = std::integral_constant<int, 4>;
  using I8 = std::integral_constant<int, 8>;
  using I16 = std::integral_constant<int, 16>;
  using I32 = std::integral_constant<int, 32>;
  if (sh.small) {
    if (sh.Ls <= 8) go(I8{}, I16{}, I4{});
    else go(I16{}, I16{}, I4{});
  } else {
    if (sh.Ls <= 8) go(I8{}, I8{}, I8{});
    else if (sh.Ls <= 16) go(I16{}, I8{}, I8{});
    else go(I32{}, I8{}, I8{});
  }
}

// One colour of line relaxation on level l.  tab: coefficient table in the
// arithmetic type R (nullptr: the level's own table).  TB != R is supported
// on the finest level only.
template <typename R, typename TB = R>
int launch_smooth(ell_grid *g, int l, int c, bool zero, const TB *b, R *u, const int *done, hipStream_t s,
                  const R *tab = nullptr) {
  const Level &Lv = g->lev[l];
  const Geo &G = Lv.geo;
  const int ncol = c ? G.ncol1 : G.ncol0;
  if (ncol == 0) return ELL_OK;
  const int nb = blocks8(ncol);
  if (!tab) tab = (const R *)Lv.tab;
  const bool rho1 = g->d.rho == 1.0;
  R *yb = (R *)g->ybuf;
  const R rho = (R)g->d.rho;
  const TB *bo = b + (long long)c * G.cs;
  const R *uo = u + (long long)(1 - c) * G.cs;
  R *own = u + (long long)c * G.cs;
  const bool hxy = G.has_x && G.has_y;
  ProfScope ps(g, ELL_K_SMOOTH0, s, l == 0);
  if (g->varying) {
    // every column its own factors, in the arithmetic type: the FP32 sweeps
    // of the mixed-precision V-cycles read the FP32 copies, the FP64 finest
    // post-smoothing the FP64 fields.  Rounding T_{k+1/2}/p_k to FP32 loses the
    // excess of a strongly coupled column (T/p = 1 - O(1e-7) or closer), so
    // FP32 factors there would undo what that sweep is for.
    if (rho1 && hxy && G.nz <= 256) {
      auto go = [&](auto z, auto fn, const auto *t3, const auto *i3, const auto *c3) {
        constexpr bool Z = decltype(z)::value, FN = decltype(fn)::value;
        using F = std::remove_cv_t<std::remove_pointer_t<decltype(t3)>>;
        seg3_launch<R, TB, F, Z, FN>(s, G, tab, c, bo, uo, own, done, t3, i3, c3);
      };
      auto go_f = [&](auto z, auto fn) {
        if constexpr (std::is_same<R, double>::value)
          go(z, fn, Lv.tz3, Lv.ip3, Lv.cf3);
        else
          go(z, fn, (const float *)Lv.tz3f, (const float *)Lv.ip3f, (const float *)Lv.cf3f);
      };
      using T_ = std::true_type;
      using F_ = std::false_type;
      if constexpr (std::is_same<R, TB>::value) {
        if (zero) { if (l == 0) go_f(T_{}, T_{}); else go_f(T_{}, F_{}); }
        else { if (l == 0) go_f(F_{}, T_{}); else go_f(F_{}, F_{}); }
      } else {  // mixed element types only on the finest level
        if (l != 0) return fail(ELL_ERR_INVALID, "mixed element types only on the finest level");
        if (zero) go_f(T_{}, T_{});
        else go_f(F_{}, T_{});
      }
      return check_launch("k_smooth_seg3");
    }
    if constexpr (std::is_same<R, TB>::value) {
      // the column kernel, with fields in the arithmetic type
      const R *t3, *i3, *c3;
      if constexpr (std::is_same<R, double>::value) {
        t3 = Lv.tz3;
        i3 = Lv.ip3;
        c3 = Lv.cf3;
      } else {
        t3 = Lv.tz3f;
        i3 = Lv.ip3f;
        c3 = Lv.cf3f;
      }
      auto go = [&](auto z, auto r1, auto fn, auto h) {
        k_smooth<R, decltype(z)::value, decltype(r1)::value, decltype(fn)::value, decltype(h)::value, true>
            <<<nb, kBlock, 0, s>>>(G, tab, c, bo, uo, own, yb, rho, done, t3, i3, c3);
      };
      using T_ = std::true_type;
      using F_ = std::false_type;
      auto go2 = [&](auto fn, auto h) {
        if (zero && rho1) go(T_{}, T_{}, fn, h);
        else if (zero) go(T_{}, F_{}, fn, h);
        else if (rho1) go(F_{}, T_{}, fn, h);
        else go(F_{}, F_{}, fn, h);
      };
      if (l == 0) { if (hxy) go2(T_{}, T_{}); else go2(T_{}, F_{}); }
      else { if (hxy) go2(F_{}, T_{}); else go2(F_{}, F_{}); }
      return check_launch("k_smooth");
    } else {
      return fail(ELL_ERR_INVALID, "no line-relaxation kernel for this level shape");
    }
  }
  if constexpr (std::is_same<R, TB>::value) {
    // after the first sweep, rho = 1: the LDS-tiled half-sweep (streaming
    // accesses on the finest level; FP32 on the coarse levels of the
    // mixed-precision V-cycle)
    constexpr bool F64 = std::is_same<R, double>::value;
    const int Ls = seg_len(G.nz, G.nseg);
    if (!zero && tile_ok(g, l) && (F64 || l >= 1)) {
      const int nbt = blocks8((long long)smooth_tiles(G) * kBlock);
      if (l == 0) {
        if constexpr (F64) {
        if (G.nseg == 16)
          k_smooth_tile<8, 16, true><<<nbt, 16 * 64, 0, s>>>(G, tab, c, bo, uo, own, done);
        else if (G.nseg == 8)
          k_smooth_tile<16, 8, true><<<nbt, 8 * 64, 0, s>>>(G, tab, c, bo, uo, own, done);
        else if (Ls <= 16)
          k_smooth_tile<16, 4, true><<<nbt, 4 * 64, 0, s>>>(G, tab, c, bo, uo, own, done);
        else
          k_smooth_tile<32, 4, true><<<nbt, 4 * 64, 0, s>>>(G, tab, c, bo, uo, own, done);
        }
      } else {
        if (G.nseg == 16)
          k_smooth_tile<8, 16, false><<<nbt, 16 * 64, 0, s>>>(G, tab, c, bo, uo, own, done);
        else if (G.nseg == 8)
          k_smooth_tile<16, 8, false><<<nbt, 8 * 64, 0, s>>>(G, tab, c, bo, uo, own, done);
        else if (Ls <= 16)
          k_smooth_tile<16, 4, false><<<nbt, 4 * 64, 0, s>>>(G, tab, c, bo, uo, own, done);
        else
          k_smooth_tile<32, 4, false><<<nbt, 4 * 64, 0, s>>>(G, tab, c, bo, uo, own, done);
      }
      return check_launch("k_smooth_tile");
    }
  }
  if (hxy) {
    const int nbs = blocks8(((long long)ncol + kSegCols - 1) / kSegCols * kBlock);
    if (seg_dispatch<R, TB>(l == 0, nbs, s, G, tab, c, zero, rho1, bo, uo, own, rho, done))
      return check_launch("k_smooth_seg");
  }
  if constexpr (!std::is_same<R, TB>::value) {
    return fail(ELL_ERR_INVALID, "no line-relaxation kernel for this level shape");
  } else {
    if (l == 0) {
      if (hxy) smooth_dispatch<R, true, true>(nb, s, G, tab, c, zero, rho1, bo, uo, own, yb, rho, done);
      else smooth_dispatch<R, true, false>(nb, s, G, tab, c, zero, rho1, bo, uo, own, yb, rho, done);
    } else {
      if (hxy) smooth_dispatch<R, false, true>(nb, s, G, tab, c, zero, rho1, bo, uo, own, yb, rho, done);
      else smooth_dispatch<R, false, false>(nb, s, G, tab, c, zero, rho1, bo, uo, own, yb, rho, done);
    }
    return check_launch("k_smooth");
  }
}

template <int SEG, int NSEG>
void tile_dot(int dot, int nbt, hipStream_t s, const Geo &G, const double *tab, int c, const double *bo,
              const double *uo, double *own, const int *done, double *partial, int pbase, const double *qc) {
  if (dot == 1)
    k_smooth_tile_dot<SEG, NSEG, 1><<<nbt, NSEG * 64, 0, s>>>(G, tab, c, bo, uo, own, done, partial, pbase, qc);
  else
    k_smooth_tile_dot<SEG, NSEG, 2><<<nbt, NSEG * 64, 0, s>>>(G, tab, c, bo, uo, own, done, partial, pbase, qc);
}

// One of the finest level's last two post-smoothing half-sweeps of a CG
// preconditioner application, with the fused partial sums (dot = 1: <r, z>;
// 2: <r, z> and <z, q>) of its colour's columns into partial[pbase + tile].
// The caller has checked tile_ok(g, 0).
int launch_smooth_dot(ell_grid *g, int c, const double *b, double *u, const double *tab, int dot, int pbase,
                      const int *done, hipStream_t s) {
  const Geo &G = g->lev[0].geo;
  const int Ls = seg_len(G.nz, G.nseg);
  const double *bo = b + (long long)c * G.cs;
  const double *uo = u + (long long)(1 - c) * G.cs;
  double *own = u + (long long)c * G.cs;
  const double *qc = g->q + (long long)c * G.cs;
  const int nbt = blocks8((long long)smooth_tiles(G) * kBlock);
  ProfScope ps(g, ELL_K_SMOOTH0, s);
  if (g->varying) {  // the per-column sweep, FP64 fields
    const Level &Lv = g->lev[0];
    if (dot == 2)
      seg3_launch<double, double, double, false, true, 2>(s, G, tab, c, bo, uo, own, done, Lv.tz3, Lv.ip3, Lv.cf3,
                                                          g->partial, pbase, nullptr, qc);
    else
      seg3_launch<double, double, double, false, true, 1>(s, G, tab, c, bo, uo, own, done, Lv.tz3, Lv.ip3, Lv.cf3,
                                                          g->partial, pbase);
    return check_launch("k_smooth_seg3");
  }
  if (G.nseg == 16) tile_dot<8, 16>(dot, nbt, s, G, tab, c, bo, uo, own, done, g->partial, pbase, qc);
  else if (G.nseg == 8) tile_dot<16, 8>(dot, nbt, s, G, tab, c, bo, uo, own, done, g->partial, pbase, qc);
  else if (Ls <= 16) tile_dot<16, 4>(dot, nbt, s, G, tab, c, bo, uo, own, done, g->partial, pbase, qc);
  else tile_dot<32, 4>(dot, nbt, s, G, tab, c, bo, uo, own, done, g->partial, pbase, qc);
  return check_launch("k_smooth_tile_dot");
}

// One half-sweep of the finest level's first pre-smoothing pair of a CG
// preconditioner application with the residual update r -= alpha q fused in
// (colour 0 from zero with the column kernel; colour 1 on the tile for FP64,
// else the column kernel).  The partial sums of ||r||^2 go to partial[pbase +
// block]; *slots receives the number of slots written.  The caller has
// checked fused_update_path.
template <typename R>
int launch_smooth_upd(ell_grid *g, int c, double *r, R *u, const R *tab, int pbase, hipStream_t s, int *slots) {
  const Geo &G = g->lev[0].geo;
  const int Ls = seg_len(G.nz, G.nseg);
  double *rc = r + (long long)c * G.cs;
  const double *qc = g->q + (long long)c * G.cs;
  const R *uo = u + (long long)(1 - c) * G.cs;
  R *own = u + (long long)c * G.cs;
  ProfScope ps(g, ELL_K_SMOOTH0, s);
  if (g->varying) {  // the per-column sweep, fields in the arithmetic type
    const Level &Lv = g->lev[0];
    const int *done = &g->st->done;
    auto go = [&](auto z, const auto *t3, const auto *i3, const auto *c3) {
      constexpr bool Z = decltype(z)::value;
      using F = std::remove_cv_t<std::remove_pointer_t<decltype(t3)>>;
      seg3_launch<R, double, F, Z, true, 0, true>(s, G, tab, c, rc, uo, own, done, t3, i3, c3, g->partial, pbase,
                                                 rc, qc, g->st);
    };
    if constexpr (std::is_same<R, double>::value) {
      if (c == 0) go(std::true_type{}, Lv.tz3, Lv.ip3, Lv.cf3);
      else go(std::false_type{}, Lv.tz3, Lv.ip3, Lv.cf3);
    } else {
      const float *t3 = (const float *)Lv.tz3f, *i3 = (const float *)Lv.ip3f, *c3 = (const float *)Lv.cf3f;
      if (c == 0) go(std::true_type{}, t3, i3, c3);
      else go(std::false_type{}, t3, i3, c3);
    }
    *slots = seg3_shape(G, c).nbs;  // every block writes its slot
    return check_launch("k_smooth_seg3");
  }
  if constexpr (std::is_same<R, double>::value) {
    if (c == 1) {
      const int nbt = blocks8((long long)smooth_tiles(G) * kBlock);
      if (G.nseg == 8)
        k_smooth_tile_upd<16, 8><<<nbt, 8 * 64, 0, s>>>(G, tab, c, rc, uo, own, qc, g->st, g->partial, pbase);
      else if (Ls <= 16)
        k_smooth_tile_upd<16, 4><<<nbt, 4 * 64, 0, s>>>(G, tab, c, rc, uo, own, qc, g->st, g->partial, pbase);
      else
        k_smooth_tile_upd<32, 4><<<nbt, 4 * 64, 0, s>>>(G, tab, c, rc, uo, own, qc, g->st, g->partial, pbase);
      *slots = smooth_tiles(G);  // blocks past the last tile return at once
      return check_launch("k_smooth_tile_upd");
    }
  }
  const int ncol = c ? G.ncol1 : G.ncol0;
  const int nbs = blocks8(((long long)ncol + kSegCols - 1) / kSegCols * kBlock);
  if (G.nseg == 8) {
    if (c == 0) k_smooth_seg_upd<R, true, 16, 8><<<nbs, 8 * 64, 0, s>>>(G, tab, c, rc, uo, own, qc, g->st, g->partial, pbase);
    else k_smooth_seg_upd<R, false, 16, 8><<<nbs, 8 * 64, 0, s>>>(G, tab, c, rc, uo, own, qc, g->st, g->partial, pbase);
  } else if (Ls <= 16) {
    if (c == 0) k_smooth_seg_upd<R, true, 16, 4><<<nbs, 4 * 64, 0, s>>>(G, tab, c, rc, uo, own, qc, g->st, g->partial, pbase);
    else k_smooth_seg_upd<R, false, 16, 4><<<nbs, 4 * 64, 0, s>>>(G, tab, c, rc, uo, own, qc, g->st, g->partial, pbase);
  } else {
    if (c == 0) k_smooth_seg_upd<R, true, 32, 4><<<nbs, 4 * 64, 0, s>>>(G, tab, c, rc, uo, own, qc, g->st, g->partial, pbase);
    else k_smooth_seg_upd<R, false, 32, 4><<<nbs, 4 * 64, 0, s>>>(G, tab, c, rc, uo, own, qc, g->st, g->partial, pbase);
  }
  *slots = nbs;  // every block writes its slot
  return check_launch("k_smooth_seg_upd");
}

// The finest level's post-smoothing (nu_post = 1) of an FP64 V-cycle whose
// CG dots are fused: the colour-1 sweep applies the coarse correction to the
// colour-0 values it reads (no prolongation pass), the colour-0 sweep forms
// <r, z> (dot = 1; and <z, q>, dot = 2) of both colours into the first
// tile-count partial slots.  The caller has checked pro_path.
// The staged coarse values of a fused prolongation load in aligned pairs
// (k_smooth_tile_pro<..., PAIR>): coarse half-width, colour and plane strides
// even, the array aligned to a pair (16 bytes in FP64, 8 in FP32).
bool pro_pairs_ok(const Geo &C, const void *uc, uintptr_t pair_bytes = 16) {
  return C.nx % 4 == 0 && C.cs % 2 == 0 && C.S % 2 == 0 && (reinterpret_cast<uintptr_t>(uc) & (pair_bytes - 1)) == 0;
}

template <int SEG, int NSEG, bool FINE, typename R>
void launch_tile_pro(int nbt, hipStream_t s, const Geo &F, const Geo &C, const R *tab, const R *b1, const R *u,
                     R *u1, const R *uc, const int *done) {
  if (pro_pairs_ok(C, uc, 2 * sizeof(R)))
    k_smooth_tile_pro<SEG, NSEG, FINE, true><<<nbt, NSEG * 64, 0, s>>>(F, C, tab, b1, u, u1, uc, done);
  else
    k_smooth_tile_pro<SEG, NSEG, FINE, false><<<nbt, NSEG * 64, 0, s>>>(F, C, tab, b1, u, u1, uc, done);
}

template <int SEG, int NSEG>
void pro_pair_k(ell_grid *g, const double *b, double *u, const int *done, hipStream_t s, int dot) {
  const Geo &F = g->lev[0].geo, &C = g->lev[1].geo;
  const double *tab = (const double *)g->lev[0].tab;
  const int nbt = blocks8((long long)smooth_tiles(F) * kBlock);
  const long long cs = F.cs;
  {
    ProfScope ps(g, ELL_K_SMOOTH0, s);
    launch_tile_pro<SEG, NSEG, true>(nbt, s, F, C, tab, b + cs, u, u + cs, (const double *)g->lev[1].u, done);
  }
  ProfScope ps(g, ELL_K_SMOOTH0, s);
  if (dot == 2)
    k_smooth_tile_dot4<SEG, NSEG><<<nbt, NSEG * 64, 0, s>>>(F, tab, b, u + cs, u, done, g->partial, b + cs, g->q,
                                                            g->q + cs);
  else
    k_smooth_tile_dot3<SEG, NSEG><<<nbt, NSEG * 64, 0, s>>>(F, tab, b, u + cs, u, done, g->partial, b + cs);
}

// A coarse level's prolongation rides on its first post-smoothing sweep the
// same way: FP64 level with a coarser one below it and the LDS-tiled sweep,
// rho = 1 (the colour-0 sweep that follows overwrites colour 0 without
// reading it, the colour-1 sweep overwrites colour 1), bilinear prolongation.
// R = float: the coarse levels of the mixed-precision V-cycle (the FP32
// prolongation's values, in FP32).
template <typename R>
bool coarse_pro_ok(const ell_grid *g, int l) {
  const bool prec = std::is_same<R, double>::value ? g->prec == ELL_FP64 : g->prec != ELL_FP64;
  return l >= 1 && l <= g->L - 2 && prec && g->fused_prolong && g->d.nu_post >= 1 && g->d.prolong == 0 &&
         tile_ok(g, l);
}

template <typename R>
int coarse_pro_sweep(ell_grid *g, int l, const R *b, R *u, const int *done, hipStream_t s) {
  const Geo &F = g->lev[l].geo, &C = g->lev[l + 1].geo;
  const R *tab = (const R *)g->lev[l].tab, *uc = (const R *)g->lev[l + 1].u;
  const int nbt = blocks8((long long)smooth_tiles(F) * kBlock);
  const int Ls = seg_len(F.nz, F.nseg);
  const long long cs = F.cs;
  if (F.nseg == 16) launch_tile_pro<8, 16, false>(nbt, s, F, C, tab, b + cs, u, u + cs, uc, done);
  else if (F.nseg == 8) launch_tile_pro<16, 8, false>(nbt, s, F, C, tab, b + cs, u, u + cs, uc, done);
  else if (Ls <= 16) launch_tile_pro<16, 4, false>(nbt, s, F, C, tab, b + cs, u, u + cs, uc, done);
  else launch_tile_pro<32, 4, false>(nbt, s, F, C, tab, b + cs, u, u + cs, uc, done);
  return check_launch("k_smooth_tile_pro");
}

int pro_pair(ell_grid *g, const double *b, double *u, const int *done, hipStream_t s, int dot) {
  const Geo &F = g->lev[0].geo;
  const int Ls = seg_len(F.nz, F.nseg);
  if (F.nseg == 16) pro_pair_k<8, 16>(g, b, u, done, s, dot);
  else if (F.nseg == 8) pro_pair_k<16, 8>(g, b, u, done, s, dot);
  else if (Ls <= 16) pro_pair_k<16, 4>(g, b, u, done, s, dot);
  else pro_pair_k<32, 4>(g, b, u, done, s, dot);
  return check_launch("k_smooth_tile_pro / k_smooth_tile_dot3 / k_smooth_tile_dot4");
}

// The first pre-smoothing pair with the fused residual update, then the
// convergence test (F_CONV) that the rest of the V-cycle is predicated on.
template <typename R>
int pre_pair_upd(ell_grid *g, double *r, R *u, const R *tab, hipStream_t s) {
  int s0 = 0, s1 = 0;
  CHK(launch_smooth_upd<R>(g, 0, r, u, tab, 0, s, &s0));
  CHK(launch_smooth_upd<R>(g, 1, r, u, tab, s0, s, &s1));
  k_finalize<<<1, kBlock, 0, s>>>(g->partial, s0 + s1, 1, g->st, F_CONV, 0.0, 0.0, 0);
  return check_launch("k_finalize");
}

// k-segments of the restriction and prolongation kernels: four on large
// levels, more on small coarse levels, where the sequential walk over a
// segment is the kernel's latency; at least 8 levels per segment.
inline int transfer_segments(long long slots, int nz) {
  int ns = slots >= 32768 ? 4 : (slots >= 8192 ? 8 : 16);
  while (ns > 4 && seg_len(nz, ns) < 8) ns /= 2;
  return ns;
}

template <typename R, typename TB = R>
int launch_restrict(ell_grid *g, int l, const TB *b, const R *u, R *bc, bool bz, const int *done,
                    hipStream_t s) {
  const Geo &F = g->lev[l].geo, &C = g->lev[l + 1].geo;
  const int nb = blocks8(2LL * C.H);
  const R *tab = (const R *)g->lev[l].tab;
  ProfScope ps(g, ELL_K_RESTRICT0, s, l == 0);
  if (g->varying) {  // per-column faces, in the arithmetic type
    const R *tz3;
    if constexpr (std::is_same<R, double>::value) tz3 = g->lev[l].tz3;
    else tz3 = g->lev[l].tz3f;
    if (bz && F.has_x && F.has_y) {  // k-segmented, colour-0 children only
      const int nbz = seg_blocks(2LL * C.H);
      const int ns = transfer_segments(2LL * C.H, F.nz);
      if (ns == 16) k_resid_restrict_bz<R, TB, 16, true><<<nbz, 16 * 64, 0, s>>>(F, C, tab, b, u, bc, done, tz3);
      else if (ns == 8) k_resid_restrict_bz<R, TB, 8, true><<<nbz, 8 * 64, 0, s>>>(F, C, tab, b, u, bc, done, tz3);
      else k_resid_restrict_bz<R, TB, 4, true><<<nbz, 4 * 64, 0, s>>>(F, C, tab, b, u, bc, done, tz3);
      return check_launch("k_resid_restrict_bz");
    }
    if (bz) k_resid_restrict<R, true, true, TB><<<nb, kBlock, 0, s>>>(F, C, tab, b, u, bc, done, tz3);
    else k_resid_restrict<R, false, true, TB><<<nb, kBlock, 0, s>>>(F, C, tab, b, u, bc, done, tz3);
    return check_launch("k_resid_restrict");
  }
  if (bz && F.has_x && F.has_y) {
    const int nbz = seg_blocks(2LL * C.H);
    const int ns = transfer_segments(2LL * C.H, F.nz);
    if (ns == 16) k_resid_restrict_bz<R, TB, 16><<<nbz, 16 * 64, 0, s>>>(F, C, tab, b, u, bc, done);
    else if (ns == 8) k_resid_restrict_bz<R, TB, 8><<<nbz, 8 * 64, 0, s>>>(F, C, tab, b, u, bc, done);
    else k_resid_restrict_bz<R, TB, 4><<<nbz, 4 * 64, 0, s>>>(F, C, tab, b, u, bc, done);
    return check_launch("k_resid_restrict_bz");
  }
  if constexpr (!std::is_same<R, TB>::value) {
    return fail(ELL_ERR_INVALID, "mixed-type restriction needs the colour-1 shortcut");
  } else {
    if (bz) k_resid_restrict<R, true><<<nb, kBlock, 0, s>>>(F, C, tab, b, u, bc, done);
    else k_resid_restrict<R, false><<<nb, kBlock, 0, s>>>(F, C, tab, b, u, bc, done);
    return check_launch("k_resid_restrict");
  }
}

template <typename R>
int launch_prolong(ell_grid *g, int l, const R *uc, R *u, bool red_only, const int *done, hipStream_t s) {
  const Geo &F = g->lev[l].geo, &C = g->lev[l + 1].geo;
  const int nb = seg_blocks(red_only ? (long long)F.ncol0 : 2LL * F.H);
  ProfScope ps(g, ELL_K_PROLONG0, s, l == 0);
  const int ns = transfer_segments(red_only ? (long long)F.ncol0 : 2LL * F.H, F.nz);
  if (red_only && g->d.prolong == 0 && g->smooth_tile && F.has_x && F.ny % 2 == 0) {
    // bilinear onto colour 0 with the coarse rows staged in LDS
    const int nbt = blocks8((long long)((F.hx2 + kSTX - 1) / kSTX) * (F.ny / 2) * kBlock);
    if (ns == 16) k_prolong_tile<R, 16><<<nbt, 16 * 64, 0, s>>>(F, C, uc, u, done);
    else if (ns == 8) k_prolong_tile<R, 8><<<nbt, 8 * 64, 0, s>>>(F, C, uc, u, done);
    else k_prolong_tile<R, 4><<<nbt, 4 * 64, 0, s>>>(F, C, uc, u, done);
    return check_launch("k_prolong_tile");
  }
  auto go = [&](auto nseg) {
    constexpr int NS = decltype(nseg)::value;
    if (g->d.prolong == 1) {
      if (red_only) k_prolong<R, true, 1, NS><<<nb, NS * 64, 0, s>>>(F, C, uc, u, done);
      else k_prolong<R, false, 1, NS><<<nb, NS * 64, 0, s>>>(F, C, uc, u, done);
    } else {
      if (red_only) k_prolong<R, true, 0, NS><<<nb, NS * 64, 0, s>>>(F, C, uc, u, done);
      else k_prolong<R, false, 0, NS><<<nb, NS * 64, 0, s>>>(F, C, uc, u, done);
    }
  };
  if (ns == 16) go(std::integral_constant<int, 16>());
  else if (ns == 8) go(std::integral_constant<int, 8>());
  else go(std::integral_constant<int, 4>());
  return check_launch("k_prolong");
}

template <typename R>
int launch_fill(R *p, long long n, hipStream_t s) {
  k_fill<R><<<flat_blocks(n / 2 + 1), kBlock, 0, s>>>(p, n, R(0));
  return check_launch("k_fill");
}

// One V-cycle from u = 0 (Alg. "Multigrid V-cycle"), levels numbered from the
// finest (0).  Pre-smoothing sweeps red then black, post-smoothing black then
// red.  With rho = 1 two exact shortcuts apply: after a black sweep the black
// residual is zero (only red children are restricted) and a black sweep
// ignores the old black values (the correction is added to red columns only).
bool pro_path(const ell_grid *g, int dot);

// The coarsest level's nu_coarse sweep pairs in one cooperative launch
// (k_coarse_sweeps) where its kernels are the 8- or 16-segment ones: rho = 1,
// both horizontal directions, FP64 with the tiled sweep after the first, FP32
// with the segmented one (segments of at most 16 levels).  Returns false if it
// does not apply or the launch was refused (the caller then launches the
// sweeps one by one, and the grid stops trying).
// The coarsest level's sweep pairs one launch each (k_coarse_pair): rho = 1,
// constant coefficients, both horizontal directions, nx and ny multiples of 8,
// the level's own segment count (8 or 16) so the columns are split as the
// half-sweep kernels split them.
bool coarse_pair_ok(const ell_grid *g, int l) {
  const Geo &G = g->lev[l].geo;
  const int Ls = seg_len(G.nz, G.nseg);
  return g->coarse_pair && l == g->L - 1 && !g->varying && g->d.rho == 1.0 && G.has_x && G.has_y &&
         G.nx % 8 == 0 && G.ny % 8 == 0 && ((G.nseg == 16 && Ls <= 16) || (G.nseg == 8 && Ls <= 32));
}

template <typename R>
int launch_coarse_pair(ell_grid *g, int l, const R *b, R *u, bool zero, const int *done, hipStream_t s) {
  const Geo &G = g->lev[l].geo;
  const R *tab = (const R *)g->lev[l].tab;
  const int Ls = seg_len(G.nz, G.nseg);
  const int nb = ((G.nx / 8) * (G.ny / 8) + 7) / 8 * 8;  // a multiple of 8 (logical_block)
  auto go = [&](auto seg, auto nseg) {
    constexpr int SEG = decltype(seg)::value, NSEG = decltype(nseg)::value;
    if (zero) k_coarse_pair<R, true, SEG, NSEG><<<nb, NSEG * 64, 0, s>>>(G, tab, b, u, done);
    else k_coarse_pair<R, false, SEG, NSEG><<<nb, NSEG * 64, 0, s>>>(G, tab, b, u, done);
  };
  using I8 = std::integral_constant<int, 8>;
  using I16 = std::integral_constant<int, 16>;
  using I32 = std::integral_constant<int, 32>;
  if (G.nseg == 16) {
    if (Ls <= 8) go(I8{}, I16{});
    else go(I16{}, I16{});
  } else {
    if (Ls <= 8) go(I8{}, I8{});
    else if (Ls <= 16) go(I16{}, I8{});
    else go(I32{}, I8{});
  }
  return check_launch("k_coarse_pair");
}

template <typename R>
bool coarse_tail_applies(const ell_grid *g, int l) {
  const Geo &G = g->lev[l].geo;
  if (!g->coarse_tail || g->varying || l != g->L - 1 || g->d.nu_coarse < 1 || g->d.rho != 1.0) return false;
  if (!(G.has_x && G.has_y) || (G.nseg != 16 && G.nseg != 8)) return false;
  if (seg_len(G.nz, G.nseg) > 16) return false;
  if constexpr (std::is_same<R, double>::value) return tile_ok(g, l);
  else return true;
}

// The instantiation of k_coarse_sweeps a level takes: its segments, the
// segmented sweep's depth (the smallest of 8 and 16 that holds a segment, as
// seg_dispatch picks) and the tiled sweep's (8 with 16 segments, else 16, as
// launch_smooth picks).
template <typename R>
const void *coarse_kernel(const Geo &G) {
  const int Ls = seg_len(G.nz, G.nseg);
  if (G.nseg == 16)
    return Ls <= 8 ? reinterpret_cast<const void *>(&k_coarse_sweeps<R, 16, 8, 8>)
                   : reinterpret_cast<const void *>(&k_coarse_sweeps<R, 16, 16, 8>);
  return Ls <= 8 ? reinterpret_cast<const void *>(&k_coarse_sweeps<R, 8, 8, 16>)
                 : reinterpret_cast<const void *>(&k_coarse_sweeps<R, 8, 16, 16>);
}

template <typename R>
bool launch_coarse_tail(ell_grid *g, int l, const R *b, R *u, const int *done, hipStream_t s) {
  if (!coarse_tail_applies<R>(g, l)) return false;
  const Geo &G = g->lev[l].geo;
  const int nb0 = (G.ncol0 + kSegCols - 1) / kSegCols;
  const int ntiles = std::is_same<R, double>::value ? smooth_tiles(G) : 0;
  const int nb = std::max(8, (std::max(nb0, ntiles) + 7) / 8 * 8);
  const int threads = G.nseg * 64;
  const void *kern = coarse_kernel<R>(G);
  // every block must be resident at once: at most what the chip holds
  int dev = 0, cus = 0, per_cu = 0;
  if (hipGetDevice(&dev) != hipSuccess ||
      hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev) != hipSuccess ||
      hipOccupancyMaxActiveBlocksPerMultiprocessor(&per_cu, kern, threads, 0) != hipSuccess ||
      nb > cus * per_cu) {
    (void)hipGetLastError();
    g->coarse_tail = 0;
    return false;
  }
  Geo Gv = G;
  const R *tab = (const R *)g->lev[l].tab;
  int sweeps = g->d.nu_coarse;
  unsigned *bar = g->st->bar;
  void *args[] = {&Gv, &tab, &b, &u, &sweeps, &done, &bar};
  if (hipLaunchCooperativeKernel(kern, dim3(nb), dim3(threads), args, 0, s) != hipSuccess) {
    (void)hipGetLastError();
    g->coarse_tail = 0;
    return false;
  }
  return true;
}

// dot > 0 (top = 0, FP64, the finest level tiled): the last two post-smoothing
// half-sweeps also form the CG dots (launch_smooth_dot).
template <typename R>
int vcycle_from(ell_grid *g, int top, const R *btop, R *utop, const int *done, hipStream_t s, int dot = 0,
                bool upd = false) {
  const int L = g->L;
  const bool rho1 = g->d.rho == 1.0;
  auto B = [&](int l) -> const R * { return l == top ? btop : (const R *)g->lev[l].b; };
  auto U = [&](int l) -> R * { return l == top ? utop : (R *)g->lev[l].u; };
  for (int l = top; l < L - 1; ++l) {
    if (g->d.nu_pre == 0) CHK(launch_fill<R>(U(l), 2 * g->lev[l].geo.cs, s));
    for (int it = 0; it < g->d.nu_pre; ++it) {
      if constexpr (std::is_same<R, double>::value) {
        if (upd && l == 0 && it == 0) {  // b is the CG residual g->r
          CHK(pre_pair_upd<double>(g, g->r, U(l), (const double *)g->lev[0].tab, s));
          continue;
        }
      }
      CHK(launch_smooth<R>(g, l, 0, it == 0, B(l), U(l), done, s));
      CHK(launch_smooth<R>(g, l, 1, false, B(l), U(l), done, s));
    }
    CHK(launch_restrict<R>(g, l, B(l), U(l), (R *)g->lev[l + 1].b, rho1 && g->d.nu_pre > 0, done, s));
  }
  {
    const int l = L - 1;
    if (g->d.nu_coarse > 0 && launch_coarse_tail<R>(g, l, B(l), U(l), done, s)) {
      // all coarsest-level sweeps in one launch
    } else if (g->d.nu_coarse > 0 && coarse_pair_ok(g, l)) {
      for (int it = 0; it < g->d.nu_coarse; ++it) CHK(launch_coarse_pair<R>(g, l, B(l), U(l), it == 0, done, s));
    } else if (g->d.nu_coarse > 0) {
      for (int it = 0; it < g->d.nu_coarse; ++it) {
        CHK(launch_smooth<R>(g, l, 0, it == 0, B(l), U(l), done, s));
        CHK(launch_smooth<R>(g, l, 1, false, B(l), U(l), done, s));
      }
    } else {
      // no coarse sweeps: smoothed like a finer level without a coarser
      // correction (red-black, then black-red); one level with one sweep each
      // is the block red/black SSOR line-relaxation preconditioner of the
      // one-level CG solver (Sec. 6.1, Sec. 7.2 Table 2)
      if (g->d.nu_pre == 0) CHK(launch_fill<R>(U(l), 2 * g->lev[l].geo.cs, s));
      for (int it = 0; it < g->d.nu_pre; ++it) {
        CHK(launch_smooth<R>(g, l, 0, it == 0, B(l), U(l), done, s));
        CHK(launch_smooth<R>(g, l, 1, false, B(l), U(l), done, s));
      }
      for (int it = 0; it < g->d.nu_post; ++it) {
        CHK(launch_smooth<R>(g, l, 1, false, B(l), U(l), done, s));
        CHK(launch_smooth<R>(g, l, 0, false, B(l), U(l), done, s));
      }
    }
  }
  for (int l = L - 2; l >= top; --l) {
    if constexpr (std::is_same<R, double>::value) {
      if (l == 0 && pro_path(g, dot)) {  // prolongation inside the post-smoothing pair
        CHK(pro_pair(g, B(0), U(0), done, s, dot));
        continue;
      }
    }
    if (coarse_pro_ok<R>(g, l)) {  // prolongation inside the first post-smoothing sweep
      CHK(coarse_pro_sweep<R>(g, l, B(l), U(l), done, s));
      CHK(launch_smooth<R>(g, l, 0, false, B(l), U(l), done, s));
      for (int it = 1; it < g->d.nu_post; ++it) {
        CHK(launch_smooth<R>(g, l, 1, false, B(l), U(l), done, s));
        CHK(launch_smooth<R>(g, l, 0, false, B(l), U(l), done, s));
      }
      continue;
    }
    CHK(launch_prolong<R>(g, l, (const R *)g->lev[l + 1].u, U(l), rho1 && g->d.nu_post > 0, done, s));
    for (int it = 0; it < g->d.nu_post; ++it) {
      if constexpr (std::is_same<R, double>::value) {
        if (dot && l == 0 && it == g->d.nu_post - 1) {
          const int nt = dot_colour_slots(g, 1);
          CHK(launch_smooth_dot(g, 1, B(l), U(l), (const double *)g->lev[0].tab, dot, 0, done, s));
          CHK(launch_smooth_dot(g, 0, B(l), U(l), (const double *)g->lev[0].tab, dot, nt, done, s));
          continue;
        }
      }
      CHK(launch_smooth<R>(g, l, 1, false, B(l), U(l), done, s));
      CHK(launch_smooth<R>(g, l, 0, false, B(l), U(l), done, s));
    }
  }
  return ELL_OK;
}

// One V-cycle from u = 0 (Alg. "Multigrid V-cycle"), levels numbered from the
// finest (0).  Pre-smoothing sweeps red then black, post-smoothing black then
// red.  With rho = 1 two exact shortcuts apply: after a black sweep the black
// residual is zero (only red children are restricted) and a black sweep
// ignores the old black values (the correction is added to red columns only).
template <typename R>
int vcycle_impl(ell_grid *g, const R *b0, R *u0, const int *done, hipStream_t s, int dot = 0, bool upd = false) {
  return vcycle_from<R>(g, 0, b0, u0, done, s, dot, upd);
}

// The mixed-precision V-cycle: FP32 everywhere except the finest level's
// post-smoothing, which runs in FP64 and writes the FP64 output z.  On the
// graded grids the bottom cells are coupled vertically ~1e10 times more
// strongly than the solution's magnitude resolves in FP32, so an FP32 output
// would carry rounding noise in exactly the stiff vertical modes (inflating
// <p, A p> and the iteration count); the final FP64 column solves remove it,
// while the coarse correction enters only through the weak horizontal
// couplings.  The finest level's FP32 pre-smoothing and restriction read the
// FP64 residual directly.
bool hybrid_ok(const ell_grid *g) {
  const Geo &G = g->lev[0].geo;
  return g->L >= 2 && g->d.rho == 1.0 && g->d.nu_pre >= 1 && g->d.nu_post >= 1 && G.has_x && G.has_y &&
         ((G.nseg == 4 && seg_len(G.nz, 4) <= 64) || (G.nseg == 8 && seg_len(G.nz, 8) <= 16));
}

// The mixed-precision V-cycle's finest prolongation rides on the first FP64
// post-smoothing sweep (colour 1): bilinear prolongation, the LDS-tiled FP64
// sweep, eight k-segments of at most 16 levels or four of at most 32.  The
// colour-0 sweep after it overwrites colour 0 of z without reading it.
bool pro32_path(const ell_grid *g) {
  const Geo &F = g->lev[0].geo;
  const int Ls = seg_len(F.nz, F.nseg);
  return g->prec != ELL_FP64 && g->fused_prolong && g->d.prolong == 0 && hybrid_ok(g) && tile_ok(g, 0) &&
         ((F.nseg == 8 && Ls <= 16) || (F.nseg == 4 && Ls <= 32));
}

// The staged FP32 coarse values load in aligned pairs: coarse half-width,
// colour and plane strides even, the array 8-byte aligned.
bool pro32_pairs_ok(const Geo &C, const void *uc) { return pro_pairs_ok(C, uc, 8); }

template <int SEG, int NSEG, int DOT>
void launch_pro32(int nbt, hipStream_t s, const Geo &F, const Geo &C, const double *tab, const double *b1,
                  const float *u0, double *z1, const float *uc, const int *done, double *partial, int pbase,
                  const double *q1) {
  if (pro32_pairs_ok(C, uc))
    k_smooth_tile_pro32<SEG, NSEG, DOT, true><<<nbt, NSEG * 64, 0, s>>>(F, C, tab, b1, u0, z1, uc, done, partial,
                                                                        pbase, q1);
  else
    k_smooth_tile_pro32<SEG, NSEG, DOT, false><<<nbt, NSEG * 64, 0, s>>>(F, C, tab, b1, u0, z1, uc, done, partial,
                                                                         pbase, q1);
}

template <int SEG, int NSEG>
void pro32_k(int dot, int nbt, hipStream_t s, const Geo &F, const Geo &C, const double *tab, const double *b1,
             const float *u0, double *z1, const float *uc, const int *done, double *partial, const double *q1) {
  if (dot == 2) launch_pro32<SEG, NSEG, 2>(nbt, s, F, C, tab, b1, u0, z1, uc, done, partial, 0, q1);
  else if (dot == 1) launch_pro32<SEG, NSEG, 1>(nbt, s, F, C, tab, b1, u0, z1, uc, done, partial, 0, q1);
  else launch_pro32<SEG, NSEG, 0>(nbt, s, F, C, tab, b1, u0, z1, uc, done, partial, 0, q1);
}

// The fused sweep of colour 1 (pro32_path checked): z1 from r1, the FP32
// colour-0 values u32 and the coarse correction; with dot, the colour's
// partial sums go to the first tile-count slots as launch_smooth_dot's.
int pro32_sweep(ell_grid *g, const double *r, const float *u32, double *z, int dot, const int *done,
                hipStream_t s) {
  const Geo &F = g->lev[0].geo, &C = g->lev[1].geo;
  const int Ls = seg_len(F.nz, F.nseg);
  const int nbt = blocks8((long long)smooth_tiles(F) * kBlock);
  const long long cs = F.cs;
  const float *uc = (const float *)g->lev[1].u;
  ProfScope ps(g, ELL_K_SMOOTH0, s);
  if (F.nseg == 8)
    pro32_k<16, 8>(dot, nbt, s, F, C, g->tab64_0, r + cs, u32, z + cs, uc, done, g->partial, g->q + cs);
  else if (Ls <= 16)
    pro32_k<16, 4>(dot, nbt, s, F, C, g->tab64_0, r + cs, u32, z + cs, uc, done, g->partial, g->q + cs);
  else
    pro32_k<32, 4>(dot, nbt, s, F, C, g->tab64_0, r + cs, u32, z + cs, uc, done, g->partial, g->q + cs);
  return check_launch("k_smooth_tile_pro32");
}

int vcycle_hybrid(ell_grid *g, const double *r, double *z, const int *done, hipStream_t s, int dot = 0,
                  bool upd = false) {
  float *u32 = (float *)g->z32;
  for (int it = 0; it < g->d.nu_pre; ++it) {
    if (upd && it == 0) {  // r is the CG residual g->r
      CHK(pre_pair_upd<float>(g, g->r, u32, (const float *)g->lev[0].tab, s));
      continue;
    }
    CHK((launch_smooth<float, double>(g, 0, 0, it == 0, r, u32, done, s)));
    CHK((launch_smooth<float, double>(g, 0, 1, false, r, u32, done, s)));
  }
  CHK((launch_restrict<float, double>(g, 0, r, u32, (float *)g->lev[1].b, true, done, s)));
  CHK(vcycle_from<float>(g, 1, (const float *)g->lev[1].b, (float *)g->lev[1].u, done, s));
  const bool pro = pro32_path(g);
  if (!pro) {
    const Geo &F = g->lev[0].geo, &C = g->lev[1].geo;
    const int nb = seg_blocks(F.ncol0);
    ProfScope ps(g, ELL_K_PROLONG0, s);
    if (g->d.prolong == 0 && g->smooth_tile && F.has_x && F.ny % 2 == 0) {
      // bilinear with the coarse rows staged in LDS (as launch_prolong)
      const int ns = transfer_segments(F.ncol0, F.nz);
      const int nbt = blocks8((long long)((F.hx2 + kSTX - 1) / kSTX) * (F.ny / 2) * kBlock);
      const float *uc = (const float *)g->lev[1].u;
      if (ns == 16) k_prolong_out_tile<float, double, 16><<<nbt, 16 * 64, 0, s>>>(F, C, uc, u32, z, done);
      else if (ns == 8) k_prolong_out_tile<float, double, 8><<<nbt, 8 * 64, 0, s>>>(F, C, uc, u32, z, done);
      else k_prolong_out_tile<float, double, 4><<<nbt, 4 * 64, 0, s>>>(F, C, uc, u32, z, done);
      CHK(check_launch("k_prolong_out_tile"));
    } else if (g->d.prolong == 1)
      k_prolong_out<float, double, 1><<<nb, kBlock, 0, s>>>(F, C, (const float *)g->lev[1].u, u32, z, done);
    else
      k_prolong_out<float, double, 0><<<nb, kBlock, 0, s>>>(F, C, (const float *)g->lev[1].u, u32, z, done);
    CHK(check_launch("k_prolong_out"));
  }
  for (int it = 0; it < g->d.nu_post; ++it) {
    const bool fused = pro && it == 0;  // colour 1 applies the coarse correction
    if (dot && it == g->d.nu_post - 1) {
      const int nt = dot_colour_slots(g, 1);
      if (fused) CHK(pro32_sweep(g, r, u32, z, dot, done, s));
      else CHK(launch_smooth_dot(g, 1, r, z, g->tab64_0, dot, 0, done, s));
      CHK(launch_smooth_dot(g, 0, r, z, g->tab64_0, dot, nt, done, s));
      continue;
    }
    if (fused) CHK(pro32_sweep(g, r, u32, z, 0, done, s));
    else CHK(launch_smooth<double>(g, 0, 1, false, r, z, done, s, g->tab64_0));
    CHK(launch_smooth<double>(g, 0, 0, false, r, z, done, s, g->tab64_0));
  }
  return ELL_OK;
}

// The CG residual update is fused into the first pre-smoothing pair of this
// grid's preconditioner application: at least two levels, rho = 1, four
// k-segments of at most 32 levels or eight of at most 16 on the finest level;
// FP64 with the tiled colour-1 sweep, or the mixed-precision V-cycle.
template <typename R>
bool fused_update_path(const ell_grid *g) {
  const Geo &G = g->lev[0].geo;
  const int Ls = seg_len(G.nz, G.nseg);
  const bool segs = g->varying ? seg3_ok(g, 0) : ((G.nseg == 8 && Ls <= 16) || (G.nseg == 4 && Ls <= 32));
  // at least two levels: the finest level's pre-smoothing, and with it the
  // convergence test, then runs once per step
  const bool base =
      g->fused_update && g->L >= 2 && g->d.rho == 1.0 && g->d.nu_pre >= 1 && G.has_x && G.has_y && segs;
  if constexpr (std::is_same<R, double>::value) return base && (tile_ok(g, 0) || g->varying);
  else return base && hybrid_ok(g);
}

// The CG dots are fused into the preconditioner application of this grid:
// the finest level's post-smoothing is FP64 and tiled (the FP64 V-cycle, or
// the mixed-precision one with its FP64 finest post-smoothing).
template <typename R>
bool fused_dot_path(const ell_grid *g) {
  const bool base = g->fused_dot && g->L >= 2 && g->d.nu_post >= 1 && (tile_ok(g, 0) || seg3_ok(g, 0));
  if constexpr (std::is_same<R, double>::value) return base;
  else return base && hybrid_ok(g);
}

// The finest prolongation rides on the first post-smoothing sweep (pro_pair):
// FP64 V-cycle with fused dots (dot = 1: <r, z>, the printed beta; 2: <r, z>
// and <z, q>, the flexible beta), one post-smoothing sweep, bilinear
// prolongation.
bool pro_path(const ell_grid *g, int dot) {
  return (dot == 1 || dot == 2) && g->fused_prolong && g->prec == ELL_FP64 && fused_dot_path<double>(g) &&
         g->d.nu_post == 1 && g->d.prolong == 0;
}

// Partial slots of one colour's fused-dot sweep (colour 1 takes the first
// ones, colour 0 follows).
int dot_colour_slots(const ell_grid *g, int c) {
  return g->varying ? seg3_shape(g->lev[0].geo, c).nbs : smooth_tiles(g->lev[0].geo);
}

// Partial slots of the fused dots.
int dot_slots(const ell_grid *g, int dot) {
  return pro_path(g, dot) ? smooth_tiles(g->lev[0].geo) : dot_colour_slots(g, 1) + dot_colour_slots(g, 0);
}

int launch_apply64(ell_grid *g, const double *x, double *y, bool dot, const int *done, hipStream_t s) {
  const Geo &G = g->lev[0].geo;
  const int nb = seg_blocks(2LL * G.H);
  // the CG operator is always FP64 (FP32 grids keep a separate FP64 table)
  const double *tab64 = g->tab64_0;
  ProfScope ps(g, ELL_K_APPLY, s, dot);
  (void)nb;
  const bool hxy = G.has_x && G.has_y;
  const int ns = g->stencil_seg;
  const int b = stencil_blocks(2LL * G.H, ns);
  if (g->varying) {
    const double *tz3 = g->lev[0].tz3;
    auto go = [&](auto nsc) {
      constexpr int NS = decltype(nsc)::value;
      if (dot) k_apply<double, true, false, NS, true><<<b, kBlock, 0, s>>>(G, tab64, x, y, g->partial, done, tz3);
      else k_apply<double, false, false, NS, true><<<b, kBlock, 0, s>>>(G, tab64, x, y, g->partial, done, tz3);
    };
    if (ns == 1) go(std::integral_constant<int, 1>{});
    else if (ns == 2) go(std::integral_constant<int, 2>{});
    else go(std::integral_constant<int, 4>{});
    return check_launch("k_apply");
  }
  if (ns == 1) {
    if (dot) k_apply<double, true, false, 1><<<b, kBlock, 0, s>>>(G, tab64, x, y, g->partial, done);
    else k_apply<double, false, false, 1><<<b, kBlock, 0, s>>>(G, tab64, x, y, g->partial, done);
  } else if (ns == 2) {
    if (dot) k_apply<double, true, false, 2><<<b, kBlock, 0, s>>>(G, tab64, x, y, g->partial, done);
    else k_apply<double, false, false, 2><<<b, kBlock, 0, s>>>(G, tab64, x, y, g->partial, done);
  } else {
    if (dot && hxy) k_apply<double, true, true, 4><<<b, kBlock, 0, s>>>(G, tab64, x, y, g->partial, done);
    else if (dot) k_apply<double, true, false, 4><<<b, kBlock, 0, s>>>(G, tab64, x, y, g->partial, done);
    else if (hxy) k_apply<double, false, true, 4><<<b, kBlock, 0, s>>>(G, tab64, x, y, g->partial, done);
    else k_apply<double, false, false, 4><<<b, kBlock, 0, s>>>(G, tab64, x, y, g->partial, done);
  }
  return check_launch("k_apply");
}

int finalize(ell_grid *g, int nblk, int nq, int mode, hipStream_t s, double rtol = 0, double atol = 0,
             int rel = 0) {
  k_finalize<<<1, kBlock, 0, s>>>(g->partial, nblk, nq, g->st, mode, rtol, atol, rel);
  return check_launch("k_finalize");
}

// z = M r; dot > 0 needs fused_dot_path<R>(g), upd fused_update_path<R>(g).
template <typename R>
int precondition(ell_grid *g, const int *done, hipStream_t s, int dot = 0, bool upd = false);

template <>
int precondition<double>(ell_grid *g, const int *done, hipStream_t s, int dot, bool upd) {
  return vcycle_impl<double>(g, g->r, g->z, done, s, dot, upd);
}

template <>
int precondition<float>(ell_grid *g, const int *done, hipStream_t s, int dot, bool upd) {
  if (hybrid_ok(g)) return vcycle_hybrid(g, g->r, g->z, done, s, dot, upd);
  const long long n2 = g->n0 / 2;
  k_cast_f64_f32<<<flat_blocks(n2), kBlock, 0, s>>>((const double2 *)g->r, (float2 *)g->b32, n2, done);
  CHK(check_launch("k_cast_f64_f32"));
  return vcycle_impl<float>(g, (const float *)g->b32, (float *)g->z32, done, s);
}

// R: arithmetic of the V-cycle; Z: element type of its output z (FP64 for
// the FP64 and the hybrid mixed-precision V-cycles, FP32 otherwise).
template <typename Z>
const typename Vec2<Z>::T *zvec(const ell_grid *g) {
  return (const typename Vec2<Z>::T *)(std::is_same<Z, double>::value ? (void *)g->z : g->z32);
}

// Start of a solve (Appendix B, Alg. PCG, before the loop): r = V f - A u0
// with ||b|| and ||r0|| (the device sets done if nothing is left to do),
// z0 = M^{-1} r0, kappa = <r0, z0>.
// Blocks of the CG operator step of a grid (single-grid launch).
int apply_dir_blocks(const ell_grid *g) {
  const Geo &G = g->lev[0].geo;
  return g->apply_tile ? blocks8(tile_blocks(G, g->apply_nseg) * kBlock) : stencil_blocks(2LL * G.H, g->stencil_seg);
}

// Caller-facing statistics of a finished solve; the return code follows the
// final status (0 converged, 1 iteration limit, -4 non-finite recurrence).
int stats_from_state(const PcgState &h, ell_solve_stats *out) {
  const int status = h.status;
  if (out) {
    out->iters = h.iter;
    out->status = status == -4 ? ELL_ERR_NUMERIC : (status == 0 ? ELL_OK : ELL_NOT_CONVERGED);
    out->r0_norm = h.r0_norm;
    out->r_norm = h.r_norm;
    out->true_r_norm = h.true_r_norm;
    out->b_norm = h.b_norm;
  }
  if (h.bar[2]) return fail(ELL_ERR_HIP, "a grid-wide barrier of the coarsest-level sweeps timed out");
  if (status == -4) return fail(ELL_ERR_NUMERIC, "non-finite value in the CG recurrence");
  return status == 0 ? ELL_OK : ELL_NOT_CONVERGED;
}

// The k-segments and blocks of the tiled start / end of a solve (the operator
// step's tiles and segments; at most 4 segments, so the partial-sum buffer
// holds their two sums per block).
int ends_nseg(const ell_grid *g) { return g->apply_tile ? g->apply_nseg : apply_segments(g->lev[0].geo.nz); }
int ends_blocks(const ell_grid *g) { return blocks8(tile_blocks(g->lev[0].geo, ends_nseg(g)) * kBlock); }

// us = u0 and r = V f - A u0 with the F_INIT partial sums; *nblk: the blocks
// whose two sums the reduction takes.
int launch_begin(ell_grid *g, const double *f, const double *u, int *nblk, hipStream_t s) {
  const Geo &G = g->lev[0].geo;
  if (g->tiled_ends) {
    *nblk = ends_blocks(g);
    k_begin_tile<<<*nblk, kBlock, 0, s>>>(G, ends_nseg(g), g->tab64_0, g->vol0, f, u, g->us, g->r, g->partial);
    return check_launch("k_begin_tile");
  }
  *nblk = seg_blocks((long long)G.nx * G.ny);
  if (g->varying)
    k_begin<true><<<*nblk, kBlock, 0, s>>>(G, g->tab64_0, g->vol0, f, u, g->us, g->r, g->partial, g->lev[0].tz3);
  else
    k_begin<><<<*nblk, kBlock, 0, s>>>(G, g->tab64_0, g->vol0, f, u, g->us, g->r, g->partial);
  return check_launch("k_begin");
}

template <typename R, typename Z>
int pcg_begin(ell_grid *g, const double *f, const double *u, const ell_solve_opts &o, hipStream_t s) {
  const long long n2 = g->n0 / 2;
  const int fb = flat_blocks(n2);
  const int *done = &g->st->done;
  // maxiter / flexible live in the state block (read by F_INIT and F_CONV)
  {
    PcgState *h = g->st_host;
    h->maxiter = o.maxiter;
    h->flexible = o.flexible;
    HIPCHK(hipMemcpyAsync(&g->st->maxiter, &h->maxiter, 2 * sizeof(int), hipMemcpyHostToDevice, s));
  }
  int bb = 0;
  CHK(launch_begin(g, f, u, &bb, s));
  k_finalize<<<1, kBlock, 0, s>>>(g->partial, bb, 2, g->st, F_INIT, o.rtol, o.atol, o.rel_to_rhs);
  CHK(check_launch("k_finalize"));
  if (fused_dot_path<R>(g)) {  // kappa_0 = <r0, z0> from the last half-sweeps
    CHK(precondition<R>(g, done, s, 1));
    return finalize(g, dot_slots(g, 1), 1, F_KAPPA, s);
  }
  CHK(precondition<R>(g, done, s));
  k_dots<Z><<<fb, kBlock, 0, s>>>((const double2 *)g->r, zvec<Z>(g), (const double2 *)g->q, n2, g->st,
                                  g->partial);
  CHK(check_launch("k_dots"));
  return finalize(g, fb, 2, F_KAPPA, s);
}

// The search direction of iteration K (deferred_updates in the kernels'
// header gives the schedule that frees the buffers).
inline double *dir_buf(ell_grid *g, int K) {
  const int i = dir_slot(K);
  return i == 0 ? g->p : (i == 1 ? g->p2 : g->p3);
}

// Iteration K (1-based) of the loop; a no-op on the device once done is set.
// The fused operator step of iteration K: p_K = z + beta p_{K-1} (z alone with
// first set), q = A p_K with <p, q>, and with defer = 2 the solution updates
// of iterations K - 2 and K - 1 (deferred_updates).
template <typename Z>
int launch_apply_dir(ell_grid *g, int K, int first, int defer, hipStream_t s) {
  const Geo &G = g->lev[0].geo;
  const int ab = apply_dir_blocks(g);
  double *pold = dir_buf(g, K - 1), *pold2 = dir_buf(g, K - 2), *pnew = dir_buf(g, K);
  ProfScope ps(g, ELL_K_APPLY, s);
  const Z *zz = (const Z *)zvec<Z>(g);
  if (g->varying && g->apply_tile) {
    k_apply_dir_tile<Z, true><<<ab, kBlock, 0, s>>>(G, g->apply_nseg, g->tab64_0, zz, pold, pold2, pnew, g->q, g->us,
                                                    g->st, first, defer, g->partial, g->lev[0].tz3);
  } else if (g->varying) {
    const double *tz3 = g->lev[0].tz3;
    if (g->stencil_seg == 1)
      k_apply_dir<Z, 1, true><<<ab, kBlock, 0, s>>>(G, g->tab64_0, zz, pold, pold2, pnew, g->q, g->us, g->st, first,
                                                    defer, g->partial, tz3);
    else if (g->stencil_seg == 2)
      k_apply_dir<Z, 2, true><<<ab, kBlock, 0, s>>>(G, g->tab64_0, zz, pold, pold2, pnew, g->q, g->us, g->st, first,
                                                    defer, g->partial, tz3);
    else
      k_apply_dir<Z, 4, true><<<ab, kBlock, 0, s>>>(G, g->tab64_0, zz, pold, pold2, pnew, g->q, g->us, g->st, first,
                                                    defer, g->partial, tz3);
  } else if (g->apply_tile)
    k_apply_dir_tile<Z><<<ab, kBlock, 0, s>>>(G, g->apply_nseg, g->tab64_0, zz, pold, pold2, pnew, g->q, g->us,
                                              g->st, first, defer, g->partial);
  else if (g->stencil_seg == 1)
    k_apply_dir<Z, 1><<<ab, kBlock, 0, s>>>(G, g->tab64_0, zz, pold, pold2, pnew, g->q, g->us, g->st, first, defer,
                                            g->partial);
  else if (g->stencil_seg == 2)
    k_apply_dir<Z, 2><<<ab, kBlock, 0, s>>>(G, g->tab64_0, zz, pold, pold2, pnew, g->q, g->us, g->st, first, defer,
                                            g->partial);
  else
    k_apply_dir<Z, 4><<<ab, kBlock, 0, s>>>(G, g->tab64_0, zz, pold, pold2, pnew, g->q, g->us, g->st, first, defer,
                                            g->partial);
  return check_launch("k_apply_dir");
}

template <typename R, typename Z>
int pcg_step(ell_grid *g, int K, hipStream_t s) {
  const long long n2 = g->n0 / 2;
  const int fb = flat_blocks(n2);
  const int ab = apply_dir_blocks(g);  // blocks of the CG operator kernel
  const int *done = &g->st->done;
  CHK(launch_apply_dir<Z>(g, K, K == 1 ? 1 : 0, deferred_updates(K), s));

  CHK(finalize(g, ab, 1, F_ALPHA, s));
  // r -= alpha q and the convergence test: fused into the first pre-smoothing
  // pair of the V-cycle, or a pass of their own before it
  const bool upd = fused_update_path<R>(g);
  if (!upd) {
    {
      ProfScope ps(g, ELL_K_UPDATE, s);
      k_update_r<<<fb, kBlock, 0, s>>>((double2 *)g->r, (const double2 *)g->q, n2, g->st, g->partial);
    }
    CHK(check_launch("k_update_r"));
    CHK(finalize(g, fb, 1, F_CONV, s));
  }
  if (fused_dot_path<R>(g)) {  // <r, z> (and <z, q>) from the last half-sweeps
    const int nq = g->st_host->flexible ? 2 : 1;
    CHK(precondition<R>(g, done, s, nq, upd));
    return finalize(g, dot_slots(g, nq), nq, F_BETA, s);
  }
  CHK(precondition<R>(g, done, s, 0, upd));
  k_dots<Z><<<fb, kBlock, 0, s>>>((const double2 *)g->r, zvec<Z>(g), (const double2 *)g->q, n2, g->st,
                                  g->partial);
  CHK(check_launch("k_dots"));
  return finalize(g, fb, 2, F_BETA, s);
}

// Stand-alone multigrid (Sec. 4.3, the V-cycle iterated as a solver):
// u_K = u_{K-1} + z_K with z_K = M r_{K-1}, r_K = r_{K-1} - A z_K.  It runs on
// the CG kernels with alpha = 1 and beta = 0 (F_UNIT): the operator step forms
// p = z, q = A z and applies the deferred updates u += p of earlier iterates
// (two at a time, as in CG), the residual update takes r -= q; no dots, no
// scalar recurrences.
template <typename R, typename Z>
int mg_begin(ell_grid *g, const double *f, const double *u, const ell_solve_opts &o, hipStream_t s) {
  {
    PcgState *h = g->st_host;
    h->maxiter = o.maxiter;
    h->flexible = 0;
    HIPCHK(hipMemcpyAsync(&g->st->maxiter, &h->maxiter, 2 * sizeof(int), hipMemcpyHostToDevice, s));
  }
  int bb = 0;
  CHK(launch_begin(g, f, u, &bb, s));
  k_finalize<<<1, kBlock, 0, s>>>(g->partial, bb, 2, g->st, F_INIT, o.rtol, o.atol, o.rel_to_rhs);
  CHK(check_launch("k_finalize"));
  k_finalize<<<1, kBlock, 0, s>>>(g->partial, 0, 0, g->st, F_UNIT, 0, 0, 0);
  return check_launch("k_finalize");
}

template <typename R, typename Z>
int mg_step(ell_grid *g, int K, hipStream_t s) {
  const long long n2 = g->n0 / 2;
  const int fb = flat_blocks(n2);
  CHK(precondition<R>(g, &g->st->done, s));
  // K = 1: p = z; later p = z + 0 p_old, with u += 1 p for the deferred updates
  CHK(launch_apply_dir<Z>(g, K, K == 1 ? 1 : 0, deferred_updates(K), s));
  {
    ProfScope ps(g, ELL_K_UPDATE, s);
    k_update_r<<<fb, kBlock, 0, s>>>((double2 *)g->r, (const double2 *)g->q, n2, g->st, g->partial);
  }
  CHK(check_launch("k_update_r"));
  return finalize(g, fb, 1, F_CONV, s);
}

// End of a solve; g->st_host must hold the final state: the last step's
// deferred solution update, u back to plane-major, the FP64 true residual.
int pcg_finish(ell_grid *g, const double *f, double *u, ell_solve_stats *out, hipStream_t s) {
  const Geo &G = g->lev[0].geo;
  const int K = g->st_host->iter;
  const int with_p = g->st_host->status != -4 ? pending_at_end(K) : 0;
  int fb = 0;
  if (g->tiled_ends) {
    fb = ends_blocks(g);
    auto go = [&](auto wp) {
      k_finish_tile<decltype(wp)::value><<<fb, kBlock, 0, s>>>(G, ends_nseg(g), g->tab64_0, g->vol0, f, g->us,
                                                               dir_buf(g, K), dir_buf(g, K - 1), g->st, u,
                                                               g->partial);
    };
    if (with_p == 2) go(std::integral_constant<int, 2>{});
    else if (with_p == 1) go(std::integral_constant<int, 1>{});
    else go(std::integral_constant<int, 0>{});
    CHK(check_launch("k_finish_tile"));
  } else {
    fb = seg_blocks(2LL * G.H);
    if (g->varying)
      k_finish<true><<<fb, kBlock, 0, s>>>(G, g->tab64_0, g->vol0, f, g->us, dir_buf(g, K), dir_buf(g, K - 1),
                                           g->st, with_p, u, g->partial, g->lev[0].tz3);
    else
      k_finish<><<<fb, kBlock, 0, s>>>(G, g->tab64_0, g->vol0, f, g->us, dir_buf(g, K), dir_buf(g, K - 1), g->st,
                                       with_p, u, g->partial);
    CHK(check_launch("k_finish"));
  }
  k_finalize<<<1, kBlock, 0, s>>>(g->partial, fb, 2, g->st, F_TRUE, 0, 0, 0);
  CHK(check_launch("k_finalize"));
  HIPCHK(hipMemcpyAsync(g->st_host, g->st, sizeof(PcgState), hipMemcpyDeviceToHost, s));
  HIPCHK(hipStreamSynchronize(s));
  return stats_from_state(*g->st_host, out);
}

template <typename R, typename Z>
int pcg_impl(ell_grid *g, const double *f, double *u, const ell_solve_opts &o, ell_solve_stats *out,
             hipStream_t s) {
  CHK((pcg_begin<R, Z>(g, f, u, o, s)));
  const int poll = o.poll_every > 0 ? o.poll_every : 4;
  int enq = 0;
  HIPCHK(hipMemcpyAsync(g->st_host, g->st, sizeof(PcgState), hipMemcpyDeviceToHost, s));
  HIPCHK(hipStreamSynchronize(s));
  while (enq < o.maxiter && !g->st_host->done) {
    const int batch = std::min(poll, o.maxiter - enq);
    for (int it = 0; it < batch; ++it) CHK((pcg_step<R, Z>(g, enq + it + 1, s)));
    enq += batch;
    HIPCHK(hipMemcpyAsync(g->st_host, g->st, sizeof(PcgState), hipMemcpyDeviceToHost, s));
    HIPCHK(hipStreamSynchronize(s));
  }
  return pcg_finish(g, f, u, out, s);
}

template <typename R, typename Z>
int mg_impl(ell_grid *g, const double *f, double *u, const ell_solve_opts &o, ell_solve_stats *out,
            hipStream_t s) {
  CHK((mg_begin<R, Z>(g, f, u, o, s)));
  const int poll = o.poll_every > 0 ? o.poll_every : 4;
  int enq = 0;
  HIPCHK(hipMemcpyAsync(g->st_host, g->st, sizeof(PcgState), hipMemcpyDeviceToHost, s));
  HIPCHK(hipStreamSynchronize(s));
  while (enq < o.maxiter && !g->st_host->done) {
    const int batch = std::min(poll, o.maxiter - enq);
    for (int it = 0; it < batch; ++it) CHK((mg_step<R, Z>(g, enq + it + 1, s)));
    enq += batch;
    HIPCHK(hipMemcpyAsync(g->st_host, g->st, sizeof(PcgState), hipMemcpyDeviceToHost, s));
    HIPCHK(hipStreamSynchronize(s));
  }
  return pcg_finish(g, f, u, out, s);
}

int check_level(const ell_grid *g, int level, bool need_coarser) {
  if (!g) return fail(ELL_ERR_INVALID, "grid is NULL");
  if (level < 0 || level >= g->L) return fail(ELL_ERR_INVALID, "level %d out of range", level);
  if (need_coarser && level + 1 >= g->L) return fail(ELL_ERR_INVALID, "level %d has no coarser level", level);
  return ELL_OK;
}

// ------------------------------------------------------------------------
// schedules: per shape, the operator-step kernel and segments and the
// smoother segments per coarse level (recorded by ell_autotune or
// ell_schedule_set, else heuristic)
// ------------------------------------------------------------------------
using SchedKey = std::array<int, 5>;
std::mutex g_sched_mu;
std::map<SchedKey, ell_schedule> g_sched;

SchedKey sched_key(const ell_grid_desc *d, int L) {
  return SchedKey{d->nx, d->ny, d->nz, L, d->precision == ELL_FP64 ? 0 : 1};
}

// A coarse level can run the segmented smoother with ns segments when a
// kernel instance covers the segment length (else it runs the sequential
// column kernel).
bool smooth_nseg_fits(int ns, int nz) {
  const int Ls = seg_len(nz, ns);
  return (ns == 4 && Ls <= 64) || (ns == 8 && Ls <= 32) || (ns == 16 && Ls <= 16);
}

ell_schedule default_schedule(const ell_grid_desc *d, int L) {
  ell_schedule s;
  std::memset(&s, 0, sizeof(s));
  s.apply_tile = (g_apply_tile && d->nx > 1 && d->ny > 1) ? 1 : 0;
  s.apply_nseg = s.apply_tile ? apply_segments(d->nz) : g_stencil_seg;
  for (int l = 0; l < L && l < ELL_MAX_LEVELS; ++l)
    s.smooth_nseg[l] = make_geo(d->nx >> l, d->ny >> l, d->nz, l == 0).nseg;
  return s;
}

int check_schedule(const ell_grid_desc *d, int L, const ell_schedule *s) {
  if (L > ELL_MAX_LEVELS) return fail(ELL_ERR_INVALID, "schedules cover at most %d levels", ELL_MAX_LEVELS);
  if (s->apply_tile != 0 && s->apply_tile != 1) return fail(ELL_ERR_INVALID, "apply_tile must be 0 or 1");
  if (s->apply_tile && (d->nx < 2 || d->ny < 2))
    return fail(ELL_ERR_INVALID, "the tiled operator step needs nx, ny > 1");
  if (s->apply_nseg != 1 && s->apply_nseg != 2 && s->apply_nseg != 4)
    return fail(ELL_ERR_INVALID, "apply_nseg must be 1, 2 or 4");
  if (s->smooth_nseg[0] != 4 && !(s->smooth_nseg[0] == 8 && seg_len(d->nz, 8) <= 16))
    return fail(ELL_ERR_INVALID, "the finest level's smoother uses 4 segments (or 8 when nz <= 128)");
  for (int l = 1; l < L; ++l) {
    const int ns = s->smooth_nseg[l];
    if (ns != 4 && ns != 8 && ns != 16) return fail(ELL_ERR_INVALID, "smooth_nseg[%d] must be 4, 8 or 16", l);
  }
  return ELL_OK;
}

ell_schedule schedule_for(const ell_grid_desc *d, int L) {
  {
    std::lock_guard<std::mutex> lk(g_sched_mu);
    auto it = g_sched.find(sched_key(d, L));
    if (it != g_sched.end()) return it->second;
  }
  return default_schedule(d, L);
}

}  // namespace

// Device area of ell_apply_A_noalloc: the finest level's stencil coefficients
// (slots TV..TZ, nz+1 values each, nz <= ELL_NOALLOC_MAX_NZ), 32.8 KB.  Every
// GPU the library runs on holds its own copy until the process ends.  Host
// code never uses this name as an address (it is a host-side stand-in): it
// takes the per-device address from noalloc_area().
static __device__ __align__(256) double scratch[4 * (ELL_NOALLOC_MAX_NZ + 1)];

namespace {

constexpr int kMaxDevices = 64;
std::mutex g_noalloc_mu;
double *g_noalloc_ptr[kMaxDevices] = {};

// Address of the current device's scratch, looked up once per device (with
// that device current) and kept.
int noalloc_area(double **out) {
  int dev = -1;
  HIPCHK(hipGetDevice(&dev));
  if (dev < 0 || dev >= kMaxDevices) return fail(ELL_ERR_INVALID, "device %d out of range", dev);
  std::lock_guard<std::mutex> lk(g_noalloc_mu);
  if (!g_noalloc_ptr[dev]) {
    void *p = nullptr;
    HIPCHK(hipGetSymbolAddress(&p, HIP_SYMBOL(scratch)));
    if (!p) return fail(ELL_ERR_HIP, "no device address for the coefficient area");
    g_noalloc_ptr[dev] = (double *)p;
  }
  *out = g_noalloc_ptr[dev];
  return ELL_OK;
}

}  // namespace

// ==========================================================================
// C ABI
// ==========================================================================
extern "C" {

const char *ell_last_error(void) { return g_err.c_str(); }

size_t ell_grid_bytes(const ell_grid_desc *desc) {
  int L = 0;
  if (validate(desc, &L) != ELL_OK) return 0;
  return grid_bytes(desc, L);
}

static int grid_create(const ell_grid_desc *desc, bool batch_layout, ell_grid **out,
                       const ell_schedule *force = nullptr, const double *lam3 = nullptr);

int ell_grid_create(const ell_grid_desc *desc, ell_grid **out) { return grid_create(desc, false, out); }

int ell_grid_create_varying(const ell_grid_desc *desc, const double *lambda2_3d, ell_grid **out) {
  if (!out) return fail(ELL_ERR_INVALID, "out is NULL");
  *out = nullptr;
  if (!desc) return fail(ELL_ERR_INVALID, "descriptor is NULL");
  if (!lambda2_3d) return fail(ELL_ERR_INVALID, "lambda2_3d is NULL");
  if (desc->precision != ELL_FP64 && desc->precision != ELL_FP32_PRECOND)
    return fail(ELL_ERR_INVALID, "horizontally varying coefficients take ELL_FP64 or ELL_FP32_PRECOND");
  if (desc->nx < 1 || desc->ny < 1 || desc->nz < 1) return fail(ELL_ERR_INVALID, "sizes must be >= 1");
  const size_t n = (size_t)desc->nx * desc->ny * desc->nz;
  for (size_t e = 0; e < n; ++e)
    if (!(lambda2_3d[e] > 0) || !std::isfinite(lambda2_3d[e]))
      return fail(ELL_ERR_INVALID, "lambda2_3d[%zu] must be positive and finite", e);
  // desc->lambda2 is not read: the z-only faces of the level tables are unused
  std::vector<double> ones((size_t)desc->nz, 1.0);
  ell_grid_desc d = *desc;
  d.lambda2 = ones.data();
  return grid_create(&d, false, out, nullptr, lambda2_3d);
}

static int grid_create(const ell_grid_desc *desc, bool batch_layout, ell_grid **out,
                       const ell_schedule *force, const double *lam3) {
  if (!out) return fail(ELL_ERR_INVALID, "out is NULL");
  *out = nullptr;
  int L = 0;
  CHK(validate(desc, &L));
  ell_grid *g = new ell_grid();
  g->d = *desc;
  g->dz.assign(desc->dz, desc->dz + desc->nz);
  g->lam.assign(desc->lambda2, desc->lambda2 + desc->nz);
  g->d.dz = g->dz.data();
  g->d.lambda2 = g->lam.data();
  g->L = L;
  g->prec = desc->precision;
  g->esz = g->prec == ELL_FP64 ? 8 : 4;
  const ell_schedule sc = force ? *force : schedule_for(desc, L);
  g->apply_tile = (sc.apply_tile && desc->nx > 1 && desc->ny > 1) ? 1 : 0;
  g->apply_nseg = g->apply_tile ? sc.apply_nseg : apply_segments(desc->nz);
  g->stencil_seg = batch_layout ? 1 : (g->apply_tile ? g_stencil_seg : sc.apply_nseg);
  g->smooth_tile = g_smooth_tile;
  g->fused_dot = g_fused_dot;
  g->fused_update = g_fused_update;
  g->fused_prolong = g_fused_prolong;
  g->tiled_ends = (g_tiled_ends && desc->nx > 1 && desc->ny > 1) ? 1 : 0;
  g->coarse_tail = g_coarse_tail && !batch_layout;
  g->coarse_pair = g_coarse_pair;
  g->batch_layout = batch_layout;
  if (lam3) {  // per-column coefficients: no LDS-tiled sweeps (tile_ok), ends or fused prolongation
    g->varying = true;
    g->fused_prolong = g->tiled_ends = 0;
  }
  g->lev.resize(L);
  auto bail = [&](int rc) {
    ell_grid_destroy(g);
    return rc;
  };
  int rc;
  std::vector<double> t64;
  std::vector<float> t32;
  for (int l = 0; l < L; ++l) {
    Level &Lv = g->lev[l];
    Lv.geo = make_geo(desc->nx >> l, desc->ny >> l, desc->nz, l == 0, batch_layout);
    if (!batch_layout && l < ELL_MAX_LEVELS && sc.smooth_nseg[l] > 0) Lv.geo.nseg = sc.smooth_nseg[l];
    Lv.hx = desc->hx * (double)(1 << l);
    Lv.hy = desc->hy * (double)(1 << l);
    level_table64(g, l, t64);
    if (g->varying) {  // the shared vertical slots mean nothing here: make any use loud
      const int P = desc->nz + 1;
      for (int sl = TZ; sl < TSLOTS; ++sl)
        for (int k = 0; k < P; ++k) t64[(size_t)sl * P + k] = std::nan("");
    }
    const size_t tb = t64.size() * g->esz;
    if ((rc = dalloc(g, &Lv.tab, tb)) != ELL_OK) return bail(rc);
    if (g->prec == ELL_FP64) {
      if (hipMemcpy(Lv.tab, t64.data(), tb, hipMemcpyHostToDevice) != hipSuccess)
        return bail(fail(ELL_ERR_HIP, "table upload failed"));
    } else {
      level_table32(g, l, t64, t32);
      if (hipMemcpy(Lv.tab, t32.data(), tb, hipMemcpyHostToDevice) != hipSuccess)
        return bail(fail(ELL_ERR_HIP, "table upload failed"));
    }
    if (l > 0) {
      const size_t vb = 2 * (size_t)Lv.geo.cs * g->esz;
      if ((rc = dalloc(g, &Lv.b, vb)) != ELL_OK) return bail(rc);
      if ((rc = dalloc(g, &Lv.u, vb)) != ELL_OK) return bail(rc);
    }
  }
  const Geo &G0 = g->lev[0].geo;
  g->n0 = 2 * G0.cs;
  const size_t vb = (size_t)g->n0 * 8;
  void *tmp;
  if ((rc = dalloc(g, &tmp, vb)) != ELL_OK) return bail(rc);
  g->us = (double *)tmp;
  if ((rc = dalloc(g, &tmp, vb)) != ELL_OK) return bail(rc);
  g->r = (double *)tmp;
  if ((rc = dalloc(g, &tmp, vb)) != ELL_OK) return bail(rc);
  g->z = (double *)tmp;
  if ((rc = dalloc(g, &tmp, vb)) != ELL_OK) return bail(rc);
  g->p = (double *)tmp;
  if ((rc = dalloc(g, &tmp, vb)) != ELL_OK) return bail(rc);
  g->q = (double *)tmp;
  if ((rc = dalloc(g, &tmp, vb)) != ELL_OK) return bail(rc);
  g->p2 = (double *)tmp;
  if ((rc = dalloc(g, &tmp, vb)) != ELL_OK) return bail(rc);
  g->p3 = (double *)tmp;
  if (g->prec != ELL_FP64) {
    if ((rc = dalloc(g, &g->b32, (size_t)g->n0 * 4)) != ELL_OK) return bail(rc);
    if ((rc = dalloc(g, &g->z32, (size_t)g->n0 * 4)) != ELL_OK) return bail(rc);
  }
  if (desc->rho != 1.0)
    if ((rc = dalloc(g, &g->ybuf, (size_t)G0.cs * g->esz)) != ELL_OK) return bail(rc);
  const long long nb = partial_blocks(G0, g->n0);
  g->partial_cap = nb * 2;
  if ((rc = dalloc(g, &tmp, (size_t)g->partial_cap * 8)) != ELL_OK) return bail(rc);
  g->partial = (double *)tmp;
  if ((rc = dalloc(g, &tmp, sizeof(PcgState))) != ELL_OK) return bail(rc);
  g->st = (PcgState *)tmp;
  if (hipMemset(g->st, 0, sizeof(PcgState)) != hipSuccess) return bail(fail(ELL_ERR_HIP, "state clear failed"));
  if (hipHostMalloc((void **)&g->st_host, sizeof(PcgState), hipHostMallocDefault) != hipSuccess) {
    g->st_host = nullptr;
    return bail(fail(ELL_ERR_OOM, "pinned state allocation failed"));
  }
  std::memset(g->st_host, 0, sizeof(PcgState));
  {
    std::vector<double> V(desc->nz);
    for (int k = 0; k < desc->nz; ++k) V[k] = desc->hx * desc->hy * desc->dz[k];
    if ((rc = dalloc(g, &tmp, V.size() * 8)) != ELL_OK) return bail(rc);
    g->vol0 = (double *)tmp;
    if (hipMemcpy(g->vol0, V.data(), V.size() * 8, hipMemcpyHostToDevice) != hipSuccess)
      return bail(fail(ELL_ERR_HIP, "volume upload failed"));
  }
  if (g->prec != ELL_FP64) {
    level_table64(g, 0, t64);
    if (g->varying) {
      const int P = desc->nz + 1;
      for (int sl = TZ; sl < TSLOTS; ++sl)
        for (int k = 0; k < P; ++k) t64[(size_t)sl * P + k] = std::nan("");
    }
    if ((rc = dalloc(g, &tmp, t64.size() * 8)) != ELL_OK) return bail(rc);
    if (hipMemcpy(tmp, t64.data(), t64.size() * 8, hipMemcpyHostToDevice) != hipSuccess)
      return bail(fail(ELL_ERR_HIP, "table upload failed"));
    g->tab64_0 = (const double *)tmp;
  } else {
    g->tab64_0 = (const double *)g->lev[0].tab;
  }
  if (g->varying && (rc = build_varying(g, lam3)) != ELL_OK) return bail(rc);
  *out = g;
  return ELL_OK;
}

int ell_grid_destroy(ell_grid *g) {
  if (!g) return ELL_OK;
  for (auto &p : g->prof)
    for (auto &e : p.ev) (void)hipEventDestroy(e);
  for (void *p : g->allocs) (void)hipFree(p);
  if (g->st_host) (void)hipHostFree(g->st_host);
  delete g;
  return ELL_OK;
}

int ell_grid_levels(const ell_grid *g) {
  if (!g) return fail(ELL_ERR_INVALID, "grid is NULL");
  return g->L;
}

int ell_grid_features(const ell_grid *g, int32_t *mask) {
  if (!g || !mask) return fail(ELL_ERR_INVALID, "NULL argument");
  int m = 0;
  const bool tail =
      g->prec == ELL_FP64 ? coarse_tail_applies<double>(g, g->L - 1) : coarse_tail_applies<float>(g, g->L - 1);
  if (tail) m |= ELL_FEAT_COARSE_TAIL;
  else if (g->d.nu_coarse > 0 && coarse_pair_ok(g, g->L - 1)) m |= ELL_FEAT_COARSE_PAIR;
  if (g->prec == ELL_FP64) {
    if (tile_ok(g, 0)) m |= ELL_FEAT_TILED_SMOOTH;
    if (fused_dot_path<double>(g)) m |= ELL_FEAT_FUSED_DOTS;
    if (fused_update_path<double>(g)) m |= ELL_FEAT_FUSED_UPDATE;
    if (pro_path(g, 1)) m |= ELL_FEAT_FUSED_PROLONG;
    if (g->tiled_ends) m |= ELL_FEAT_TILED_ENDS;
    for (int l = 1; l <= g->L - 2; ++l)
      if (coarse_pro_ok<double>(g, l)) m |= ELL_FEAT_COARSE_PROLONG;
  } else if (hybrid_ok(g)) {  // the FP64 post-smoothing of the mixed-precision V-cycle
    if (tile_ok(g, 0)) m |= ELL_FEAT_TILED_SMOOTH;
    if (fused_dot_path<float>(g)) m |= ELL_FEAT_FUSED_DOTS;
    if (fused_update_path<float>(g)) m |= ELL_FEAT_FUSED_UPDATE;
    if (pro32_path(g)) m |= ELL_FEAT_FUSED_PROLONG;
    if (g->tiled_ends) m |= ELL_FEAT_TILED_ENDS;
    for (int l = 1; l <= g->L - 2; ++l)
      if (coarse_pro_ok<float>(g, l)) m |= ELL_FEAT_COARSE_PROLONG;
  }
  *mask = m;
  return ELL_OK;
}

int ell_apply_A(ell_grid *g, const double *x, double *y, hipStream_t s) {
  if (!g || !x || !y) return fail(ELL_ERR_INVALID, "NULL argument");
  if (x == y) return fail(ELL_ERR_INVALID, "x and y must not alias");
  const Geo &G = g->lev[0].geo;
  const int cb = blocks8(2LL * G.H);
  k_nat2split<double, double><<<cb, kBlock, 0, s>>>(G, x, g->p, nullptr);
  CHK(check_launch("k_nat2split"));
  CHK(launch_apply64(g, g->p, g->q, false, nullptr, s));
  k_split2nat<double, double><<<cb, kBlock, 0, s>>>(G, g->q, y);
  return check_launch("k_split2nat");
}

int ell_apply_A_noalloc(const ell_grid_desc *desc, const double *x, double *y, hipStream_t s) {
  int L = 0;
  CHK(validate(desc, &L));
  if (desc->nz > ELL_NOALLOC_MAX_NZ)
    return fail(ELL_ERR_INVALID, "nz = %d exceeds ELL_NOALLOC_MAX_NZ = %d of the allocation-free apply",
                desc->nz, ELL_NOALLOC_MAX_NZ);
  if (!x || !y) return fail(ELL_ERR_INVALID, "NULL argument");
  if (x == y) return fail(ELL_ERR_INVALID, "x and y must not alias");
  double *area = nullptr;
  CHK(noalloc_area(&area));
  // the table is built on the host (the same values a grid's finest level
  // holds) and travels in kernel arguments, a chunk per launch
  double tab[4 * (ELL_NOALLOC_MAX_NZ + 1)];
  stencil_coeffs(*desc, desc->dz, desc->lambda2, 0, tab);
  const int n = 4 * (desc->nz + 1);
  TabChunk c;
  for (int off = 0; off < n; off += kTabChunk) {
    c.off = off;
    c.n = std::min(kTabChunk, n - off);
    std::memcpy(c.v, tab + off, sizeof(double) * c.n);
    k_put_table<<<1, kBlock, 0, s>>>(area, c);
    CHK(check_launch("k_put_table"));
  }
  const long long plane = (long long)desc->nx * desc->ny;
  const int nseg = apply_segments(desc->nz);
  const dim3 grid((unsigned)((plane + kBlock - 1) / kBlock), (unsigned)nseg);
  k_apply_nat<<<grid, kBlock, 0, s>>>(desc->nx, desc->ny, desc->nz, nseg, area, x, y);
  return check_launch("k_apply_nat");
}

int ell_vcycle(ell_grid *g, const double *r, double *z, hipStream_t s) {
  if (!g || !r || !z) return fail(ELL_ERR_INVALID, "NULL argument");
  if (r == z) return fail(ELL_ERR_INVALID, "r and z must not alias");
  const Geo &G = g->lev[0].geo;
  const int cb = blocks8(2LL * G.H);
  if (g->prec == ELL_FP64) {
    k_nat2split<double, double><<<cb, kBlock, 0, s>>>(G, r, g->r, nullptr);
    CHK(check_launch("k_nat2split"));
    CHK(vcycle_impl<double>(g, g->r, g->z, nullptr, s));
    k_split2nat<double, double><<<cb, kBlock, 0, s>>>(G, g->z, z);
  } else if (hybrid_ok(g)) {
    k_nat2split<double, double><<<cb, kBlock, 0, s>>>(G, r, g->r, nullptr);
    CHK(check_launch("k_nat2split"));
    CHK(vcycle_hybrid(g, g->r, g->z, nullptr, s));
    k_split2nat<double, double><<<cb, kBlock, 0, s>>>(G, g->z, z);
  } else {
    k_nat2split<double, float><<<cb, kBlock, 0, s>>>(G, r, (float *)g->b32, nullptr);
    CHK(check_launch("k_nat2split"));
    CHK(vcycle_impl<float>(g, (const float *)g->b32, (float *)g->z32, nullptr, s));
    k_split2nat<float, double><<<cb, kBlock, 0, s>>>(G, (const float *)g->z32, z);
  }
  return check_launch("k_split2nat");
}

int ell_pcg_solve(ell_grid *g, const double *f, double *u, const ell_solve_opts *opts,
                  ell_solve_stats *stats, hipStream_t s) {
  if (!g || !f || !u) return fail(ELL_ERR_INVALID, "NULL argument");
  if ((const void *)f == (const void *)u) return fail(ELL_ERR_INVALID, "f and u must not alias");
  ell_solve_opts o;
  if (opts) o = *opts;
  else {
    o.rtol = 1e-5;
    o.atol = 0.0;
    o.maxiter = 500;
    o.flexible = 1;
    o.rel_to_rhs = 0;
    o.poll_every = 4;
  }
  if (o.maxiter <= 0 || !(o.rtol >= 0) || !(o.atol >= 0))
    return fail(ELL_ERR_INVALID, "maxiter must be > 0 and tolerances >= 0");
  if (g->prec == ELL_FP64) return pcg_impl<double, double>(g, f, u, o, stats, s);
  if (hybrid_ok(g)) return pcg_impl<float, double>(g, f, u, o, stats, s);
  return pcg_impl<float, float>(g, f, u, o, stats, s);
}

int ell_mg_solve(ell_grid *g, const double *f, double *u, const ell_solve_opts *opts, ell_solve_stats *stats,
                 hipStream_t s) {
  if (!g || !f || !u) return fail(ELL_ERR_INVALID, "NULL argument");
  if ((const void *)f == (const void *)u) return fail(ELL_ERR_INVALID, "f and u must not alias");
  ell_solve_opts o{1e-5, 0.0, 500, 0, 0, 4};
  if (opts) o = *opts;
  if (o.maxiter <= 0 || !(o.rtol >= 0) || !(o.atol >= 0))
    return fail(ELL_ERR_INVALID, "maxiter must be > 0 and tolerances >= 0");
  if (g->prec == ELL_FP64) return mg_impl<double, double>(g, f, u, o, stats, s);
  if (hybrid_ok(g)) return mg_impl<float, double>(g, f, u, o, stats, s);
  return mg_impl<float, float>(g, f, u, o, stats, s);
}

size_t ell_level_elems(const ell_grid *g, int level) {
  if (!g || level < 0 || level >= g->L) return 0;
  return 2 * (size_t)g->lev[level].geo.cs;
}

int ell_to_split(ell_grid *g, int level, const double *src, void *dst, hipStream_t s) {
  CHK(check_level(g, level, false));
  if (!src || !dst) return fail(ELL_ERR_INVALID, "NULL argument");
  const Geo &G = g->lev[level].geo;
  const int cb = blocks8(2LL * G.H);
  if (g->prec == ELL_FP64) k_nat2split<double, double><<<cb, kBlock, 0, s>>>(G, src, (double *)dst, nullptr);
  else k_nat2split<double, float><<<cb, kBlock, 0, s>>>(G, src, (float *)dst, nullptr);
  return check_launch("k_nat2split");
}

int ell_from_split(ell_grid *g, int level, const void *src, double *dst, hipStream_t s) {
  CHK(check_level(g, level, false));
  if (!src || !dst) return fail(ELL_ERR_INVALID, "NULL argument");
  const Geo &G = g->lev[level].geo;
  const int cb = blocks8(2LL * G.H);
  if (g->prec == ELL_FP64) k_split2nat<double, double><<<cb, kBlock, 0, s>>>(G, (const double *)src, dst);
  else k_split2nat<float, double><<<cb, kBlock, 0, s>>>(G, (const float *)src, dst);
  return check_launch("k_split2nat");
}

int ell_level_smooth(ell_grid *g, int level, int colour, int zero_init, const void *b, void *u,
                     hipStream_t s) {
  CHK(check_level(g, level, false));
  if (colour != 0 && colour != 1) return fail(ELL_ERR_INVALID, "colour must be 0 or 1");
  if (!b || !u) return fail(ELL_ERR_INVALID, "NULL argument");
  if (g->prec == ELL_FP64)
    return launch_smooth<double>(g, level, colour, zero_init != 0, (const double *)b, (double *)u, nullptr, s);
  return launch_smooth<float>(g, level, colour, zero_init != 0, (const float *)b, (float *)u, nullptr, s);
}

int ell_level_resid_restrict(ell_grid *g, int level, const void *b, const void *u, void *bc,
                             int black_zero, hipStream_t s) {
  CHK(check_level(g, level, true));
  if (!b || !u || !bc) return fail(ELL_ERR_INVALID, "NULL argument");
  if (g->prec == ELL_FP64)
    return launch_restrict<double>(g, level, (const double *)b, (const double *)u, (double *)bc,
                                   black_zero != 0, nullptr, s);
  return launch_restrict<float>(g, level, (const float *)b, (const float *)u, (float *)bc, black_zero != 0,
                                nullptr, s);
}

int ell_level_prolong_add(ell_grid *g, int level, const void *uc, void *u, int red_only, hipStream_t s) {
  CHK(check_level(g, level, true));
  if (!uc || !u) return fail(ELL_ERR_INVALID, "NULL argument");
  if (g->prec == ELL_FP64)
    return launch_prolong<double>(g, level, (const double *)uc, (double *)u, red_only != 0, nullptr, s);
  return launch_prolong<float>(g, level, (const float *)uc, (float *)u, red_only != 0, nullptr, s);
}

int ell_level_apply(ell_grid *g, int level, const void *x, void *y, hipStream_t s) {
  CHK(check_level(g, level, false));
  if (!x || !y || x == y) return fail(ELL_ERR_INVALID, "bad vector arguments");
  const Geo &G = g->lev[level].geo;
  const int nb = seg_blocks(2LL * G.H);
  if (g->varying && g->prec == ELL_FP64)
    k_apply<double, false, false, 4, true><<<nb, kBlock, 0, s>>>(G, (const double *)g->lev[level].tab,
                                                                 (const double *)x, (double *)y, nullptr, nullptr,
                                                                 g->lev[level].tz3);
  else if (g->varying)
    k_apply<float, false, false, 4, true><<<nb, kBlock, 0, s>>>(G, (const float *)g->lev[level].tab,
                                                                (const float *)x, (float *)y, nullptr, nullptr,
                                                                g->lev[level].tz3f);
  else if (g->prec == ELL_FP64)
    k_apply<double, false, false, 4><<<nb, kBlock, 0, s>>>(G, (const double *)g->lev[level].tab,
                                                           (const double *)x, (double *)y, nullptr, nullptr);
  else
    k_apply<float, false, false, 4><<<nb, kBlock, 0, s>>>(G, (const float *)g->lev[level].tab,
                                                          (const float *)x, (float *)y, nullptr, nullptr);
  return check_launch("k_apply");
}

int ell_profile_enable(ell_grid *g, int family, int max_events) {
  if (!g || family < 0 || family >= ELL_K_COUNT || max_events < 0)
    return fail(ELL_ERR_INVALID, "bad profiling arguments");
  Prof &p = g->prof[family];
  for (auto &e : p.ev) (void)hipEventDestroy(e);
  p.ev.assign(2 * (size_t)max_events, nullptr);
  // device-scope release only: the timestamps are read after the stream has
  // been synchronized, and a record without the system-scope fence adds less
  // idle time to the stream (and to the launches it brackets)
  for (auto &e : p.ev) HIPCHK(hipEventCreateWithFlags(&e, hipEventDisableSystemFence));
  p.cap = max_events;
  p.n = 0;
  p.paused = false;
  return ELL_OK;
}

int ell_profile_pause(ell_grid *g, int family, int paused) {
  if (!g || family < 0 || family >= ELL_K_COUNT) return fail(ELL_ERR_INVALID, "bad profiling arguments");
  g->prof[family].paused = paused != 0;
  return ELL_OK;
}

int ell_profile_read(ell_grid *g, int family, int *count, double *total_ms) {
  if (!g || family < 0 || family >= ELL_K_COUNT || !count || !total_ms)
    return fail(ELL_ERR_INVALID, "bad profiling arguments");
  Prof &p = g->prof[family];
  double tot = 0.0;
  for (int i = 0; i < p.n; ++i) {
    HIPCHK(hipEventSynchronize(p.ev[2 * i + 1]));
    float ms = 0.0f;
    HIPCHK(hipEventElapsedTime(&ms, p.ev[2 * i], p.ev[2 * i + 1]));
    tot += ms;
  }
  *count = p.n;
  *total_ms = tot;
  return ELL_OK;
}

int ell_profile_times(ell_grid *g, int family, float *ms, int cap) {
  if (!g || family < 0 || family >= ELL_K_COUNT || !ms || cap < 0)
    return fail(ELL_ERR_INVALID, "bad profiling arguments");
  Prof &p = g->prof[family];
  for (int i = 0; i < p.n && i < cap; ++i) {
    HIPCHK(hipEventSynchronize(p.ev[2 * i + 1]));
    HIPCHK(hipEventElapsedTime(&ms[i], p.ev[2 * i], p.ev[2 * i + 1]));
  }
  return p.n;
}

int ell_level_layout(const ell_grid *g, int level, int64_t *cols, int64_t *plane_stride,
                     int64_t *colour_stride) {
  CHK(check_level(g, level, false));
  if (!cols || !plane_stride || !colour_stride) return fail(ELL_ERR_INVALID, "NULL argument");
  const Geo &G = g->lev[level].geo;
  *cols = G.H;
  *plane_stride = G.S;
  *colour_stride = G.cs;
  return ELL_OK;
}

int ell_schedule_get(const ell_grid_desc *desc, ell_schedule *out) {
  if (!out) return fail(ELL_ERR_INVALID, "out is NULL");
  int L = 0;
  CHK(validate(desc, &L));
  if (L > ELL_MAX_LEVELS) return fail(ELL_ERR_INVALID, "schedules cover at most %d levels", ELL_MAX_LEVELS);
  *out = schedule_for(desc, L);
  return ELL_OK;
}

int ell_schedule_set(const ell_grid_desc *desc, const ell_schedule *s) {
  int L = 0;
  CHK(validate(desc, &L));
  const SchedKey key = sched_key(desc, L);
  if (!s) {
    std::lock_guard<std::mutex> lk(g_sched_mu);
    g_sched.erase(key);
    return ELL_OK;
  }
  CHK(check_schedule(desc, L, s));
  ell_schedule c = *s;
  for (int l = L; l < ELL_MAX_LEVELS; ++l) c.smooth_nseg[l] = 0;
  std::lock_guard<std::mutex> lk(g_sched_mu);
  g_sched[key] = c;
  return ELL_OK;
}

int ell_autotune(const ell_grid_desc *desc, int32_t iters, ell_schedule *best) {
  if (!best) return fail(ELL_ERR_INVALID, "best is NULL");
  int L = 0;
  CHK(validate(desc, &L));
  if (L > ELL_MAX_LEVELS) return fail(ELL_ERR_INVALID, "schedules cover at most %d levels", ELL_MAX_LEVELS);
  if (iters <= 0) iters = 4;
  const long long n = (long long)desc->nx * desc->ny * desc->nz;
  double *f = nullptr, *u = nullptr;
  if (hipMalloc((void **)&f, n * 8) != hipSuccess || hipMalloc((void **)&u, n * 8) != hipSuccess) {
    if (f) (void)hipFree(f);
    (void)hipGetLastError();
    return fail(ELL_ERR_OOM, "autotune vectors do not fit");
  }
  auto release = [&](int rc) {
    (void)hipFree(f);
    (void)hipFree(u);
    return rc;
  };
  k_fill_hash<<<1024, kBlock>>>(f, n);
  if (check_launch("k_fill_hash") != ELL_OK || hipDeviceSynchronize() != hipSuccess)
    return release(fail(ELL_ERR_HIP, "autotune input fill failed"));
  // milliseconds per iteration of a schedule: median of three timed solves
  auto time_of = [&](const ell_schedule &sch, double *ms) -> int {
    ell_grid *g = nullptr;
    CHK(grid_create(desc, false, &g, &sch));
    const ell_solve_opts warm{0.0, 0.0, 1, 1, 0, 1};
    const ell_solve_opts run{0.0, 0.0, iters, 1, 0, iters};
    std::vector<double> t;
    int rc = ELL_OK;
    for (int rep = 0; rep < 4; ++rep) {
      if (hipMemset(u, 0, n * 8) != hipSuccess || hipDeviceSynchronize() != hipSuccess) {
        rc = fail(ELL_ERR_HIP, "autotune reset failed");
        break;
      }
      const auto t0 = std::chrono::steady_clock::now();
      rc = ell_pcg_solve(g, f, u, rep == 0 ? &warm : &run, nullptr, nullptr);
      const auto t1 = std::chrono::steady_clock::now();
      if (rc != ELL_OK && rc != ELL_NOT_CONVERGED) break;
      rc = ELL_OK;
      if (rep > 0) t.push_back(std::chrono::duration<double, std::milli>(t1 - t0).count());
    }
    ell_grid_destroy(g);
    if (rc != ELL_OK) return rc;
    std::sort(t.begin(), t.end());
    *ms = t[t.size() / 2] / iters;
    return ELL_OK;
  };
  ell_schedule cur = default_schedule(desc, L);
  double best_ms = 0.0;
  int rc = time_of(cur, &best_ms);
  if (rc != ELL_OK) return release(rc);
  auto consider = [&](const ell_schedule &c) -> int {
    double ms = 0.0;
    CHK(time_of(c, &ms));
    if (ms < 0.99 * best_ms) {
      best_ms = ms;
      cur = c;
    }
    return ELL_OK;
  };
  // the operator step
  for (int tile = 1; tile >= 0; --tile) {
    if (tile && (desc->nx < 2 || desc->ny < 2)) continue;
    for (int ns : {1, 2, 4}) {
      if (tile == cur.apply_tile && ns == cur.apply_nseg) continue;
      ell_schedule c = cur;
      c.apply_tile = tile;
      c.apply_nseg = ns;
      if ((rc = consider(c)) != ELL_OK) return release(rc);
    }
  }
  // the smoother segments of the finest level, then of each coarse level
  for (int ns : {4, 8}) {
    if (ns == cur.smooth_nseg[0] || (ns == 8 && seg_len(desc->nz, 8) > 16)) continue;
    ell_schedule c = cur;
    c.smooth_nseg[0] = ns;
    if ((rc = consider(c)) != ELL_OK) return release(rc);
  }
  for (int l = 1; l < L; ++l) {
    for (int ns : {4, 8, 16}) {
      if (ns == cur.smooth_nseg[l] || !smooth_nseg_fits(ns, desc->nz)) continue;
      ell_schedule c = cur;
      c.smooth_nseg[l] = ns;
      if ((rc = consider(c)) != ELL_OK) return release(rc);
    }
  }
  cur.ms_per_iter = best_ms;
  {
    std::lock_guard<std::mutex> lk(g_sched_mu);
    g_sched[sched_key(desc, L)] = cur;
  }
  *best = cur;
  return release(ELL_OK);
}

int ell_set_tuning(int key, int value) {
  if (value < 0 || value > (1 << 20)) return fail(ELL_ERR_INVALID, "tuning value out of range");
  switch (key) {
    case ELL_TUNE_PLANE_PAD: g_plane_pad = value; return ELL_OK;
    case ELL_TUNE_COLOUR_PAD: g_colour_pad = value; return ELL_OK;
    case ELL_TUNE_STENCIL_SEG:
      if (value != 1 && value != 2 && value != 4) return fail(ELL_ERR_INVALID, "segments must be 1, 2 or 4");
      g_stencil_seg = value;
      return ELL_OK;
    case ELL_TUNE_APPLY_TILE:
      if (value != 0 && value != 1) return fail(ELL_ERR_INVALID, "apply tiling is 0 or 1");
      g_apply_tile = value;
      return ELL_OK;
    case ELL_TUNE_BATCH_GRAPH:
      if (value != 0 && value != 1) return fail(ELL_ERR_INVALID, "batch graphs are 0 or 1");
      g_batch_graph = value;
      return ELL_OK;
    case ELL_TUNE_SMOOTH_TILE:
      if (value != 0 && value != 1) return fail(ELL_ERR_INVALID, "smoother tiling is 0 or 1");
      g_smooth_tile = value;
      return ELL_OK;
    case ELL_TUNE_FUSED_DOT:
      if (value != 0 && value != 1) return fail(ELL_ERR_INVALID, "fused dots are 0 or 1");
      g_fused_dot = value;
      return ELL_OK;
    case ELL_TUNE_FUSED_UPDATE:
      if (value != 0 && value != 1) return fail(ELL_ERR_INVALID, "the fused residual update is 0 or 1");
      g_fused_update = value;
      return ELL_OK;
    case ELL_TUNE_FUSED_PROLONG:
      if (value != 0 && value != 1) return fail(ELL_ERR_INVALID, "the fused prolongation is 0 or 1");
      g_fused_prolong = value;
      return ELL_OK;
    case ELL_TUNE_TILED_ENDS:
      if (value != 0 && value != 1) return fail(ELL_ERR_INVALID, "tiled solve ends are 0 or 1");
      g_tiled_ends = value;
      return ELL_OK;
    case ELL_TUNE_COARSE_TAIL:
      if (value != 0 && value != 1) return fail(ELL_ERR_INVALID, "the coarse tail is 0 or 1");
      g_coarse_tail = value;
      return ELL_OK;
    case ELL_TUNE_COARSE_PAIR:
      if (value != 0 && value != 1) return fail(ELL_ERR_INVALID, "the coarse sweep pairs are 0 or 1");
      g_coarse_pair = value;
      return ELL_OK;
    default: return fail(ELL_ERR_INVALID, "unknown tuning key %d", key);
  }
}

}  // extern "C"

#include "ell_batch.inl"
