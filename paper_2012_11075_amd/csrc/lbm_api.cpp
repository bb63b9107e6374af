// lbm_api.cpp -- host side of the C ABI declared in include/lbm.h.
//
// Validation, workspace layout, the ping-pong state, the FP32 storage shift,
// HIP-graph replay of step sequences and the fixed-order final reduction of
// the observe pass.  All device work is in lbm_kernels.hip.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <bitset>
#include <cmath>
#include <cstdio>
#include <cstring>
#include <mutex>
#include <string>
#include <vector>

#include "lbm.h"
#include "lbm_kernels3d.h"

using lbmk::Q;

namespace {

constexpr double W[Q] = {4.0 / 9.0,  1.0 / 9.0,  1.0 / 9.0,  1.0 / 9.0, 1.0 / 9.0,
                         1.0 / 36.0, 1.0 / 36.0, 1.0 / 36.0, 1.0 / 36.0};
constexpr size_t ALIGN = 256;
constexpr int MIN_ROWS = 4;
constexpr int MIN_BLOCK = 64;

thread_local std::string g_thread_error;

size_t align_up(size_t v, size_t a) { return (v + a - 1) / a * a; }

bool is_finite(double v) { return std::isfinite(v); }

// Layout of a context's workspace.
struct Layout {
  lbmk::Geometry g;
  lbmk::Geometry3 g3;   // 3-D lattices (nz > 1) only
  bool d3 = false;
  int q = Q;            // populations per node: 9 (D2Q9), 19 (D3Q19) or 27 (D3Q27)
  size_t elem;
  size_t state_bytes;   // one population copy
  size_t staging_bytes; // dense double fields: 4 (2-D: rho, ux, uy, mu) or 5 (3-D: + uz)
  size_t partial_count; // blocks of the smallest tiling
  size_t off_a, off_b, off_staging, off_partials, total;
};

// Velocities of a 3-D lattice: 19 (D3Q19, lattice3 = 0 or 19) or 27.
int q3_of(const lbm_params& p) { return p.lattice3 == lbmk::Q27 ? lbmk::Q27 : lbmk::Q3; }

bool valid_params(const lbm_params* p, std::string* why) {
  if (!p) return *why = "params is NULL", false;
  if (p->nx < 1 || p->ny < 1) return *why = "nx and ny must be >= 1", false;
  if (p->nz < 0) return *why = "nz must be >= 0", false;
  if ((long long)p->nx * p->ny * std::max(1, p->nz) > (1LL << 31))
    return *why = "lattice larger than 2^31 nodes", false;
  if (!is_finite(p->tau) || p->tau <= 0.5) return *why = "tau must be finite and > 1/2", false;
  if (!is_finite(p->beta) || p->beta < 0) return *why = "beta must be finite and >= 0", false;
  if (!is_finite(p->kappa) || p->kappa < 0) return *why = "kappa must be finite and >= 0", false;
  if (!is_finite(p->rho_l) || !is_finite(p->rho_v) || !is_finite(p->rho0) || !is_finite(p->rho_ref))
    return *why = "densities must be finite", false;
  if (p->precision != LBM_FP64 && p->precision != LBM_FP32_SHIFTED)
    return *why = "unknown precision", false;
  if (p->force_stencil != 0 && p->force_stencil != 1) return *why = "force_stencil must be 0 or 1", false;
  if (p->force_stencil == 1 && p->ny > 65535)
    return *why = "the fourth-order force stencil needs ny <= 65535", false;
  // the 2-D kernels hold the row pitch, 9 * nx rounded up to 32 elements, in
  // an int
  if (p->nz <= 1 && (long long)Q * (((long long)p->nx + 31) / 32 * 32) > 0x7fffffffLL)
    return *why = "2-D lattices need 9 * nx (rounded up to 32) <= 2^31 - 1", false;
  if (p->lattice3 != 0 && p->lattice3 != lbmk::Q3 && p->lattice3 != lbmk::Q27)
    return *why = "lattice3 must be 0, 19 or 27", false;
  if (p->nz <= 1 && p->lattice3 != 0) return *why = "lattice3 applies to 3-D lattices (nz > 1)", false;
  if (p->nz > 1) {
    if (p->force_stencil != 0) return *why = "3-D lattices use the central force stencil", false;
    if (p->ny > 65535 || p->nz > 65535) return *why = "3-D lattices need ny, nz <= 65535", false;
    // the fused step addresses one z-plane of populations with 32-bit offsets
    const long long px = ((long long)p->nx + 31) / 32 * 32;
    const long long elem = p->precision == LBM_FP64 ? 8 : 4;
    if ((long long)p->ny * q3_of(*p) * px * elem > 0xffffffffLL)
      return *why = "3-D lattices need a z-plane of populations (q * ny * nx * element bytes) "
                    "below 4 GiB",
             false;
  }
  return true;
}

Layout make_layout(const lbm_params& p) {
  Layout L{};
  L.elem = p.precision == LBM_FP64 ? 8 : 4;
  L.g.nx = p.nx;
  L.g.ny = p.ny;
  // Row-interleaved planes, f[y][q][x]: the nine population rows of a lattice
  // row are contiguous (each 32-element aligned), so a row's loads and stores
  // stream through one region of memory instead of nine.
  const size_t px = align_up((size_t)p.nx, 32);
  L.g.plane = (long long)px;         // elements between populations of a row
  L.g.pitch = (int)(Q * px);         // elements between lattice rows
  L.state_bytes = align_up((size_t)p.ny * Q * px * L.elem, ALIGN);
  L.staging_bytes = align_up((size_t)4 * p.nx * p.ny * sizeof(double), ALIGN);
  const size_t strips = (p.nx + MIN_BLOCK - 1) / MIN_BLOCK;
  const size_t chunks = (p.ny + MIN_ROWS - 1) / MIN_ROWS;
  L.partial_count = strips * chunks;
  if (p.nz > 1) {
    // D3Q19 or D3Q27, f[z][y][q][x]: the q population rows of a lattice row
    // are contiguous, as in two dimensions
    L.d3 = true;
    L.q = q3_of(p);
    L.g3.nx = p.nx;
    L.g3.ny = p.ny;
    L.g3.nz = p.nz;
    L.g3.q = L.q;
    L.g3.plane = (long long)px;
    L.g3.pitch = (long long)L.q * px;
    L.g3.slab = L.g3.pitch * p.ny;
    const size_t n = (size_t)p.nx * p.ny * p.nz;
    L.state_bytes = align_up((size_t)p.nz * p.ny * L.q * px * L.elem, ALIGN);
    L.staging_bytes = align_up(5 * n * sizeof(double), ALIGN);
    L.partial_count = (size_t)lbmk::blocks3(L.g3);
  }
  L.off_a = 0;
  L.off_b = L.off_a + L.state_bytes;
  L.off_staging = L.off_b + L.state_bytes;
  L.off_partials = L.off_staging + L.staging_bytes;
  L.total = L.off_partials + align_up(L.partial_count * lbmk::NPART * sizeof(double), ALIGN);
  return L;
}

// Equilibrium at rest feq_i(rho, 0) of a scheme (Eq. 3 for both standard
// forms / Eq. 24).
void feq_rest(const lbm_params& p, int scheme, double rho, double* f) {
  for (int i = 0; i < Q; ++i) {
    if (scheme != LBM_WELL_BALANCED)
      f[i] = W[i] * rho;
    else
      f[i] = (i == 0) ? rho - (1.0 - W[0]) * p.rho0 : W[i] * p.rho0;
  }
}

// Storage shift s_i of a scheme (zero for FP64): the scheme's equilibrium at
// rest at rho_ref, so that stored values are departures from it (for WB with
// rho0 = 0 that is rho_ref on f_0 only); shift_all selects w_i rho_ref for
// either scheme.
void shift_of(const lbm_params& p, int scheme, double* s) {
  for (int i = 0; i < Q; ++i) s[i] = 0.0;
  if (p.precision == LBM_FP64) return;
  if (p.shift_all) {
    for (int i = 0; i < Q; ++i) s[i] = W[i] * p.rho_ref;
  } else {
    feq_rest(p, scheme, p.rho_ref, s);
  }
}

lbmk::Physics make_physics(const lbm_params& p, int scheme) {
  lbmk::Physics ph{};
  ph.omega = 1.0 / p.tau;
  ph.fpre = 1.0 - 0.5 / p.tau;
  ph.beta = p.beta;
  ph.kappa = p.kappa;
  ph.rho_l = p.rho_l;
  ph.rho_v = p.rho_v;
  ph.rho_ref = p.precision == LBM_FP64 ? 0.0 : p.rho_ref;
  double s[Q], fr[Q];
  shift_of(p, scheme, s);
  feq_rest(p, scheme, ph.rho_ref, fr);
  for (int i = 0; i < Q; ++i) ph.geq_c[i] = fr[i] - s[i];
  return ph;
}

// 3-D weights in the kernels' velocity order: rest, 6 axis, 12 edge and
// (D3Q27) 8 corner directions.
double w3(int q, int i) {
  if (q == lbmk::Q3) return i == 0 ? 1.0 / 3.0 : (i < 7 ? 1.0 / 18.0 : 1.0 / 36.0);
  return i == 0 ? 8.0 / 27.0 : (i < 7 ? 2.0 / 27.0 : (i < 19 ? 1.0 / 54.0 : 1.0 / 216.0));
}

// The 3-D counterparts of feq_rest and shift_of (q3_of(p) entries; the
// arrays hold QMAX3).
void feq3_rest(const lbm_params& p, int scheme, double rho, double* f) {
  const int q = q3_of(p);
  for (int i = 0; i < lbmk::QMAX3; ++i) f[i] = 0.0;
  for (int i = 0; i < q; ++i) {
    if (scheme != LBM_WELL_BALANCED)
      f[i] = w3(q, i) * rho;
    else
      f[i] = (i == 0) ? rho - (1.0 - w3(q, 0)) * p.rho0 : w3(q, i) * p.rho0;
  }
}

void shift3_of(const lbm_params& p, int scheme, double* s) {
  const int q = q3_of(p);
  for (int i = 0; i < lbmk::QMAX3; ++i) s[i] = 0.0;
  if (p.precision == LBM_FP64) return;
  if (p.shift_all) {
    for (int i = 0; i < q; ++i) s[i] = w3(q, i) * p.rho_ref;
  } else {
    feq3_rest(p, scheme, p.rho_ref, s);
  }
}

lbmk::Physics3 make_physics3(const lbm_params& p, int scheme) {
  lbmk::Physics3 ph{};
  ph.omega = 1.0 / p.tau;
  ph.fpre = 1.0 - 0.5 / p.tau;
  ph.beta = p.beta;
  ph.kappa = p.kappa;
  ph.rho_l = p.rho_l;
  ph.rho_v = p.rho_v;
  ph.rho0 = p.rho0;
  ph.rho_ref = p.precision == LBM_FP64 ? 0.0 : p.rho_ref;
  double fr[lbmk::QMAX3];
  shift3_of(p, scheme, ph.s);
  feq3_rest(p, scheme, ph.rho_ref, fr);
  for (int i = 0; i < lbmk::QMAX3; ++i) ph.c[i] = fr[i] - ph.s[i];
  return ph;
}

lbmk::Tiling make_tiling(const lbmk::Geometry& g, int block, int rows, int depth) {
  lbmk::Tiling t{};
  t.block = block;
  t.depth = depth;
  t.rows = std::max(MIN_ROWS, std::min(rows, g.ny));
  t.strips = (g.nx + block - 1) / block;
  t.chunks = (g.ny + t.rows - 1) / t.rows;
  return t;
}

// Default tile, by lattice width (measured with 100-step graphs).  Lattices
// up to 512 wide are latency-bound: a step lasts about as long as one
// block's march through its chunk, so they get many 4-row chunks in 64-wide
// strips (256-wide at depth 1 for the force-stencil variant, whose block
// widths are 256 and 512): a 256^2 step takes ~12 us instead of ~35 us with
// 256 x 16 tiles.  Up to 1024 wide: 256-wide strips, chunks of at least 8
// rows, about 2048 blocks.  Wider: about 512 blocks with chunks of at least
// 16 rows (2048^2 FP64: 32-row chunks, 114 us, against 115 us with 16 and
// 121 us with 8).
lbmk::Tiling default_tiling(const lbmk::Geometry& g, bool stencil4) {
  int block = 256, depth = 2;
  long long target = 2048, min_rows = 16;
  if (g.nx <= 512) {
    block = stencil4 ? 256 : 64;
    depth = stencil4 ? 1 : 2;
    min_rows = 4;
  } else if (g.nx <= 1024) {
    min_rows = 8;
  } else {
    target = 512;
  }
  const int strips = (g.nx + block - 1) / block;
  long long rows = ((long long)g.ny * strips + target - 1) / target;
  rows = std::max<long long>(min_rows, std::min<long long>(rows, 128));
  return make_tiling(g, block, (int)rows, depth);
}

}  // namespace

struct lbm_ctx {
  lbm_params prm{};
  Layout L{};
  lbmk::Tiling tl{};
  lbmk::Tiling3 tl3{};  // fused 3-D step (nz > 1)
  char* ws = nullptr;
  hipStream_t stream = nullptr;
  int cur = 0;           // 0: state in buffer A, 1: in buffer B
  bool initialised = false;
  int scheme = LBM_WELL_BALANCED;  // scheme the storage shift currently follows
  int64_t step = 0;
  int graph_steps = 0;
  hipGraphExec_t graph[3][2] = {};  // [scheme][cur]
  std::string err;

  void* buf(int which) const { return ws + (which == 0 ? L.off_a : L.off_b); }
  void* state() const { return buf(cur); }
  double* staging() const { return (double*)(ws + L.off_staging); }
  double* partials() const { return (double*)(ws + L.off_partials); }
  int storage() const { return prm.precision == LBM_FP64 ? lbmk::FP64 : lbmk::FP32; }
  long long nodes() const { return (long long)prm.nx * prm.ny * std::max(1, prm.nz); }
  bool d3() const { return L.d3; }
};

namespace {

lbm_status fail(lbm_ctx* c, lbm_status s, const std::string& msg) {
  if (c)
    c->err = msg;
  else
    g_thread_error = msg;
  return s;
}

lbm_status hip_fail(lbm_ctx* c, hipError_t e, const char* what) {
  return fail(c, LBM_EHIP, std::string(what) + ": " + hipGetErrorString(e));
}

#define HIPCHK(ctx, call)                                    \
  do {                                                       \
    hipError_t e_ = (call);                                  \
    if (e_ != hipSuccess) return hip_fail((ctx), e_, #call); \
  } while (0)

void drop_graphs(lbm_ctx* c) {
  for (auto& row : c->graph)
    for (auto& g : row)
      if (g) {
        (void)hipGraphExecDestroy(g);
        g = nullptr;
      }
}

// Enqueue n plain step launches.
// Tile depth 4 selects the two-step kernel (2-D lattices with the central
// stencil, blocks of 128 or 256 threads; lbm_set_tile checks).
bool fused_pairs(const lbm_ctx* c) { return !c->d3() && c->tl.depth == 4; }

lbm_status launch_steps(lbm_ctx* c, int64_t n, int scheme, hipStream_t s) {
  const lbmk::Physics ph = make_physics(c->prm, scheme);
  const lbmk::Physics3 ph3 = make_physics3(c->prm, scheme);
  if (fused_pairs(c)) {
    // two steps per launch; an odd count ends with one step of the same tile
    int64_t k = 0;
    for (; k + 2 <= n; k += 2) {
      HIPCHK(c, lbmk::launch_step2(c->storage(), scheme, c->tl.block, c->L.g, ph, c->tl.rows,
                                   c->buf(c->cur), c->buf(1 - c->cur), s));
      c->cur = 1 - c->cur;
    }
    if (k < n) {
      lbmk::Tiling t1 = c->tl;
      t1.depth = 3;
      HIPCHK(c, lbmk::launch_step(c->storage(), scheme, c->L.g, ph, t1, c->buf(c->cur),
                                  c->buf(1 - c->cur), s));
      c->cur = 1 - c->cur;
    }
    return LBM_OK;
  }
  for (int64_t k = 0; k < n; ++k) {
    if (c->d3()) {
      HIPCHK(c, lbmk::launch_step3(c->storage(), scheme, c->L.g3, ph3, c->tl3, c->buf(c->cur),
                                   c->buf(1 - c->cur), s));
    } else if (c->prm.force_stencil == 1) {
      HIPCHK(c, lbmk::launch_step4(c->storage(), scheme, c->L.g, ph, c->tl, c->buf(c->cur),
                                   c->buf(1 - c->cur), s));
    } else {
      HIPCHK(c, lbmk::launch_step(c->storage(), scheme, c->L.g, ph, c->tl, c->buf(c->cur),
                                  c->buf(1 - c->cur), s));
    }
    c->cur = 1 - c->cur;
  }
  return LBM_OK;
}

// Graph of graph_steps steps starting from the current buffer, kept per
// starting buffer (even count: one-step launches leave the buffer parity as
// it was; two-step launches flip it when graph_steps / 2 is odd, and
// lbm_step follows that flip).
lbm_status get_graph(lbm_ctx* c, int scheme, hipGraphExec_t* out) {
  hipGraphExec_t& slot = c->graph[scheme][c->cur];
  if (!slot) {
    hipStream_t cs;
    HIPCHK(c, hipStreamCreateWithFlags(&cs, hipStreamNonBlocking));
    hipError_t e = hipStreamBeginCapture(cs, hipStreamCaptureModeRelaxed);
    if (e != hipSuccess) {
      (void)hipStreamDestroy(cs);
      return hip_fail(c, e, "hipStreamBeginCapture");
    }
    const int cur0 = c->cur;
    lbm_status st = launch_steps(c, c->graph_steps, scheme, cs);
    c->cur = cur0;
    hipGraph_t graph = nullptr;
    e = hipStreamEndCapture(cs, &graph);
    (void)hipStreamDestroy(cs);
    if (st != LBM_OK) {
      if (graph) (void)hipGraphDestroy(graph);
      return st;
    }
    if (e != hipSuccess) return hip_fail(c, e, "hipStreamEndCapture");
    e = hipGraphInstantiate(&slot, graph, nullptr, nullptr, 0);
    (void)hipGraphDestroy(graph);
    if (e != hipSuccess) {
      slot = nullptr;
      return hip_fail(c, e, "hipGraphInstantiate");
    }
  }
  *out = slot;
  return LBM_OK;
}

lbm_status convert_shift(lbm_ctx* c, int to_scheme) {
  if (c->prm.precision == LBM_FP64 || to_scheme == c->scheme) {
    c->scheme = to_scheme;
    return LBM_OK;
  }
  if (c->d3()) {
    lbmk::Physics3 d{};
    double so[lbmk::QMAX3], sn[lbmk::QMAX3];
    shift3_of(c->prm, c->scheme, so);
    shift3_of(c->prm, to_scheme, sn);
    bool same = true;
    for (int i = 0; i < lbmk::QMAX3; ++i) {
      d.s[i] = so[i] - sn[i];
      same = same && d.s[i] == 0.0;
    }
    if (!same) HIPCHK(c, lbmk::launch_reshift3(c->storage(), c->L.g3, d, c->state(), c->stream));
    c->scheme = to_scheme;
    return LBM_OK;
  }
  double so[Q], sn[Q], d[Q];
  shift_of(c->prm, c->scheme, so);
  shift_of(c->prm, to_scheme, sn);
  bool same = true;
  for (int i = 0; i < Q; ++i) {
    d[i] = so[i] - sn[i];
    same = same && d[i] == 0.0;
  }
  if (!same) HIPCHK(c, lbmk::launch_reshift(c->storage(), c->L.g, d, c->state(), c->stream));
  c->scheme = to_scheme;
  return LBM_OK;
}

bool valid_scheme(int s) {
  return s == LBM_STANDARD || s == LBM_WELL_BALANCED || s == LBM_STANDARD_EQ_FORCING;
}

// nullptr if the context can run `scheme`, else the reason it cannot.
const char* scheme_error(const lbm_ctx*, int scheme) {
  return valid_scheme(scheme) ? nullptr : "unknown scheme";
}

}  // namespace

extern "C" {

size_t lbm_workspace_bytes(const lbm_params* p) {
  std::string why;
  if (!valid_params(p, &why)) return 0;
  return make_layout(*p).total;
}

lbm_status lbm_create(const lbm_params* p, void* ws, size_t bytes, void* stream, lbm_ctx** out) {
  std::string why;
  if (!out) return fail(nullptr, LBM_EINVAL, "out is NULL");
  *out = nullptr;
  if (!valid_params(p, &why)) return fail(nullptr, LBM_EINVAL, why);
  if (!ws) return fail(nullptr, LBM_EINVAL, "workspace is NULL");
  if ((uintptr_t)ws % ALIGN) return fail(nullptr, LBM_EINVAL, "workspace not 256-byte aligned");
  Layout L = make_layout(*p);
  if (bytes < L.total)
    return fail(nullptr, LBM_ENOSPACE,
                "workspace too small: need " + std::to_string(L.total) + " bytes");
  lbmk::Tiling3 t3{};
  if (L.d3) {
    // default chunking, measured at 256^3: D3Q19 about 1024 blocks for FP64
    // (two rounds of two blocks per CU), 512 for FP32 (one round, long
    // chunks), one plane in flight; D3Q27 (one block per CU in FP64) 512
    // blocks, with two planes in flight in FP64 (2.05 ms against 2.19 ms)
    if (L.q == lbmk::Q27)
      t3 = lbmk::make_tiling3(L.g3, 8, 0, p->precision == LBM_FP64 ? 2 : 1, 512);
    else
      t3 = lbmk::make_tiling3(L.g3, 8, 0, 1, p->precision == LBM_FP64 ? 1024 : 512);
    if (lbmk::blocks_of(t3) > 0x7fffffffLL)
      return fail(nullptr, LBM_EINVAL, "3-D lattice too large for one launch");
  }
  lbm_ctx* c = new lbm_ctx();
  c->prm = *p;
  c->L = L;
  c->ws = (char*)ws;
  c->stream = (hipStream_t)stream;
  c->tl = default_tiling(L.g, p->force_stencil == 1);
  c->tl3 = t3;
  *out = c;
  return LBM_OK;
}

}  // extern "C"

namespace {

// Populations f = feq(rho, u) of the scheme from host fields (uz: 3-D only).
lbm_status init_impl(lbm_ctx* c, const double* rho, const double* ux, const double* uy,
                     const double* uz, int scheme) {
  if (!c) return fail(nullptr, LBM_EINVAL, "ctx is NULL");
  if (!rho) return fail(c, LBM_EINVAL, "rho is NULL");
  if (const char* why = scheme_error(c, scheme)) return fail(c, LBM_EINVAL, why);
  const bool d3 = c->d3();
  if (!d3 && uz) return fail(c, LBM_EINVAL, "uz is for 3-D lattices");
  if (!d3 && (ux == nullptr) != (uy == nullptr))
    return fail(c, LBM_EINVAL, "give both ux and uy or neither");
  if (d3 && !((ux && uy && uz) || (!ux && !uy && !uz)))
    return fail(c, LBM_EINVAL, "give ux, uy and uz or none of them");
  const long long n = c->nodes();
  for (long long k = 0; k < n; ++k) {
    if (!is_finite(rho[k]) || !(rho[k] > 0.0))
      return fail(c, LBM_EINVAL, "rho must be finite and > 0 (node " + std::to_string(k) + ")");
    if (ux && (!is_finite(ux[k]) || !is_finite(uy[k]) || (uz && !is_finite(uz[k]))))
      return fail(c, LBM_EINVAL, "u must be finite (node " + std::to_string(k) + ")");
  }
  double* st = c->staging();
  const size_t fb = (size_t)n * sizeof(double);
  HIPCHK(c, hipMemcpyAsync(st, rho, fb, hipMemcpyHostToDevice, c->stream));
  if (ux) {
    HIPCHK(c, hipMemcpyAsync(st + n, ux, fb, hipMemcpyHostToDevice, c->stream));
    HIPCHK(c, hipMemcpyAsync(st + 2 * n, uy, fb, hipMemcpyHostToDevice, c->stream));
    if (uz) HIPCHK(c, hipMemcpyAsync(st + 3 * n, uz, fb, hipMemcpyHostToDevice, c->stream));
  }
  c->cur = 0;
  c->scheme = scheme;
  if (d3) {
    HIPCHK(c, lbmk::launch_init3(c->storage(), scheme, c->L.g3, make_physics3(c->prm, scheme), st,
                                 ux ? st + n : nullptr, ux ? st + 2 * n : nullptr,
                                 ux ? st + 3 * n : nullptr, c->state(), c->stream));
  } else {
    const lbmk::Physics ph = make_physics(c->prm, scheme);
    HIPCHK(c, lbmk::launch_init(c->storage(), scheme, c->L.g, ph, st, ux ? st + n : nullptr,
                                ux ? st + 2 * n : nullptr, c->state(), c->stream));
  }
  HIPCHK(c, hipStreamSynchronize(c->stream));
  c->step = 0;
  c->initialised = true;
  return LBM_OK;
}

}  // namespace

extern "C" {

lbm_status lbm_init(lbm_ctx* c, const double* rho, const double* ux, const double* uy,
                    lbm_scheme scheme) {
  if (c && c->d3() && (ux || uy))
    return fail(c, LBM_EINVAL, "3-D lattices take u through lbm_init3d");
  return init_impl(c, rho, ux, uy, nullptr, scheme);
}

lbm_status lbm_init3d(lbm_ctx* c, const double* rho, const double* ux, const double* uy,
                      const double* uz, lbm_scheme scheme) {
  return init_impl(c, rho, ux, uy, uz, scheme);
}

lbm_status lbm_step(lbm_ctx* c, int64_t n, lbm_scheme scheme) {
  if (!c) return fail(nullptr, LBM_EINVAL, "ctx is NULL");
  if (n < 0) return fail(c, LBM_EINVAL, "n must be >= 0");
  if (const char* why = scheme_error(c, scheme)) return fail(c, LBM_EINVAL, why);
  if (!c->initialised) return fail(c, LBM_ESTATE, "lbm_step before lbm_init");
  lbm_status st = convert_shift(c, scheme);
  if (st != LBM_OK) return st;
  int64_t left = n;
  if (c->graph_steps >= 2) {
    while (left >= c->graph_steps) {
      hipGraphExec_t ge;
      st = get_graph(c, scheme, &ge);
      if (st != LBM_OK) return st;
      HIPCHK(c, hipGraphLaunch(ge, c->stream));
      // a replay of two-step launches swaps the buffers once per two steps
      if (fused_pairs(c) && ((c->graph_steps / 2) & 1)) c->cur = 1 - c->cur;
      left -= c->graph_steps;
    }
  }
  st = launch_steps(c, left, scheme, c->stream);
  if (st != LBM_OK) return st;
  c->step += n;
  return LBM_OK;
}

}  // extern "C"

namespace {

// Fixed-order finish of `count` per-tile records (lbmk::NPART doubles each):
// max of max|u| and of the non-finite flag, compensated (Neumaier) sums of
// mass, kinetic energy and momentum, tiles in order.  Returns true when the
// state holds a non-finite value or rho <= 0.
bool finish_partials(const double* part, size_t count, int64_t step, lbm_observation* obs) {
  double umax = 0.0, bad = 0.0;
  double sum[5] = {0.0, 0.0, 0.0, 0.0, 0.0}, comp[5] = {0.0, 0.0, 0.0, 0.0, 0.0};
  auto neumaier = [](double& s, double& c, double v) {
    const double t = s + v;
    if (std::fabs(s) >= std::fabs(v))
      c += (s - t) + v;
    else
      c += (v - t) + s;
    s = t;
  };
  for (size_t b = 0; b < count; ++b) {
    const double* q = part + lbmk::NPART * b;
    umax = std::max(umax, q[0]);
    bad = std::max(bad, q[3]);
    neumaier(sum[0], comp[0], q[1]);
    neumaier(sum[1], comp[1], q[2]);
    for (int a = 0; a < 3; ++a) neumaier(sum[2 + a], comp[2 + a], q[4 + a]);
    if (!is_finite(q[1]) || !is_finite(q[2])) bad = 1.0;
  }
  if (obs) {
    obs->step = step;
    obs->max_u = umax;
    obs->mass = sum[0] + comp[0];
    obs->kinetic_energy = sum[1] + comp[1];
    obs->nonfinite = bad != 0.0;
    for (int a = 0; a < 3; ++a) obs->momentum[a] = sum[2 + a] + comp[2 + a];
  }
  return bad != 0.0;
}

lbm_status observe_impl(lbm_ctx* c, double* rho, double* ux, double* uy, double* uz, double* mu,
                        lbm_observation* obs) {
  if (!c) return fail(nullptr, LBM_EINVAL, "ctx is NULL");
  if (!c->initialised) return fail(c, LBM_ESTATE, "lbm_observe before lbm_init");
  if (uz && !c->d3()) return fail(c, LBM_EINVAL, "uz is for 3-D lattices");
  const long long n = c->nodes();
  double* st = c->staging();
  double* st_mu = st + (c->d3() ? 4 : 3) * n;
  int nb = 0;
  if (c->d3()) {
    // the 3-D pass always computes rho and mu (staging fields 0 and 4)
    const lbmk::ObserveOut3 o{st, ux ? st + n : nullptr, uy ? st + 2 * n : nullptr,
                              uz ? st + 3 * n : nullptr, st_mu, c->partials()};
    HIPCHK(c, lbmk::launch_observe3(c->storage(), c->scheme, c->L.g3,
                                    make_physics3(c->prm, c->scheme), c->state(), st, st_mu, o,
                                    c->stream));
    nb = lbmk::blocks3(c->L.g3);
  } else {
    lbmk::ObserveOut o{rho ? st : nullptr, ux ? st + n : nullptr, uy ? st + 2 * n : nullptr,
                       mu ? st_mu : nullptr, c->partials()};
    const lbmk::Physics ph = make_physics(c->prm, c->scheme);
    if (c->prm.force_stencil == 1) {
      // the variant always computes rho and mu into staging fields 0 and 3
      HIPCHK(c, lbmk::launch_observe4(c->storage(), c->scheme, c->L.g, ph, c->state(), st, st_mu,
                                      o, c->stream));
      nb = lbmk::stencil4_blocks(c->L.g);
    } else {
      HIPCHK(c, lbmk::launch_observe(c->storage(), c->scheme, c->L.g, ph, c->tl, c->state(), o,
                                     c->stream));
      nb = c->tl.blocks();
    }
  }
  const size_t fb = (size_t)n * sizeof(double);
  if (rho) HIPCHK(c, hipMemcpyAsync(rho, st, fb, hipMemcpyDeviceToHost, c->stream));
  if (ux) HIPCHK(c, hipMemcpyAsync(ux, st + n, fb, hipMemcpyDeviceToHost, c->stream));
  if (uy) HIPCHK(c, hipMemcpyAsync(uy, st + 2 * n, fb, hipMemcpyDeviceToHost, c->stream));
  if (uz) HIPCHK(c, hipMemcpyAsync(uz, st + 3 * n, fb, hipMemcpyDeviceToHost, c->stream));
  if (mu) HIPCHK(c, hipMemcpyAsync(mu, st_mu, fb, hipMemcpyDeviceToHost, c->stream));
  std::vector<double> part((size_t)nb * lbmk::NPART);
  HIPCHK(c, hipMemcpyAsync(part.data(), c->partials(), part.size() * sizeof(double),
                           hipMemcpyDeviceToHost, c->stream));
  HIPCHK(c, hipStreamSynchronize(c->stream));
  const bool bad = finish_partials(part.data(), (size_t)nb, c->step, obs);
  if (bad) return fail(c, LBM_ENONFINITE, "state holds NaN/Inf or rho <= 0");
  return LBM_OK;
}

}  // namespace

extern "C" {

lbm_status lbm_observe(lbm_ctx* c, double* rho, double* ux, double* uy, double* mu,
                       lbm_observation* obs) {
  return observe_impl(c, rho, ux, uy, nullptr, mu, obs);
}

lbm_status lbm_observe3d(lbm_ctx* c, double* rho, double* ux, double* uy, double* uz, double* mu,
                         lbm_observation* obs) {
  return observe_impl(c, rho, ux, uy, uz, mu, obs);
}

}  // extern "C"

namespace {

// Reduction records of lbm_observe_noalloc: one record of lbmk::NPART
// doubles per tile of the observe launch, kNoallocTiles at most (8 MiB).
// Every GPU the library runs on holds its own copy until the process ends.
// Host code never uses the array's name as an address: the device address
// of each GPU's copy comes from hipGetSymbolAddress (noalloc_scratch below).
constexpr int kNoallocTiles = 131072;
static __device__ __align__(256) double scratch[(size_t)kNoallocTiles * lbmk::NPART];

constexpr int kMaxDevices = 64;
std::mutex g_scratch_mu;
double* g_scratch_dev[kMaxDevices] = {};

// Device address of the current GPU's copy of `scratch`, looked up once per
// device (with that device current) and kept.
lbm_status noalloc_scratch(lbm_ctx* c, double** out) {
  int dev = -1;
  HIPCHK(c, hipGetDevice(&dev));
  if (dev < 0 || dev >= kMaxDevices) return fail(c, LBM_EINVAL, "device index out of range");
  std::lock_guard<std::mutex> lock(g_scratch_mu);
  if (!g_scratch_dev[dev]) {
    void* ptr = nullptr;
    HIPCHK(c, hipGetSymbolAddress(&ptr, HIP_SYMBOL(scratch)));
    if (!ptr) return fail(c, LBM_EHIP, "hipGetSymbolAddress returned no address");
    g_scratch_dev[dev] = (double*)ptr;
  }
  *out = g_scratch_dev[dev];
  return LBM_OK;
}

}  // namespace

extern "C" {

lbm_status lbm_observe_noalloc(lbm_ctx* c, double* dev_out) {
  if (!c) return fail(nullptr, LBM_EINVAL, "ctx is NULL");
  if (!dev_out) return fail(c, LBM_EINVAL, "dev_out is NULL");
  if (c->d3() || c->prm.force_stencil != 0)
    return fail(c, LBM_EINVAL,
                "lbm_observe_noalloc covers 2-D lattices with the central force stencil");
  const long long nb = c->tl.blocks();
  if (nb > kNoallocTiles)
    return fail(c, LBM_EINVAL,
                "lbm_observe_noalloc holds at most " + std::to_string(kNoallocTiles) +
                    " tiles; this tiling has " + std::to_string(nb) + " (use larger tiles)");
  if (!c->initialised) return fail(c, LBM_ESTATE, "lbm_observe_noalloc before lbm_init");
  double* part = nullptr;
  lbm_status st = noalloc_scratch(c, &part);
  if (st != LBM_OK) return st;
  // every tile writes its whole record, so nothing needs clearing first
  const lbmk::ObserveOut o{nullptr, nullptr, nullptr, nullptr, part};
  HIPCHK(c, lbmk::launch_observe(c->storage(), c->scheme, c->L.g, make_physics(c->prm, c->scheme),
                                 c->tl, c->state(), o, c->stream));
  HIPCHK(c, lbmk::launch_finish_partials(part, (int)nb, dev_out, c->stream));
  return LBM_OK;
}

lbm_status lbm_get_populations_window(lbm_ctx* c, int32_t x0, int32_t y0, int32_t w, int32_t h,
                                      double* f) {
  if (!c) return fail(nullptr, LBM_EINVAL, "ctx is NULL");
  if (!f) return fail(c, LBM_EINVAL, "f is NULL");
  if (c->d3()) return fail(c, LBM_EINVAL, "windows are read from 2-D lattices");
  if (x0 < 0 || y0 < 0 || x0 >= c->prm.nx || y0 >= c->prm.ny)
    return fail(c, LBM_EINVAL, "window origin outside the lattice");
  if (w < 1 || h < 1 || w > c->prm.nx || h > c->prm.ny)
    return fail(c, LBM_EINVAL, "window size must be 1..nx by 1..ny");
  if (!c->initialised) return fail(c, LBM_ESTATE, "no state yet");
  double s[Q];
  shift_of(c->prm, c->scheme, s);
  // through the staging area (4 dense fields) in groups of up to 4 populations
  const size_t n = (size_t)w * h;
  for (int q0 = 0; q0 < Q; q0 += 4) {
    const int m = std::min(4, Q - q0);
    HIPCHK(c, lbmk::launch_unpack_window(c->storage(), c->L.g, s, c->state(), x0, y0, w, h, q0,
                                         m, c->staging(), c->stream));
    HIPCHK(c, hipMemcpyAsync(f + (size_t)q0 * n, c->staging(), (size_t)m * n * sizeof(double),
                             hipMemcpyDeviceToHost, c->stream));
    HIPCHK(c, hipStreamSynchronize(c->stream));
  }
  return LBM_OK;
}

lbm_status lbm_get_populations(lbm_ctx* c, double* f) {
  if (!c) return fail(nullptr, LBM_EINVAL, "ctx is NULL");
  if (!f) return fail(c, LBM_EINVAL, "f is NULL");
  if (!c->initialised) return fail(c, LBM_ESTATE, "no state yet");
  const long long n = c->nodes();
  double s[Q];
  shift_of(c->prm, c->scheme, s);
  const int nq = c->L.q;
  for (int q0 = 0; q0 < nq; q0 += 4) {
    const int m = std::min(4, nq - q0);
    if (c->d3())
      HIPCHK(c, lbmk::launch_unpack3(c->storage(), c->L.g3, make_physics3(c->prm, c->scheme),
                                     c->state(), q0, m, c->staging(), c->stream));
    else
      HIPCHK(c, lbmk::launch_unpack(c->storage(), c->L.g, s, c->state(), q0, m, c->staging(),
                                    c->stream));
    HIPCHK(c, hipMemcpyAsync(f + (size_t)q0 * n, c->staging(), (size_t)m * n * sizeof(double),
                             hipMemcpyDeviceToHost, c->stream));
    HIPCHK(c, hipStreamSynchronize(c->stream));
  }
  return LBM_OK;
}

lbm_status lbm_set_populations(lbm_ctx* c, const double* f, lbm_scheme scheme, int64_t step) {
  if (!c) return fail(nullptr, LBM_EINVAL, "ctx is NULL");
  if (!f) return fail(c, LBM_EINVAL, "f is NULL");
  if (const char* why = scheme_error(c, scheme)) return fail(c, LBM_EINVAL, why);
  const long long n = c->nodes();
  const int nq = c->L.q;
  for (long long k = 0; k < (long long)nq * n; ++k)
    if (!is_finite(f[k])) return fail(c, LBM_EINVAL, "populations must be finite");
  double s[Q];
  shift_of(c->prm, scheme, s);
  c->cur = 0;
  for (int q0 = 0; q0 < nq; q0 += 4) {
    const int m = std::min(4, nq - q0);
    HIPCHK(c, hipMemcpyAsync(c->staging(), f + (size_t)q0 * n, (size_t)m * n * sizeof(double),
                             hipMemcpyHostToDevice, c->stream));
    if (c->d3())
      HIPCHK(c, lbmk::launch_pack3(c->storage(), c->L.g3, make_physics3(c->prm, scheme),
                                   c->staging(), q0, m, c->state(), c->stream));
    else
      HIPCHK(c, lbmk::launch_pack(c->storage(), c->L.g, s, c->staging(), q0, m, c->state(),
                                  c->stream));
    HIPCHK(c, hipStreamSynchronize(c->stream));
  }
  c->scheme = scheme;
  c->step = step;
  c->initialised = true;
  return LBM_OK;
}

lbm_status lbm_set_tile(lbm_ctx* c, int32_t block, int32_t rows, int32_t depth) {
  if (!c) return fail(nullptr, LBM_EINVAL, "ctx is NULL");
  if (c->d3()) {
    // fused 3-D step: block = 32 x ty threads, rows = planes per chunk,
    // depth = planes of populations in flight per thread
    const int ty = block == 0 ? c->tl3.ty : (block % lbmk::M3X ? 0 : block / lbmk::M3X);
    const int d = depth == 0 ? c->tl3.depth : depth;
    if (!lbmk::tiling3_supported(c->L.q, ty, d))
      return fail(c, LBM_EINVAL,
                  c->L.q == lbmk::Q3
                      ? "D3Q19 tiles: block 256 with depth 1..3 or block 512 with depth 1..2"
                      : "D3Q27 tiles: block 256 with depth 1..2");
    if (rows < 0) return fail(c, LBM_EINVAL, "rows (planes per chunk) must be >= 1");
    const lbmk::Tiling3 t = lbmk::make_tiling3(c->L.g3, ty, rows == 0 ? c->tl3.zc : rows, d, 0);
    if (lbmk::blocks_of(t) > 0x7fffffffLL) return fail(c, LBM_EINVAL, "too many blocks");
    drop_graphs(c);
    c->tl3 = t;
    return LBM_OK;
  }
  if (block == 0) block = c->tl.block;
  if (rows == 0) rows = c->tl.rows;
  if (depth == 0) depth = c->tl.depth;
  if (depth == 4) {
    if (c->prm.force_stencil != 0 || !lbmk::step2_block_supported(block))
      return fail(c, LBM_EINVAL,
                  "depth 4 (two steps per launch) needs the central stencil and block 128 or "
                  "256");
  } else if (depth < 1 || depth > 3) {
    return fail(c, LBM_EINVAL, "depth must be 1, 2 or 3 (4: two steps per launch)");
  }
  if (!lbmk::block_width_supported(block))
    return fail(c, LBM_EINVAL, "unsupported block width " + std::to_string(block));
  if (c->prm.force_stencil == 1 && !lbmk::stencil4_block_supported(block))
    return fail(c, LBM_EINVAL, "the force-stencil variant runs on block widths 256 and 512");
  if (rows < MIN_ROWS) return fail(c, LBM_EINVAL, "rows must be >= 4");
  lbmk::Tiling t = make_tiling(c->L.g, block, rows, depth);
  if ((size_t)t.blocks() > c->L.partial_count)
    return fail(c, LBM_EINVAL, "tiling exceeds the reduction area");
  drop_graphs(c);
  c->tl = t;
  return LBM_OK;
}

lbm_status lbm_get_tile(const lbm_ctx* c, int32_t* block, int32_t* rows, int32_t* depth) {
  if (!c) return fail(nullptr, LBM_EINVAL, "ctx is NULL");
  const bool d3 = c->d3();
  if (block) *block = d3 ? lbmk::M3X * c->tl3.ty : c->tl.block;
  if (rows) *rows = d3 ? c->tl3.zc : c->tl.rows;
  if (depth) *depth = d3 ? c->tl3.depth : c->tl.depth;
  return LBM_OK;
}

lbm_status lbm_set_graph_steps(lbm_ctx* c, int32_t steps) {
  if (!c) return fail(nullptr, LBM_EINVAL, "ctx is NULL");
  if (steps < 0 || steps > 4096) return fail(c, LBM_EINVAL, "graph steps must be in [0, 4096]");
  if (steps >= 2 && (steps & 1)) return fail(c, LBM_EINVAL, "graph steps must be even");
  drop_graphs(c);
  c->graph_steps = steps;
  return LBM_OK;
}

lbm_status lbm_destroy(lbm_ctx* c) {
  if (!c) return LBM_OK;
  drop_graphs(c);
  delete c;
  return LBM_OK;
}

const char* lbm_status_string(lbm_status s) {
  switch (s) {
    case LBM_OK: return "ok";
    case LBM_EINVAL: return "invalid argument";
    case LBM_ENOSPACE: return "workspace too small";
    case LBM_EHIP: return "HIP runtime error";
    case LBM_ENONFINITE: return "non-finite state";
    case LBM_ESTATE: return "call out of order";
    case LBM_EBUSY: return "no free slot";
  }
  return "unknown status";
}

const char* lbm_last_error(const lbm_ctx* c) {
  return c ? c->err.c_str() : g_thread_error.c_str();
}

int32_t lbm_kernels_per_step(const lbm_ctx* c) {
  return 1;
}

int32_t lbm_steps_per_launch(const lbm_ctx* c) {
  return c && fused_pairs(c) ? 2 : 1;
}

}  // extern "C"

// ---------------------------------------------------------------- batches

namespace {

constexpr int kBatchBlocks[3] = {64, 128, 256};
// Launch groups: storage x scheme x block x depth for the main step, then
// storage x scheme x depth for the force-stencil variant (block width
// kBatch4Block), then storage x scheme x block width (128, 256) x {two steps
// per launch, one step} for the slots of tile depth 4 (each such slot is in
// both tables, the one-step table serving the last step of an odd step count
// and the observe pass), then storage x scheme x lattice (D3Q19,
// D3Q27) x depth (1, 2) for 3-D lattices (tiles of 32 x kBatch3Ty).
constexpr int kPlainGroups = 2 * 3 * 3 * 3;
constexpr int kStencil4Base = kPlainGroups;
constexpr int kPairBase = kStencil4Base + 2 * 3 * 3;
constexpr int k3dBase = kPairBase + 2 * 3 * 2 * 2;
constexpr int kGroups = k3dBase + 2 * 3 * 2 * 2;
using GroupMask = std::bitset<kGroups>;
enum GroupKind { kMain = 0, kStencil4 = 1, k3d = 2, kPair = 3, kPairOne = 4 };
// Each group's slots are split into two lanes (even and odd slot index), each
// with its own table, launched on its own stream: the lanes hold disjoint
// lattices, so one lane's next step fills the compute units that the other
// lane's step leaves idle at its end.
constexpr int kLanes = 2;

int block_index(int block) {
  for (int i = 0; i < 3; ++i)
    if (kBatchBlocks[i] == block) return i;
  return -1;
}

struct Range {
  size_t off, size;
};

}  // namespace

struct lbm_batch {
  char* arena = nullptr;
  size_t bytes = 0;
  hipStream_t stream = nullptr;
  int max_slots = 0;
  size_t tab_stride = 0;   // bytes per 2-D group table
  size_t tab3_stride = 0;  // bytes per 3-D group table
  size_t tab3_off = 0;     // 3-D tables
  size_t part_off = 0;     // partials region
  size_t part_cap = 0;     // tiles it can hold
  size_t heap_off = 0;     // start of the slot heap

  struct Slot {
    int status = LBM_SLOT_FREE;
    lbm_ctx* ctx = nullptr;
    Range r{0, 0};
    double tol = 0.0;
    int64_t cap = 0;
    int scheme = LBM_WELL_BALANCED;
    lbm_observation last{};
    size_t part_index = 0;  // first tile's index in the partials region
    int tiles = 0;
  };
  std::vector<Slot> slots;
  std::vector<Range> free_ranges;  // sorted by offset, coalesced

  std::vector<std::vector<char>> host_tab;  // per group and lane
  GroupMask group_mask;                     // groups that have ever held a slot
  GroupMask active_mask[kLanes];            // per lane: groups with an active slot (launched)
  bool dirty = true;
  int graph_steps = 0;
  // per lane and parity of the two-step launches before the replay (a
  // replay of graph_steps steps makes graph_steps / 2 of them: when that is
  // odd, consecutive replays alternate between the two graphs)
  hipGraphExec_t graph[kLanes][2] = {};
  GroupMask graph_mask[kLanes][2];
  int tiles_of[kLanes][kGroups] = {};        // work items (tiles) of each table, as uploaded
  int graph_tiles[kLanes][2][kGroups] = {};  // the same when a graph was captured
  hipStream_t side = nullptr;             // the second lane's stream
  hipEvent_t fork = nullptr, join = nullptr;
  std::string err;

  lbmk::BatchTable* dev_tab(int g, int lane) const {
    return (lbmk::BatchTable*)(arena + (size_t)(g * kLanes + lane) * tab_stride);
  }
  lbmk::BatchTable3* dev_tab3(int g, int lane) const {
    return (lbmk::BatchTable3*)(arena + tab3_off + (size_t)((g - k3dBase) * kLanes + lane) * tab3_stride);
  }
  double* partials() const { return (double*)(arena + part_off); }
};

namespace {

lbm_status bfail(lbm_batch* b, lbm_status s, const std::string& msg) {
  if (b)
    b->err = msg;
  else
    g_thread_error = msg;
  return s;
}

#define BHIP(b, call)                                                                 \
  do {                                                                                \
    hipError_t e_ = (call);                                                           \
    if (e_ != hipSuccess)                                                             \
      return bfail((b), LBM_EHIP, std::string(#call) + ": " + hipGetErrorString(e_)); \
  } while (0)

int group_of(const lbm_ctx* c, int scheme) {
  if (c->d3())
    return k3dBase + ((c->storage() * 3 + scheme) * 2 + (c->L.q == lbmk::Q27 ? 1 : 0)) * 2 +
           (c->tl3.depth - 1);
  if (c->prm.force_stencil == 1)
    return kStencil4Base + (c->storage() * 3 + scheme) * 3 + (c->tl.depth - 1);
  if (fused_pairs(c))
    return kPairBase + ((c->storage() * 3 + scheme) * 2 + (c->tl.block == 256 ? 1 : 0)) * 2;
  const int bi = block_index(c->tl.block);
  return ((c->storage() * 3 + scheme) * 3 + bi) * 3 + (c->tl.depth - 1);
}

// Whether a slot's tiles are in the table of group g: its own group, and for
// a slot of two-step launches also the one-step group after it.
bool in_group(const lbm_ctx* c, int scheme, int g) {
  const int own = group_of(c, scheme);
  return g == own || (fused_pairs(c) && g == own + 1);
}

void mark_groups(lbm_batch* b, const lbm_ctx* c, int scheme) {
  const int own = group_of(c, scheme);
  b->group_mask.set(own);
  if (fused_pairs(c)) b->group_mask.set(own + 1);
}

// Launch parameters of group g; q is the 3-D velocity count (0 in 2-D).
struct Group {
  GroupKind kind;
  int storage, scheme, block, depth, q;
};

Group group_decode(int g) {
  Group d{};
  if (g >= k3dBase) {
    g -= k3dBase;
    d.kind = k3d;
    d.depth = g % 2 + 1;
    g /= 2;
    d.q = g % 2 ? lbmk::Q27 : lbmk::Q3;
    g /= 2;
    d.block = lbmk::M3X * lbmk::kBatch3Ty;
  } else if (g >= kPairBase) {
    g -= kPairBase;
    d.kind = g % 2 ? kPairOne : kPair;
    d.depth = g % 2 ? 3 : 4;
    g /= 2;
    d.block = g % 2 ? 256 : 128;
    g /= 2;
  } else if (g >= kStencil4Base) {
    g -= kStencil4Base;
    d.kind = kStencil4;
    d.depth = g % 3 + 1;
    g /= 3;
    d.block = lbmk::kBatch4Block;
  } else {
    d.kind = kMain;
    d.depth = g % 3 + 1;
    g /= 3;
    d.block = kBatchBlocks[g % 3];
    g /= 3;
  }
  d.scheme = g % 3;
  d.storage = g / 3;
  return d;
}

// Slots observed one by one at a poll (their own observe passes) rather
// than by a batched observe launch: 3-D lattices and the force-stencil
// variant.
bool polled_alone(const lbm_ctx* c) { return c->d3() || c->prm.force_stencil == 1; }

size_t part_capacity(size_t arena_bytes) { return arena_bytes / 8192 + 1024; }

void free_range(lbm_batch* b, Range r) {
  auto& v = b->free_ranges;
  auto it = std::lower_bound(v.begin(), v.end(), r.off,
                             [](const Range& a, size_t off) { return a.off < off; });
  it = v.insert(it, r);
  // coalesce with neighbours
  size_t i = it - v.begin();
  if (i + 1 < v.size() && v[i].off + v[i].size == v[i + 1].off) {
    v[i].size += v[i + 1].size;
    v.erase(v.begin() + i + 1);
  }
  if (i > 0 && v[i - 1].off + v[i - 1].size == v[i].off) {
    v[i - 1].size += v[i].size;
    v.erase(v.begin() + i);
  }
}

bool alloc_range(lbm_batch* b, size_t size, Range* out) {
  for (size_t i = 0; i < b->free_ranges.size(); ++i) {
    Range& f = b->free_ranges[i];
    if (f.size >= size) {
      *out = Range{f.off, size};
      f.off += size;
      f.size -= size;
      if (f.size == 0) b->free_ranges.erase(b->free_ranges.begin() + i);
      return true;
    }
  }
  return false;
}

// Rebuild the group tables from the active slots and upload them.
lbm_status upload_tables(lbm_batch* b) {
  size_t part = 0;
  GroupMask active[kLanes];
  for (int g = 0; g < kGroups; ++g) {
    if (!b->group_mask.test(g)) continue;
    for (int lane = 0; lane < kLanes; ++lane) {
      std::vector<char>& h = b->host_tab[g * kLanes + lane];
      std::fill(h.begin(), h.end(), 0);
      if (g >= k3dBase) {
        auto* tab = (lbmk::BatchTable3*)h.data();
        int n = 0, tiles = 0;
        for (size_t s = lane; s < b->slots.size(); s += kLanes) {
          lbm_batch::Slot& sl = b->slots[s];
          if (sl.status != LBM_SLOT_ACTIVE || group_of(sl.ctx, sl.scheme) != g) continue;
          lbm_ctx* c = sl.ctx;
          lbmk::BatchSlot3& d = tab->slot[n++];
          d.g = c->L.g3;
          d.ph = make_physics3(c->prm, sl.scheme);
          d.tl = c->tl3;
          d.buf[0] = c->buf(0);
          d.buf[1] = c->buf(1);
          d.cur = c->cur;
          d.tile0 = tiles;
          sl.part_index = 0;
          sl.tiles = (int)lbmk::blocks_of(c->tl3);
          tiles += sl.tiles;
        }
        tab->nslots = n;
        tab->total_tiles = tiles;
        if (n > 0) active[lane].set(g);
        b->tiles_of[lane][g] = tiles;
        const size_t used =
            sizeof(lbmk::BatchTable3) + (size_t)(n > 1 ? n - 1 : 0) * sizeof(lbmk::BatchSlot3);
        BHIP(b, hipMemcpyAsync(b->dev_tab3(g, lane), h.data(), used, hipMemcpyHostToDevice,
                               b->stream));
        continue;
      }
      const GroupKind kind = group_decode(g).kind;
      auto* tab = (lbmk::BatchTable*)h.data();
      int n = 0, tiles = 0;
      for (size_t s = lane; s < b->slots.size(); s += kLanes) {
        lbm_batch::Slot& sl = b->slots[s];
        if (sl.status != LBM_SLOT_ACTIVE || !in_group(sl.ctx, sl.scheme, g)) continue;
        lbm_ctx* c = sl.ctx;
        lbmk::BatchSlot& d = tab->slot[n++];
        d.g = c->L.g;
        d.ph = make_physics(c->prm, sl.scheme);
        d.tl = c->tl;
        d.buf[0] = c->buf(0);
        d.buf[1] = c->buf(1);
        d.cur = c->cur;
        d.tile0 = tiles;
        if (kind == kPair) {
          // two-step strips of BW - 6 columns; no observe records
          d.tl.strips = lbmk::step2_strips(c->L.g.nx, c->tl.block);
          d.partials = nullptr;
          tiles += d.tl.blocks();
          continue;
        }
        if (kind == kPairOne) d.tl.depth = 3;
        d.partials = b->partials() + lbmk::NPART * (part + tiles);
        sl.part_index = part + tiles;
        sl.tiles = c->tl.blocks();
        tiles += sl.tiles;
      }
      tab->nslots = n;
      tab->total_tiles = tiles;
      if (n > 0) active[lane].set(g);
      b->tiles_of[lane][g] = tiles;
      if (kind != kPair) part += tiles;
      if (part > b->part_cap)
        return bfail(b, LBM_ENOSPACE, "batch holds more tiles than its partials area");
      const size_t used =
          sizeof(lbmk::BatchTable) + (size_t)(n > 1 ? n - 1 : 0) * sizeof(lbmk::BatchSlot);
      BHIP(b, hipMemcpyAsync(b->dev_tab(g, lane), h.data(), used, hipMemcpyHostToDevice,
                             b->stream));
    }
  }
  // the host copies must stay intact until the uploads have been consumed
  BHIP(b, hipStreamSynchronize(b->stream));
  std::copy(active, active + kLanes, b->active_mask);
  b->dirty = false;
  return LBM_OK;
}

// `steps` steps of one lane's groups on stream s.  Slots of two-step launches
// get one launch at every even step with a step after it and a one-step
// launch for the last step of an odd count; `pair0` is the parity of the
// two-step launches made since the tables were uploaded (their buffers swap
// once per launch).
lbm_status batch_launches(lbm_batch* b, int lane, int steps, hipStream_t s, int pair0) {
  for (int j = 0; j < steps; ++j) {
    for (int g = 0; g < kGroups; ++g) {
      if (!b->active_mask[lane].test(g)) continue;
      const Group d = group_decode(g);
      const int tiles = b->tiles_of[lane][g];
      if (d.kind == kPair || d.kind == kPairOne) {
        const int par = ((j >> 1) + pair0) & 1;
        if (d.kind == kPair && (j & 1) == 0 && j + 1 < steps)
          BHIP(b, lbmk::launch_batch2(d.storage, d.scheme, d.block, b->dev_tab(g, lane), tiles, par,
                                      s));
        else if (d.kind == kPairOne && (steps & 1) && j == steps - 1)
          BHIP(b, lbmk::launch_batch(d.storage, d.scheme, d.block, d.depth, false,
                                     b->dev_tab(g, lane), tiles, par, s));
      } else if (d.kind == k3d)
        BHIP(b, lbmk::launch_batch3(d.storage, d.scheme, d.q, d.depth, b->dev_tab3(g, lane), tiles,
                                    j & 1, s));
      else if (d.kind == kStencil4)
        BHIP(b, lbmk::launch_batch4(d.storage, d.scheme, d.depth, b->dev_tab(g, lane), tiles,
                                    j & 1, s));
      else
        BHIP(b, lbmk::launch_batch(d.storage, d.scheme, d.block, d.depth, false,
                                   b->dev_tab(g, lane), tiles, j & 1, s));
    }
  }
  return LBM_OK;
}

void drop_batch_graph(lbm_batch* b) {
  for (auto& lane : b->graph)
    for (auto& g : lane)
      if (g) {
        (void)hipGraphExecDestroy(g);
        g = nullptr;
      }
}

// Whether a lane launches slots of two-step launches.
bool lane_pairs(const lbm_batch* b, int lane) {
  for (int g = kPairBase; g < k3dBase; g += 2)
    if (b->active_mask[lane].test(g)) return true;
  return false;
}

lbm_status batch_graph(lbm_batch* b, int lane, int pair0, hipGraphExec_t* out) {
  // a captured launch holds its group's grid (one block per tile), so a
  // lane's graph is re-captured when its launched groups or their tile
  // counts change
  hipGraphExec_t& ge = b->graph[lane][pair0];
  if (ge && b->graph_mask[lane][pair0] == b->active_mask[lane] &&
      std::equal(b->tiles_of[lane], b->tiles_of[lane] + kGroups, b->graph_tiles[lane][pair0])) {
    *out = ge;
    return LBM_OK;
  }
  if (ge) {
    (void)hipGraphExecDestroy(ge);
    ge = nullptr;
  }
  hipStream_t cs;
  BHIP(b, hipStreamCreateWithFlags(&cs, hipStreamNonBlocking));
  hipError_t e = hipStreamBeginCapture(cs, hipStreamCaptureModeRelaxed);
  if (e != hipSuccess) {
    (void)hipStreamDestroy(cs);
    return bfail(b, LBM_EHIP, std::string("hipStreamBeginCapture: ") + hipGetErrorString(e));
  }
  lbm_status st = batch_launches(b, lane, b->graph_steps, cs, pair0);
  hipGraph_t graph = nullptr;
  e = hipStreamEndCapture(cs, &graph);
  (void)hipStreamDestroy(cs);
  if (st != LBM_OK) {
    if (graph) (void)hipGraphDestroy(graph);
    return st;
  }
  if (e != hipSuccess)
    return bfail(b, LBM_EHIP, std::string("hipStreamEndCapture: ") + hipGetErrorString(e));
  e = hipGraphInstantiate(&ge, graph, nullptr, nullptr, 0);
  (void)hipGraphDestroy(graph);
  if (e != hipSuccess) {
    ge = nullptr;
    return bfail(b, LBM_EHIP, std::string("hipGraphInstantiate: ") + hipGetErrorString(e));
  }
  b->graph_mask[lane][pair0] = b->active_mask[lane];
  std::copy(b->tiles_of[lane], b->tiles_of[lane] + kGroups, b->graph_tiles[lane][pair0]);
  *out = ge;
  return LBM_OK;
}

lbm_batch::Slot* slot_of(lbm_batch* b, int32_t slot) {
  if (!b || slot < 0 || slot >= (int32_t)b->slots.size()) return nullptr;
  lbm_batch::Slot* s = &b->slots[slot];
  return s->status == LBM_SLOT_FREE ? nullptr : s;
}

}  // namespace

extern "C" {

size_t lbm_batch_slot_bytes(const lbm_params* p) {
  return align_up(lbm_workspace_bytes(p), ALIGN);
}

size_t lbm_batch_overhead_bytes(size_t arena_bytes, int32_t max_slots) {
  if (max_slots < 1) return 0;
  const size_t stride = align_up(lbmk::batch_table_bytes(max_slots), ALIGN);
  const size_t stride3 = align_up(lbmk::batch_table3_bytes(max_slots), ALIGN);
  return (size_t)k3dBase * kLanes * stride + (size_t)(kGroups - k3dBase) * kLanes * stride3 +
         align_up(part_capacity(arena_bytes) * lbmk::NPART * sizeof(double), ALIGN);
}

lbm_status lbm_batch_create(void* arena, size_t bytes, int32_t max_slots, void* stream,
                            lbm_batch** out) {
  if (!out) return bfail(nullptr, LBM_EINVAL, "out is NULL");
  *out = nullptr;
  if (!arena) return bfail(nullptr, LBM_EINVAL, "arena is NULL");
  if ((uintptr_t)arena % ALIGN) return bfail(nullptr, LBM_EINVAL, "arena not 256-byte aligned");
  if (max_slots < 1 || max_slots > 65536) return bfail(nullptr, LBM_EINVAL, "max_slots out of range");
  const size_t over = lbm_batch_overhead_bytes(bytes, max_slots);
  if (bytes <= over) return bfail(nullptr, LBM_ENOSPACE, "arena smaller than the batch tables");
  hipStream_t side = nullptr;
  hipEvent_t fork = nullptr, join = nullptr;
  hipError_t e = hipStreamCreateWithFlags(&side, hipStreamNonBlocking);
  if (e == hipSuccess) e = hipEventCreateWithFlags(&fork, hipEventDisableTiming);
  if (e == hipSuccess) e = hipEventCreateWithFlags(&join, hipEventDisableTiming);
  if (e != hipSuccess) {
    if (join) (void)hipEventDestroy(join);
    if (fork) (void)hipEventDestroy(fork);
    if (side) (void)hipStreamDestroy(side);
    return bfail(nullptr, LBM_EHIP, std::string("batch stream: ") + hipGetErrorString(e));
  }
  lbm_batch* b = new lbm_batch();
  b->arena = (char*)arena;
  b->bytes = bytes;
  b->stream = (hipStream_t)stream;
  b->side = side;
  b->fork = fork;
  b->join = join;
  b->max_slots = max_slots;
  b->tab_stride = align_up(lbmk::batch_table_bytes(max_slots), ALIGN);
  b->tab3_stride = align_up(lbmk::batch_table3_bytes(max_slots), ALIGN);
  b->tab3_off = (size_t)k3dBase * kLanes * b->tab_stride;
  b->part_off = b->tab3_off + (size_t)(kGroups - k3dBase) * kLanes * b->tab3_stride;
  b->part_cap = part_capacity(bytes);
  b->heap_off = over;
  b->slots.resize(max_slots);
  b->free_ranges.push_back(Range{b->heap_off, bytes - b->heap_off});
  b->host_tab.resize(kGroups * kLanes);
  for (int g = 0; g < kGroups; ++g)
    for (int lane = 0; lane < kLanes; ++lane)
      b->host_tab[g * kLanes + lane].assign(
          g >= k3dBase ? lbmk::batch_table3_bytes(max_slots) : lbmk::batch_table_bytes(max_slots), 0);
  *out = b;
  return LBM_OK;
}

lbm_status lbm_batch_admit(lbm_batch* b, const lbm_params* p, const double* rho, lbm_scheme scheme,
                           double tol, int64_t cap, int32_t* slot) {
  if (!b) return bfail(nullptr, LBM_EINVAL, "batch is NULL");
  if (!slot || !rho) return bfail(b, LBM_EINVAL, "slot and rho must not be NULL");
  if (!valid_scheme(scheme)) return bfail(b, LBM_EINVAL, "unknown scheme");
  std::string why;
  if (!valid_params(p, &why)) return bfail(b, LBM_EINVAL, why);
  int idx = -1;
  for (int i = 0; i < b->max_slots; ++i)
    if (b->slots[i].status == LBM_SLOT_FREE) {
      idx = i;
      break;
    }
  if (idx < 0) return bfail(b, LBM_EBUSY, "no free slot");
  const size_t need = lbm_batch_slot_bytes(p);
  Range r;
  if (!alloc_range(b, need, &r)) return bfail(b, LBM_EBUSY, "no arena range of " + std::to_string(need) + " bytes");
  lbm_ctx* c = nullptr;
  lbm_status st = lbm_create(p, b->arena + r.off, need, b->stream, &c);
  if (st != LBM_OK) {
    free_range(b, r);
    return bfail(b, st, lbm_last_error(nullptr));
  }
  // default tile of a 2-D slot (callers normally set a tuned one): block
  // width by lattice width, 32-row chunks, two rows in flight; the
  // force-stencil variant runs 256-wide blocks.  A 3-D slot keeps the
  // single lattice's default tiling (32 x 8 tiles, one or two planes in
  // flight), which batches run.
  if (!c->d3()) {
    const int block =
        p->force_stencil == 1 ? lbmk::kBatch4Block : (p->nx <= 64 ? 64 : (p->nx <= 128 ? 128 : 256));
    c->tl = make_tiling(c->L.g, block, 32, 2);
  }
  st = lbm_init(c, rho, nullptr, nullptr, scheme);
  if (st != LBM_OK) {
    std::string m = c->err;
    lbm_destroy(c);
    free_range(b, r);
    return bfail(b, st, m);
  }
  lbm_batch::Slot& s = b->slots[idx];
  s = lbm_batch::Slot();
  s.status = LBM_SLOT_ACTIVE;
  s.ctx = c;
  s.r = r;
  s.tol = tol;
  s.cap = cap;
  s.scheme = scheme;
  mark_groups(b, c, scheme);
  b->dirty = true;
  *slot = idx;
  return LBM_OK;
}

lbm_status lbm_batch_set_tile(lbm_batch* b, int32_t slot, int32_t block, int32_t rows, int32_t depth) {
  lbm_batch::Slot* s = slot_of(b, slot);
  if (!s) return bfail(b, LBM_EINVAL, "no such slot");
  const lbm_ctx* c = s->ctx;
  if (depth == 4) {
    // two steps per launch: the single lattice's rule
    if (c->d3() || c->prm.force_stencil == 1 ||
        !lbmk::step2_block_supported(block ? block : c->tl.block))
      return bfail(b, LBM_EINVAL,
                   "batch depth 4 (two steps per launch) needs a 2-D slot with the central "
                   "stencil and block 128 or 256");
  } else {
    if (block != 0 && block_index(block) < 0)
      return bfail(b, LBM_EINVAL, "batch block width must be 64, 128 or 256");
    if (block != 0 && c->prm.force_stencil == 1 && block != lbmk::kBatch4Block)
      return bfail(b, LBM_EINVAL, "force-stencil slots run 256-wide blocks");
    if (c->d3() && ((block != 0 && block != lbmk::M3X * lbmk::kBatch3Ty) || depth > 2))
      return bfail(b, LBM_EINVAL, "3-D slots run 256-thread tiles (32 x 8) with depth 1 or 2");
    if (depth < 0 || depth > 3) return bfail(b, LBM_EINVAL, "batch depth must be 1, 2, 3 or 4");
  }
  lbm_status st = lbm_set_tile(s->ctx, block, rows, depth);
  if (st != LBM_OK) return bfail(b, st, s->ctx->err);
  mark_groups(b, s->ctx, s->scheme);
  b->dirty = true;
  return LBM_OK;
}

lbm_status lbm_batch_set_graph_steps(lbm_batch* b, int32_t steps) {
  if (!b) return bfail(nullptr, LBM_EINVAL, "batch is NULL");
  if (steps < 0 || steps > 4096 || (steps >= 2 && (steps & 1)))
    return bfail(b, LBM_EINVAL, "graph steps must be even and in [0, 4096]");
  drop_batch_graph(b);
  b->graph_steps = steps;
  return LBM_OK;
}

lbm_status lbm_batch_run(lbm_batch* b, int32_t k) {
  if (!b) return bfail(nullptr, LBM_EINVAL, "batch is NULL");
  if (k < 0) return bfail(b, LBM_EINVAL, "k must be >= 0");
  if (k == 0) return LBM_OK;
  if (b->dirty) {
    lbm_status st = upload_tables(b);
    if (st != LBM_OK) return st;
  }
  // lane 0 on the caller's stream, lane 1 on the side stream after the work
  // already queued on the caller's; the caller's stream then waits for both
  BHIP(b, hipEventRecord(b->fork, b->stream));
  BHIP(b, hipStreamWaitEvent(b->side, b->fork, 0));
  for (int lane = 0; lane < kLanes; ++lane) {
    if (b->active_mask[lane].none()) continue;
    hipStream_t ls = lane == 0 ? b->stream : b->side;
    int left = k;
    int pair0 = 0;
    if (b->graph_steps >= 2) {
      const int flip = lane_pairs(b, lane) ? (b->graph_steps / 2) & 1 : 0;
      while (left >= b->graph_steps) {
        hipGraphExec_t ge;
        lbm_status st = batch_graph(b, lane, pair0, &ge);
        if (st != LBM_OK) return st;
        BHIP(b, hipGraphLaunch(ge, ls));
        left -= b->graph_steps;
        pair0 ^= flip;
      }
    }
    lbm_status st = batch_launches(b, lane, left, ls, pair0);
    if (st != LBM_OK) return st;
  }
  BHIP(b, hipEventRecord(b->join, b->side));
  BHIP(b, hipStreamWaitEvent(b->stream, b->join, 0));
  // launches per slot: k, or k / 2 two-step launches and one more for an odd
  // k; each swaps the slot's buffers
  const int pair_launches = k / 2 + (k & 1);
  for (auto& s : b->slots) {
    if (s.status != LBM_SLOT_ACTIVE) continue;
    s.ctx->step += k;
    if ((fused_pairs(s.ctx) ? pair_launches : k) & 1) {
      s.ctx->cur ^= 1;
      b->dirty = true;
    }
  }
  return LBM_OK;
}

lbm_status lbm_batch_poll(lbm_batch* b, int32_t* retired, int32_t cap, int32_t* n_retired) {
  if (!b) return bfail(nullptr, LBM_EINVAL, "batch is NULL");
  if (n_retired) *n_retired = 0;
  if (b->dirty) {
    lbm_status st = upload_tables(b);
    if (st != LBM_OK) return st;
  }
  // partial records of the slots observed by batched launches
  size_t total = 0;
  for (const auto& s : b->slots)
    if (s.status == LBM_SLOT_ACTIVE && !polled_alone(s.ctx))
      total = std::max(total, s.part_index + s.tiles);
  std::vector<double> part(total * lbmk::NPART);
  if (total > 0) {
    for (int lane = 0; lane < kLanes; ++lane)
      for (int g = 0; g < k3dBase; ++g) {
        if (!b->active_mask[lane].test(g)) continue;
        const Group d = group_decode(g);
        if (d.kind != kMain && d.kind != kPairOne) continue;
        BHIP(b, lbmk::launch_batch(d.storage, d.scheme, d.block, d.depth, true,
                                   b->dev_tab(g, lane), b->tiles_of[lane][g], 0, b->stream));
      }
    BHIP(b, hipMemcpyAsync(part.data(), b->partials(), part.size() * sizeof(double),
                           hipMemcpyDeviceToHost, b->stream));
    BHIP(b, hipStreamSynchronize(b->stream));
  }
  int n = 0;
  bool changed = false;
  for (size_t i = 0; i < b->slots.size(); ++i) {
    lbm_batch::Slot& s = b->slots[i];
    if (s.status != LBM_SLOT_ACTIVE) continue;
    bool bad;
    if (polled_alone(s.ctx)) {
      // the observe pass of a 3-D lattice or of the force-stencil variant
      // (three launches into the slot's own staging and partials), as
      // lbm_observe on the slot alone
      const lbm_status os = observe_impl(s.ctx, nullptr, nullptr, nullptr, nullptr, nullptr, &s.last);
      if (os != LBM_OK && os != LBM_ENONFINITE) return bfail(b, os, s.ctx->err);
      bad = os == LBM_ENONFINITE;
    } else {
      bad = finish_partials(&part[lbmk::NPART * s.part_index], (size_t)s.tiles, s.ctx->step,
                            &s.last);
    }
    const double umax = s.last.max_u;
    int st = LBM_SLOT_ACTIVE;
    if (bad)
      st = LBM_SLOT_DIVERGED;
    else if (s.tol > 0.0 && umax < s.tol)
      st = LBM_SLOT_CONVERGED;
    else if (s.cap > 0 && s.ctx->step >= s.cap)
      st = LBM_SLOT_CAPPED;
    if (st != LBM_SLOT_ACTIVE) {
      s.status = st;
      changed = true;
      if (retired && n < cap) retired[n] = (int32_t)i;
      ++n;
    }
  }
  if (n_retired) *n_retired = std::min(n, std::max(cap, 0));
  if (changed) b->dirty = true;
  return LBM_OK;
}

lbm_status lbm_batch_slot_info(const lbm_batch* b, int32_t slot, int32_t* status,
                               lbm_observation* obs) {
  if (!b || slot < 0 || slot >= (int32_t)b->slots.size())
    return bfail(const_cast<lbm_batch*>(b), LBM_EINVAL, "no such slot");
  const lbm_batch::Slot& s = b->slots[slot];
  if (status) *status = s.status;
  if (obs) *obs = s.last;
  return LBM_OK;
}

lbm_status lbm_batch_fetch(lbm_batch* b, int32_t slot, double* rho, double* ux, double* uy,
                           double* mu, lbm_observation* obs) {
  lbm_batch::Slot* s = slot_of(b, slot);
  if (!s) return bfail(b, LBM_EINVAL, "no such slot");
  lbm_status st = lbm_observe(s->ctx, rho, ux, uy, mu, obs);
  if (st != LBM_OK && st != LBM_ENONFINITE) return bfail(b, st, s->ctx->err);
  if (obs) s->last = *obs;
  return st;
}

lbm_status lbm_batch_get_populations(lbm_batch* b, int32_t slot, double* f) {
  lbm_batch::Slot* s = slot_of(b, slot);
  if (!s) return bfail(b, LBM_EINVAL, "no such slot");
  lbm_status st = lbm_get_populations(s->ctx, f);
  return st == LBM_OK ? st : bfail(b, st, s->ctx->err);
}

lbm_status lbm_batch_release(lbm_batch* b, int32_t slot) {
  lbm_batch::Slot* s = slot_of(b, slot);
  if (!s) return bfail(b, LBM_EINVAL, "no such slot");
  // work already enqueued on the stream may still use the slot's memory
  BHIP(b, hipStreamSynchronize(b->stream));
  lbm_destroy(s->ctx);
  free_range(b, s->r);
  *s = lbm_batch::Slot();
  b->dirty = true;
  return LBM_OK;
}

lbm_status lbm_batch_destroy(lbm_batch* b) {
  if (!b) return LBM_OK;
  (void)hipStreamSynchronize(b->stream);
  (void)hipStreamSynchronize(b->side);
  drop_batch_graph(b);
  for (auto& s : b->slots)
    if (s.ctx) lbm_destroy(s.ctx);
  (void)hipEventDestroy(b->join);
  (void)hipEventDestroy(b->fork);
  (void)hipStreamDestroy(b->side);
  delete b;
  return LBM_OK;
}

const char* lbm_batch_last_error(const lbm_batch* b) {
  return b ? b->err.c_str() : g_thread_error.c_str();
}

}  // extern "C"
