// Host orchestration behind the C ABI of include/tufrg.h: context set-up,
// argument checks, the right-hand-side pipeline and the flow integrators.
//
// Right-hand side at scale Lambda (one evaluation, all on the context stream):
//   kval      regulator K(e_m(k)) for every band and fine k
//   loop      compact loops of both channels (partials per k-chunk)
//   finalize  fixed-order FP64 sum of the partials, hermitian completion
//   ft        P(q), C(q) -> P(rho), C(rho) for rho in D = S - S
//   gather    rho-space gathers of the four cross projections
//   assemble  VP(q), VC(q)
//   bundle    dP = VP Lpp VP, dC = 2 VC Lph VC
#include <algorithm>
#include <cmath>
#include <cstdio>
#include <cstring>
#include <map>
#include <mutex>
#include <string>
#include <utility>
#include <vector>

#include "../../include/tufrg.h"
#include "common.h"
#include "kernels.h"
#include "tune_cache.h"

namespace tufrg {
hipError_t launch_unpack_pi(int n_o, int Nf, const double *pi, double *out, hipStream_t st);
}

using namespace tufrg;

namespace tufrg {
tufrg_status mlp_forward_internal(tufrg_mlp *m, long long n, const float *X, float *Y);
int mlp_n_in(const tufrg_mlp *m);
int mlp_n_out(const tufrg_mlp *m);
hipStream_t mlp_stream(const tufrg_mlp *m);
}  // namespace tufrg

struct tufrg_ctx {
  hipStream_t st = nullptr;
  int device = 0;  // the device current at creation
  int n_o = 0, n_ff = 0, B = 0, Lq = 0, n_ref = 0, Lf = 0, Nq = 0, Nf = 0, no2 = 0, no4 = 0;
  int nD = 0, ndx = 0, ndy = 0, scheme = 0, prec = 0, nkyb = 0, nkxc = 0;
  size_t proj_ws = 0;  // doubles of the projection workspace (whole qx rows of the intermediate)
  std::vector<int> ff, dlist, didx, ffgrid, dgrid, pairs;
  int *d_ff = nullptr, *d_dlist = nullptr, *d_didx = nullptr, *d_ffgrid = nullptr, *d_dgrid = nullptr;
  int *d_hopR = nullptr;
  int *d_pairs = nullptr;  // loop entry pairs (tau, conjugate partner) for more than two orbitals
  int n_pairs = 0;
  double *d_ekv64 = nullptr, *d_pi4_64 = nullptr;  // two orbitals: k-major 4-vectors of the loop kernel
  float *d_ekv32 = nullptr, *d_pi4_32 = nullptr;
  double *d_phy64 = nullptr;  // ky phases of the multi-orbital loop kernel, [Lf][ndy][2]
  float *d_phy32 = nullptr;
  double *d_hopt = nullptr;
  double *d_band64 = nullptr;
  float *d_band32 = nullptr;
  double *d_bandk64 = nullptr;  // k-major copies for more than two orbitals
  float *d_bandk32 = nullptr;
  double *d_kv64 = nullptr;
  float *d_kv32 = nullptr;
  double *d_c0 = nullptr;     // static C-channel term of a non-local initial interaction, [Nq][B][B]
  double *d_ceff = nullptr;   // C + C0 for the projections
  bool has_c0 = false;
  double *d_p0 = nullptr;     // static P-channel term of the bare vertex (band basis), [Nq][B][B]
  double *d_peff = nullptr;   // P + P0 for the projections
  bool has_p0 = false;
  double temp = 0.0;          // momentum-shell scheme: the fixed temperature of its bubbles
  double *d_cv64 = nullptr;   // momentum-shell scheme: shell factors (see LoopArgs::cv)
  float *d_cv32 = nullptr;
  double *d_twf = nullptr, *d_twq = nullptr;
  // projections: phases of the distinct rho_y over D per qy, and per rho of D
  // (rho_x mod Lq) | slot of rho_y << 16
  double *d_pphy = nullptr;
  int *d_dtab = nullptr;
  int ny = 0;
  // SU(2)-reduced flows (one orbital): index of -R per form factor, and the
  // workspaces (p^x, rho-space coefficients, gathers, d~ and a~^x, the d update)
  int *d_fneg = nullptr;
  double *d_s_px = nullptr, *d_s_rA = nullptr, *d_s_rB = nullptr, *d_s_G3 = nullptr, *d_s_Vd = nullptr,
         *d_s_Vax = nullptr, *d_s_dd = nullptr;
  float *d_twf32 = nullptr;
  double *d_partial = nullptr;
  double *d_loop = nullptr;
  double *d_ftpart = nullptr, *d_real = nullptr, *d_G = nullptr;
  double *d_v0p = nullptr, *d_v0c = nullptr, *d_VP = nullptr, *d_VC = nullptr;
  unsigned long long *d_bits = nullptr;
  unsigned int *d_flag = nullptr;
  unsigned long long *h_bits = nullptr;  // pinned
  unsigned int *h_flag = nullptr;        // pinned
  // flow workspace (lazy)
  double *d_dP = nullptr, *d_dC = nullptr;
  double *d_btmp = nullptr;  // bundle workspace for B > 64 (BF16X3: split planes)
  size_t btmp_bytes = 0;
  double *d_basis_tmp = nullptr;  // basis sandwich workspace, [Nq][B][B] complex (lazy)
  double *d_basis_c = nullptr;    // compact basis matrix, [Nq][nD][n_o^4] complex (lazy)
  double *d_basis_rows = nullptr; // its kx-row sums for a chunk of coarse q (lazy)
  double *d_ffA = nullptr;        // form-factor change matrix, at most 25 x 25 complex (lazy)
  std::vector<double *> d_stage;  // DP5: 7 k's per channel + stage state per channel
  std::string err;
  std::vector<void *> allocs;
  // optional per-kernel timing with HIP events on the context stream
  struct Timer {
    std::vector<hipEvent_t> ev;
    size_t used = 0;
    double ms = 0.0;
    int count = 0;
  };
  bool timing = false;
  Timer timers[TUFRG_TIMER_COUNT];
  // loop surrogate
  tufrg_mlp *sur = nullptr;
  std::vector<double> sur_lnlam, sur_lns;  // target scale table, ln Lambda ascending -> ln s
  float *d_surX = nullptr, *d_surY = nullptr;  // features of all blocks, network rows of a chunk
  double *d_samp = nullptr;                    // plain loops of sampled q_x rows, [row][2][Lq][nD][no4]
  int samp_rows = 0;
  unsigned long long *d_sbits = nullptr;       // max |diff|, max |ref|, float max
  int *d_rows = nullptr, *h_rows = nullptr;    // sampled q_x rows (device, pinned host)
  float *d_yrow = nullptr;                     // BF16X3 loops: row buffers of a chunk of coarse q
  double *d_lamb = nullptr;                    // BF16X3 loops: real-basis sums of a chunk
  int *d_hmap = nullptr;                       // BF16X3 loops: half-plane point of each difference vector
  int mfma_chunk = 0;
  int mfma_kxr = 1;        // kx rows per work item of the matrix-core loop (tunable)
  void *d_apre = nullptr;  // the matrix-core loop's precomputed A operand (once per context)
  int apre_pair = 0;       // the pairing d_apre was computed for
  // BF16X3 loops: bands (0,1), (2,3), (4,5) degenerate at every k (Kramers
  // pairs), found at creation; then the loops sum them by pairs unless
  // pair_enable is cleared
  int bands_paired = 0, pair_enable = 1;
  float *d_pir32 = nullptr;   // [Nf][3][36] pair sums of the packed projectors (FP32, BF16X3)
  double *d_pir64 = nullptr;  // the same in FP64
  size_t partial_cap = 0;  // doubles allocated at d_partial
  unsigned long long *h_sbits = nullptr;       // pinned
  // Euler steps in HIP graphs: the executable graph, the capture stream (the
  // context's stream, or a private one when that is the null stream), one
  // max-coupling slot per step of a graph, and the state at a graph's start
  hipGraphExec_t gexec = nullptr;
  hipStream_t gst = nullptr;
  bool own_gst = false;
  unsigned long long *d_gbits = nullptr, *h_gbits = nullptr;  // h_: pinned
  unsigned int *d_gflag = nullptr, *h_gflag = nullptr;
  double *d_bkP = nullptr, *d_bkC = nullptr;
  // set during tufrg_flow
  const tufrg_flow_opts *fopts = nullptr;
  tufrg_flow_result *fres = nullptr;
  double cur_max = 0.0;
};

static thread_local std::string g_err;

static tufrg_status fail(tufrg_ctx *c, tufrg_status s, const std::string &m) {
  if (c)
    c->err = m;
  else
    g_err = m;
  return s;
}

#define HIPCHK(ctx, call)                                                                   \
  do {                                                                                      \
    hipError_t e_ = (call);                                                                 \
    if (e_ != hipSuccess) {                                                                 \
      (void)hipGetLastError();                                                              \
      return fail(ctx, TUFRG_E_HIP, std::string(#call) + ": " + hipGetErrorString(e_));      \
    }                                                                                       \
  } while (0)

template <typename T>
static tufrg_status dalloc(tufrg_ctx *c, T **p, size_t n) {
  void *v = nullptr;
  hipError_t e = hipMalloc(&v, std::max<size_t>(n, 1) * sizeof(T));
  if (e != hipSuccess) {
    (void)hipGetLastError();
    return fail(c, TUFRG_E_NOMEM, std::string("hipMalloc failed: ") + hipGetErrorString(e));
  }
  c->allocs.push_back(v);
  *p = (T *)v;
  return TUFRG_OK;
}

#define TRY(x)                         \
  do {                                 \
    tufrg_status s_ = (x);             \
    if (s_ != TUFRG_OK) return s_;     \
  } while (0)

// Static scratch of tufrg_project_static: the rho-space buffers of the
// projections (chunk partials of the q -> rho transform, the coefficients
// P(rho), C(rho) and the gathers) for callers that cannot allocate.  Each GPU
// holds its own copy until the process ends; host code reaches it only through
// the device address looked up once per device (g_scratch_ptr), never through
// the array's name.
static constexpr size_t STATIC_SCRATCH_DOUBLES = (size_t)4 << 20;  // 32 MiB
static __device__ __align__(256) double scratch[STATIC_SCRATCH_DOUBLES];
static constexpr int MAX_DEVICES = 64;
static std::mutex g_scratch_mu;
static double *g_scratch_ptr[MAX_DEVICES];

// device address of the static scratch on the current device (looked up on
// the first call per device)
static hipError_t static_scratch_lookup(int dev) {
  if (dev < 0 || dev >= MAX_DEVICES) return hipErrorInvalidDevice;
  std::lock_guard<std::mutex> lock(g_scratch_mu);
  if (g_scratch_ptr[dev]) return hipSuccess;
  void *ptr = nullptr;
  hipError_t e = hipGetSymbolAddress(&ptr, HIP_SYMBOL(scratch));
  if (e != hipSuccess) return e;
  g_scratch_ptr[dev] = (double *)ptr;
  return hipSuccess;
}

static bool is_device_ptr(const void *p) {
  if (!p) return false;
  hipPointerAttribute_t a;
  hipError_t e = hipPointerGetAttributes(&a, p);
  if (e != hipSuccess) {
    (void)hipGetLastError();
    return false;
  }
  return a.type == hipMemoryTypeDevice || a.type == hipMemoryTypeManaged;
}

static hipError_t timer_mark(tufrg_ctx *c, int id) {
  if (!c->timing) return hipSuccess;
  auto &t = c->timers[id];
  if (t.used == t.ev.size()) {
    hipEvent_t e;
    hipError_t r = hipEventCreate(&e);
    if (r != hipSuccess) return r;
    t.ev.push_back(e);
  }
  return hipEventRecord(t.ev[t.used++], c->st);
}

static void destroy_all(tufrg_ctx *c) {
  if (c->gexec) (void)hipGraphExecDestroy(c->gexec);
  c->gexec = nullptr;
  if (c->own_gst && c->gst) (void)hipStreamDestroy(c->gst);
  c->gst = nullptr;
  if (c->h_gbits) (void)hipHostFree(c->h_gbits);
  if (c->h_gflag) (void)hipHostFree(c->h_gflag);
  c->h_gbits = nullptr;
  c->h_gflag = nullptr;
  for (auto &t : c->timers)
    for (hipEvent_t e : t.ev) (void)hipEventDestroy(e);
  for (void *p : c->allocs) (void)hipFree(p);
  c->allocs.clear();
  if (c->h_bits) (void)hipHostFree(c->h_bits);
  if (c->h_flag) (void)hipHostFree(c->h_flag);
  if (c->h_sbits) (void)hipHostFree(c->h_sbits);
  if (c->h_rows) (void)hipHostFree(c->h_rows);
  c->h_rows = nullptr;
  c->h_bits = nullptr;
  c->h_flag = nullptr;
  c->h_sbits = nullptr;
}

extern "C" const char *tufrg_last_error(const tufrg_ctx *ctx) { return ctx ? ctx->err.c_str() : g_err.c_str(); }

extern "C" tufrg_status tufrg_create(const tufrg_model *m, const tufrg_setup *s, void *stream, tufrg_ctx **out) {
  if (!m || !s || !out) return fail(nullptr, TUFRG_E_INVAL, "null argument");
  *out = nullptr;
  if (m->n_orb != 1 && m->n_orb != 2 && m->n_orb != 6)
    return fail(nullptr, TUFRG_E_UNSUPPORTED,
                "the library supports n_orb = 2 or 6 spin-orbitals, or 1 orbital (SU(2)-reduced flows)");
  if (m->n_hop < 1 || !m->hop_R || !m->hop_t || !m->V0) return fail(nullptr, TUFRG_E_INVAL, "empty model");
  if (s->n_ff < 1 || !s->ff_R) return fail(nullptr, TUFRG_E_INVAL, "empty form-factor set");
  if (s->ff_R[0] != 0 || s->ff_R[1] != 0) return fail(nullptr, TUFRG_E_INVAL, "ff_R[0] must be (0,0)");
  if (s->cutoff != TUFRG_CUT_TEMPERATURE && s->cutoff != TUFRG_CUT_OMEGA && s->cutoff != TUFRG_CUT_SHELL)
    return fail(nullptr, TUFRG_E_INVAL, "unknown cutoff");
  if (s->cutoff == TUFRG_CUT_SHELL && !(s->temperature > 0.0 && std::isfinite(s->temperature)))
    return fail(nullptr, TUFRG_E_INVAL, "the momentum-shell cutoff needs a temperature > 0");
  if (s->precision != TUFRG_FP64 && s->precision != TUFRG_FP32 && s->precision != TUFRG_BF16X3)
    return fail(nullptr, TUFRG_E_INVAL, "unknown precision");
  if (s->precision == TUFRG_BF16X3 && m->n_orb != 6)
    return fail(nullptr, TUFRG_E_UNSUPPORTED, "BF16X3 loops are built for six spin-orbitals");
  if (s->n_ref < 1 || s->Lq < 1 || (long long)s->Lq * s->n_ref > 4096)
    return fail(nullptr, TUFRG_E_INVAL, "mesh sizes out of range");
  if (s->basis != TUFRG_BASIS_ORBITAL && s->basis != TUFRG_BASIS_BAND)
    return fail(nullptr, TUFRG_E_INVAL, "unknown single-particle basis");
  if (m->n_orb == 1 && (s->precision != TUFRG_FP64 || s->cutoff == TUFRG_CUT_SHELL || s->basis != TUFRG_BASIS_ORBITAL))
    return fail(nullptr, TUFRG_E_UNSUPPORTED,
                "the SU(2)-reduced path runs FP64 with the temperature or Omega cutoff in the orbital basis");
  int rmax = 0;
  std::vector<std::pair<int, int>> ffv;
  for (int i = 0; i < s->n_ff; ++i) {
    int x = s->ff_R[2 * i], y = s->ff_R[2 * i + 1];
    if (std::abs(x) > 2 || std::abs(y) > 2) return fail(nullptr, TUFRG_E_INVAL, "form factor beyond |R| <= 2");
    rmax = std::max(rmax, std::max(std::abs(x), std::abs(y)));
    for (auto &p : ffv)
      if (p.first == x && p.second == y) return fail(nullptr, TUFRG_E_INVAL, "duplicate form factor");
    ffv.push_back({x, y});
  }
  for (auto &p : ffv) {
    bool found = false;
    for (auto &q : ffv) found |= (q.first == -p.first && q.second == -p.second);
    if (!found) return fail(nullptr, TUFRG_E_INVAL, "form-factor set not closed under R -> -R");
  }
  if (s->Lq <= 4 * rmax) return fail(nullptr, TUFRG_E_INVAL, "Lq must exceed 4 max|R| (aliasing)");

  tufrg_ctx *c = new tufrg_ctx();
  c->st = (hipStream_t)stream;
  c->n_o = m->n_orb;
  c->no2 = c->n_o * c->n_o;
  c->no4 = c->no2 * c->no2;
  c->n_ff = s->n_ff;
  c->B = c->n_ff * c->no2;
  c->Lq = s->Lq;
  c->n_ref = s->n_ref;
  c->Lf = s->Lq * s->n_ref;
  c->Nq = c->Lq * c->Lq;
  c->Nf = c->Lf * c->Lf;
  c->scheme = s->cutoff;
  c->temp = s->cutoff == TUFRG_CUT_SHELL ? s->temperature : 0.0;
  c->prec = s->precision;
  c->ff.assign(s->ff_R, s->ff_R + 2 * s->n_ff);
  // D = S - S, sorted; lookup grids over [-8, 8]^2
  std::map<std::pair<int, int>, int> dmap;
  for (int i = 0; i < c->n_ff; ++i)
    for (int j = 0; j < c->n_ff; ++j) dmap[{c->ff[2 * i] - c->ff[2 * j], c->ff[2 * i + 1] - c->ff[2 * j + 1]}] = 0;
  int idx = 0, mdx = 0, mdy = 0;
  for (auto &kv : dmap) {
    kv.second = idx++;
    c->dlist.push_back(kv.first.first);
    c->dlist.push_back(kv.first.second);
    mdx = std::max(mdx, std::abs(kv.first.first));
    mdy = std::max(mdy, std::abs(kv.first.second));
  }
  c->nD = idx;
  c->ffgrid.assign(17 * 17, -1);
  c->dgrid.assign(17 * 17, -1);
  for (int i = 0; i < c->n_ff; ++i) c->ffgrid[(c->ff[2 * i] + 8) * 17 + c->ff[2 * i + 1] + 8] = i;
  for (auto &kv : dmap) c->dgrid[(kv.first.first + 8) * 17 + kv.first.second + 8] = kv.second;
  c->didx.resize(c->n_ff * c->n_ff);
  for (int i = 0; i < c->n_ff; ++i)
    for (int j = 0; j < c->n_ff; ++j)
      c->didx[i * c->n_ff + j] = dmap[{c->ff[2 * i] - c->ff[2 * j], c->ff[2 * i + 1] - c->ff[2 * j + 1]}];
  // computed box of the loop kernel: dx in [0, ndx), dy in [-ndy, ndy]
  if (mdx <= 1 && mdy <= 1) {
    c->ndx = 2;
    c->ndy = 1;
  } else if (mdx <= 2 && mdy <= 2) {
    c->ndx = 3;
    c->ndy = 2;
  } else {
    c->ndx = 5;
    c->ndy = 4;
  }
  if (c->n_o == 2) {
    c->nkyb = (c->Lf + 63) / 64;
    long long base = 2LL * c->Nq * c->nkyb;
    // enough work items to fill the chip, and kx chunks short enough that the
    // k rows of one chunk (each XCD sweeps one chunk over many q at a time)
    // take about 3 MB of its 4 MB L2
    const long long row_bytes = (long long)c->Lf * 8 * (c->prec == 0 ? 8 : 4);
    const long long fill = (4096 + base - 1) / base;
    const long long l2 = ((long long)c->Lf * row_bytes + 3000000 - 1) / 3000000;
    int want = (int)std::max<long long>(1, std::max(fill, l2));
    c->nkxc = std::max(1, std::min(want, std::max(1, c->Lf / 8)));
    // chunks of kxper rows each; drop chunks that would start at or beyond Lf
    const int kxper = (c->Lf + c->nkxc - 1) / c->nkxc;
    c->nkxc = (c->Lf + kxper - 1) / kxper;
  } else if (c->n_o == 1) {
    // the one-band loop kernel: kx chunks so that about 2048 workgroups fill the chip
    c->nkyb = 1;
    c->nkxc = (int)std::max<long long>(1, std::min<long long>(c->Lf, (2048 + 2LL * c->Nq - 1) / (2LL * c->Nq)));
  } else {
    // the multi-orbital loop kernel sums every k of a (q, channel) in one workgroup
    c->nkyb = 1;
    c->nkxc = 1;
    if (!(c->ndx == 5 && c->ndy == 4) && !(c->ndx == 3 && c->ndy == 2)) {
      c->ndx = 3;
      c->ndy = 2;
    }
    // the six-orbital kernels compute the 5 x 5 box (ndy = 2) or the diamond
    // |dx| + |dy| <= 4 (ndy = 4) of difference vectors; a set whose S - S
    // leaves that shape is not supported
    for (size_t i = 0; i < c->dlist.size(); i += 2) {
      const int dx = std::abs(c->dlist[i]), dy = std::abs(c->dlist[i + 1]);
      const bool inside = c->ndy == 2 ? (dx <= 2 && dy <= 2) : (dx + dy <= 4);
      if (!inside) {
        c->err = "six-orbital loops cover R1 - R2 with |dx| + |dy| <= 4 (or the 5 x 5 box); (" +
                 std::to_string(c->dlist[i]) + ", " + std::to_string(c->dlist[i + 1]) + ") is outside";
        g_err = c->err;
        delete c;
        return TUFRG_E_UNSUPPORTED;
      }
    }
  }
  {
    // distinct rho_y over D (the projections' qy phases); D lies in [-4, 4]^2
    // for form factors with |R| <= 2
    std::vector<int> ys;
    for (int i = 0; i < c->nD; ++i)
      if (std::find(ys.begin(), ys.end(), c->dlist[2 * i + 1]) == ys.end()) ys.push_back(c->dlist[2 * i + 1]);
    c->ny = (int)ys.size();
    // the projections' intermediate: whole qx rows of [2][ny][B^2] complex, up
    // to about 1 GB
    const size_t per_row = 2 * 2 * (size_t)c->ny * c->B * c->B;
    const size_t rows = std::max<size_t>(1, std::min<size_t>((size_t)c->Lq, ((size_t)1 << 27) / per_row));
    c->proj_ws = rows * per_row;
  }
  auto bail = [&](tufrg_status st) {
    g_err = c->err;
    destroy_all(c);
    delete c;
    return st;
  };
  {
    // the device of the context, and (once per device) the address of the
    // static scratch of tufrg_project_static on it
    hipError_t e = hipGetDevice(&c->device);
    if (e == hipSuccess) e = static_scratch_lookup(c->device);
    if (e != hipSuccess) {
      (void)hipGetLastError();
      c->err = std::string("device set-up failed: ") + hipGetErrorString(e);
      return bail(TUFRG_E_HIP);
    }
  }
#define CTRY(x)                          \
  do {                                   \
    tufrg_status s_ = (x);               \
    if (s_ != TUFRG_OK) return bail(s_); \
  } while (0)
#define CHIP(x)                                                                       \
  do {                                                                                \
    hipError_t e_ = (x);                                                              \
    if (e_ != hipSuccess) {                                                           \
      (void)hipGetLastError();                                                        \
      c->err = std::string(#x) + ": " + hipGetErrorString(e_);                         \
      return bail(TUFRG_E_HIP);                                                       \
    }                                                                                 \
  } while (0)

  const size_t Nf = c->Nf, BB = (size_t)c->B * c->B;
  CTRY(dalloc(c, &c->d_ff, c->ff.size()));
  CTRY(dalloc(c, &c->d_fneg, c->n_ff));
  CTRY(dalloc(c, &c->d_dlist, c->dlist.size()));
  CTRY(dalloc(c, &c->d_didx, c->didx.size()));
  CTRY(dalloc(c, &c->d_ffgrid, c->ffgrid.size()));
  CTRY(dalloc(c, &c->d_dgrid, c->dgrid.size()));
  CTRY(dalloc(c, &c->d_hopR, 2 * (size_t)m->n_hop));
  CTRY(dalloc(c, &c->d_hopt, 2 * (size_t)m->n_hop * c->no2));
  CTRY(dalloc(c, &c->d_band64, Nf * (c->n_o + c->n_o * c->no2)));
  CTRY(dalloc(c, &c->d_band32, Nf * (c->n_o + c->n_o * c->no2)));
  if (c->n_o == 2) {
    CTRY(dalloc(c, &c->d_ekv64, 4 * Nf));
    CTRY(dalloc(c, &c->d_ekv32, 4 * Nf));
    CTRY(dalloc(c, &c->d_pi4_64, 4 * Nf));
    CTRY(dalloc(c, &c->d_pi4_32, 4 * Nf));
  }
  if (c->n_o > 2) {
    CTRY(dalloc(c, &c->d_bandk64, Nf * (c->n_o + c->n_o * c->no2)));
    CTRY(dalloc(c, &c->d_bandk32, Nf * (c->n_o + c->n_o * c->no2)));
    // entry (a,b,c,d) and its partner (c,d,a,b): one of each pair, in entry order
    const int no2 = c->no2;
    for (int t = 0; t < c->no4; ++t) {
      const int tb = (t % no2) * no2 + t / no2;
      if (t <= tb) {
        c->pairs.push_back(t);
        c->pairs.push_back(tb);
      }
    }
    c->n_pairs = (int)c->pairs.size() / 2;
    CTRY(dalloc(c, &c->d_pairs, c->pairs.size()));
    CTRY(dalloc(c, &c->d_phy64, 2 * (size_t)c->Lf * c->ndy));
    CTRY(dalloc(c, &c->d_phy32, 2 * (size_t)c->Lf * c->ndy));
  }
  CTRY(dalloc(c, &c->d_kv64, Nf * c->n_o));
  CTRY(dalloc(c, &c->d_kv32, Nf * c->n_o));
  if (c->scheme == CUT_SHELL) {
    CTRY(dalloc(c, &c->d_cv64, 2 * Nf * c->n_o));
    CTRY(dalloc(c, &c->d_cv32, 2 * Nf * c->n_o));
  }
  CTRY(dalloc(c, &c->d_twf, 2 * (size_t)c->Lf));
  CTRY(dalloc(c, &c->d_twf32, 2 * (size_t)c->Lf));
  CTRY(dalloc(c, &c->d_twq, 2 * (size_t)c->Lq));
  CTRY(dalloc(c, &c->d_dtab, c->nD + 81));
  const size_t nparts = (size_t)c->nkyb * c->nkxc;
  c->partial_cap = c->n_o == 1 ? loop1_partial_doubles(c->Nq, c->nD, c->nkxc)
                               : 2 * 2 * (size_t)c->Nq * nparts * c->ndx * (2 * c->ndy + 1) * c->no4;
  CTRY(dalloc(c, &c->d_partial, c->partial_cap));
  CTRY(dalloc(c, &c->d_loop, 2 * 2 * (size_t)c->Nq * c->nD * c->no4));
  CTRY(dalloc(c, &c->d_ftpart, c->proj_ws));
  CTRY(dalloc(c, &c->d_real, 2 * 2 * (size_t)c->nD * BB));
  CTRY(dalloc(c, &c->d_G, 2 * 2 * (size_t)c->nD * BB));
  CTRY(dalloc(c, &c->d_v0p, 2 * BB));
  CTRY(dalloc(c, &c->d_v0c, 2 * BB));
  CTRY(dalloc(c, &c->d_VP, 2 * BB * c->Nq));
  CTRY(dalloc(c, &c->d_VC, 2 * BB * c->Nq));
  if (c->B > 64) {
    size_t nd = 2 * BB * c->Nq;
    if (c->prec == TUFRG_BF16X3) nd = std::max(nd, (bundle_split_bytes_per_q(c->B) + 7) / 8);
    CTRY(dalloc(c, &c->d_btmp, nd));
    c->btmp_bytes = nd * sizeof(double);
  }
  CTRY(dalloc(c, &c->d_bits, 4));
  CTRY(dalloc(c, &c->d_flag, 4));
  CHIP(hipHostMalloc((void **)&c->h_bits, 4 * sizeof(unsigned long long), hipHostMallocDefault));
  CHIP(hipHostMalloc((void **)&c->h_flag, 4 * sizeof(unsigned int), hipHostMallocDefault));
  CTRY(dalloc(c, &c->d_sbits, 4));
  CHIP(hipHostMalloc((void **)&c->h_sbits, 4 * sizeof(unsigned long long), hipHostMallocDefault));
  CTRY(dalloc(c, &c->d_rows, c->Lq));
  CHIP(hipHostMalloc((void **)&c->h_rows, c->Lq * sizeof(int), hipHostMallocDefault));

  // tables
  std::vector<double> twf(2 * c->Lf), twq(2 * c->Lq);
  for (int j = 0; j < c->Lf; ++j) {
    const double a = 2.0 * M_PI * (double)j / (double)c->Lf;
    twf[2 * j] = std::cos(a);
    twf[2 * j + 1] = -std::sin(a);
  }
  for (int j = 0; j < c->Lq; ++j) {
    const double a = 2.0 * M_PI * (double)j / (double)c->Lq;
    twq[2 * j] = std::cos(a);
    twq[2 * j + 1] = std::sin(a);
  }
  std::vector<double> phy64;
  std::vector<float> phy32;
  if (c->n_o > 2) {
    for (int ky = 0; ky < c->Lf; ++ky)
      for (int dy = 1; dy <= c->ndy; ++dy) {
        const int j = (int)(((long long)ky * dy) % c->Lf);
        phy64.push_back(twf[2 * j]);
        phy64.push_back(twf[2 * j + 1]);
      }
    phy32.assign(phy64.begin(), phy64.end());
  }
  std::vector<double> v0p(2 * BB, 0.0), v0c(2 * BB, 0.0);
  const int n = c->n_o;
  for (int a = 0; a < n; ++a)
    for (int b = 0; b < n; ++b)
      for (int cc = 0; cc < n; ++cc)
        for (int d = 0; d < n; ++d) {
          const size_t e = (size_t)(a * n + b) * c->B + (cc * n + d);
          const tufrg_c64 vp = m->V0[((a * n + b) * n + d) * n + cc];  // V0_{a b d c}
          const tufrg_c64 vc = m->V0[((a * n + d) * n + b) * n + cc];  // V0_{a d b c}
          v0p[2 * e] = vp.re;
          v0p[2 * e + 1] = vp.im;
          v0c[2 * e] = vc.re;
          v0c[2 * e + 1] = vc.im;
        }
  hipStream_t st = c->st;
  CHIP(hipMemcpyAsync(c->d_ff, c->ff.data(), c->ff.size() * sizeof(int), hipMemcpyHostToDevice, st));
  if (c->n_pairs)
    CHIP(hipMemcpyAsync(c->d_pairs, c->pairs.data(), c->pairs.size() * sizeof(int), hipMemcpyHostToDevice, st));
  CHIP(hipMemcpyAsync(c->d_dlist, c->dlist.data(), c->dlist.size() * sizeof(int), hipMemcpyHostToDevice, st));
  CHIP(hipMemcpyAsync(c->d_didx, c->didx.data(), c->didx.size() * sizeof(int), hipMemcpyHostToDevice, st));
  CHIP(hipMemcpyAsync(c->d_ffgrid, c->ffgrid.data(), c->ffgrid.size() * sizeof(int), hipMemcpyHostToDevice, st));
  CHIP(hipMemcpyAsync(c->d_dgrid, c->dgrid.data(), c->dgrid.size() * sizeof(int), hipMemcpyHostToDevice, st));
  CHIP(hipMemcpyAsync(c->d_hopR, m->hop_R, 2 * (size_t)m->n_hop * sizeof(int), hipMemcpyHostToDevice, st));
  CHIP(hipMemcpyAsync(c->d_hopt, m->hop_t, (size_t)m->n_hop * c->no2 * sizeof(tufrg_c64), hipMemcpyHostToDevice,
                      st));
  CHIP(hipMemcpyAsync(c->d_twf, twf.data(), twf.size() * sizeof(double), hipMemcpyHostToDevice, st));
  std::vector<float> twf32(twf.begin(), twf.end());
  CHIP(hipMemcpyAsync(c->d_twf32, twf32.data(), twf32.size() * sizeof(float), hipMemcpyHostToDevice, st));
  CHIP(hipMemcpyAsync(c->d_twq, twq.data(), twq.size() * sizeof(double), hipMemcpyHostToDevice, st));
  // e^{i q.rho} = e^{2 pi i qx rho_x / Lq} e^{2 pi i qy rho_y / Lq}, both from
  // exact integer phases mod Lq: the qy factors of the distinct rho_y, and per
  // rho its rho_x and the slot of its rho_y
  {
    auto mod = [&](long long v) { return (int)(((v % c->Lq) + c->Lq) % c->Lq); };
    std::vector<int> ys;
    for (int i = 0; i < c->nD; ++i)
      if (std::find(ys.begin(), ys.end(), c->dlist[2 * i + 1]) == ys.end()) ys.push_back(c->dlist[2 * i + 1]);
    std::sort(ys.begin(), ys.end());
    if (c->ny != (int)ys.size() || c->ny > 9) {  // D lies in [-4, 4]^2 for form factors with |R| <= 2
      c->err = "more than nine distinct rho_y in D";
      return bail(TUFRG_E_UNSUPPORTED);
    }
    std::vector<double> pphy(2 * (size_t)c->Lq * c->ny);
    for (int qy = 0; qy < c->Lq; ++qy)
      for (int y = 0; y < c->ny; ++y) {
        const int j = mod((long long)qy * ys[y]);
        pphy[2 * ((size_t)qy * c->ny + y)] = twq[2 * j];
        pphy[2 * ((size_t)qy * c->ny + y) + 1] = twq[2 * j + 1];
      }
    // dtab [nD], then the slot table [9][9]
    std::vector<int> dtab(c->nD + 81, -1), fill(9, 0);
    for (int i = 0; i < c->nD; ++i) {
      const int sl = (int)(std::find(ys.begin(), ys.end(), c->dlist[2 * i + 1]) - ys.begin());
      dtab[i] = mod(c->dlist[2 * i]) | (sl << 16);
      if (fill[sl] >= 9) {  // at most nine rho_x per rho_y in [-4, 4]^2
        c->err = "more than nine rho with one rho_y in D";
        return bail(TUFRG_E_UNSUPPORTED);
      }
      dtab[c->nD + 9 * sl + fill[sl]++] = i | (mod(c->dlist[2 * i]) << 16);
    }
    CTRY(dalloc(c, &c->d_pphy, pphy.size()));
    CHIP(hipMemcpyAsync(c->d_pphy, pphy.data(), pphy.size() * sizeof(double), hipMemcpyHostToDevice, st));
    CHIP(hipMemcpyAsync(c->d_dtab, dtab.data(), dtab.size() * sizeof(int), hipMemcpyHostToDevice, st));
    CHIP(hipStreamSynchronize(st));  // the host tables end with this block
  }
  if (c->n_o > 2) {
    CHIP(hipMemcpyAsync(c->d_phy64, phy64.data(), phy64.size() * sizeof(double), hipMemcpyHostToDevice, st));
    CHIP(hipMemcpyAsync(c->d_phy32, phy32.data(), phy32.size() * sizeof(float), hipMemcpyHostToDevice, st));
  }
  std::vector<int> fneg(c->n_ff, 0);
  for (int i = 0; i < c->n_ff; ++i)
    for (int j = 0; j < c->n_ff; ++j)
      if (c->ff[2 * j] == -c->ff[2 * i] && c->ff[2 * j + 1] == -c->ff[2 * i + 1]) fneg[i] = j;
  CHIP(hipMemcpyAsync(c->d_fneg, fneg.data(), fneg.size() * sizeof(int), hipMemcpyHostToDevice, st));
  CHIP(hipMemcpyAsync(c->d_v0p, v0p.data(), v0p.size() * sizeof(double), hipMemcpyHostToDevice, st));
  CHIP(hipMemcpyAsync(c->d_v0c, v0c.data(), v0c.size() * sizeof(double), hipMemcpyHostToDevice, st));
  CHIP(launch_band(c->n_o, c->Lf, m->n_hop, c->d_hopR, c->d_hopt, m->mu, s->basis == TUFRG_BASIS_BAND ? 1 : 0,
                   c->d_band64, c->d_band64 + Nf * c->n_o, c->d_band32, c->d_band32 + Nf * c->n_o, st));
  if (c->n_o > 2) CHIP(launch_to_kmajor(c->n_o + c->n_o * c->no2, (int)Nf, c->d_band64, c->d_bandk64, c->d_bandk32, st));
  if (c->n_o == 2) CHIP(launch_pi4((int)Nf, c->d_band64, c->d_pi4_64, c->d_pi4_32, st));
  CHIP(hipStreamSynchronize(st));
  if (c->n_o == 6) {
    // Kramers pairs: e_{2p} = e_{2p+1} at every k up to the eigensolver's
    // rounding (sorted bands); then the sum over bands in the loops groups
    // exactly into three pairs with the summed projectors
    std::vector<double> e(6 * Nf);
    CHIP(hipMemcpy(e.data(), c->d_band64, e.size() * sizeof(double), hipMemcpyDeviceToHost));
    double emax = 0.0, split = 0.0;
    for (size_t i = 0; i < e.size(); ++i) emax = std::max(emax, std::fabs(e[i]));
    for (int p = 0; p < 3; ++p)
      for (size_t k = 0; k < Nf; ++k) split = std::max(split, std::fabs(e[(2 * p) * Nf + k] - e[(2 * p + 1) * Nf + k]));
    if (split <= 1e-10 * std::max(1.0, emax)) {
      if (c->prec == TUFRG_FP64)
        CTRY(dalloc(c, &c->d_pir64, Nf * 3 * 36));
      else
        CTRY(dalloc(c, &c->d_pir32, Nf * 3 * 36));
      CHIP(launch_pair_pi((int)Nf, c->d_band64, c->d_pir32, c->d_pir64, st));
      CHIP(hipStreamSynchronize(st));
      c->bands_paired = 1;
    }
  }
  *out = c;
  return TUFRG_OK;
#undef CTRY
#undef CHIP
}

extern "C" tufrg_status tufrg_destroy(tufrg_ctx *c) {
  if (!c) return TUFRG_OK;
  (void)hipStreamSynchronize(c->st);
  destroy_all(c);
  delete c;
  return TUFRG_OK;
}

extern "C" tufrg_status tufrg_dims(const tufrg_ctx *c, int32_t *B, int32_t *Nq, int32_t *Nf, int32_t *n_dR) {
  if (!c) return fail(nullptr, TUFRG_E_INVAL, "null context");
  if (B) *B = c->B;
  if (Nq) *Nq = c->Nq;
  if (Nf) *Nf = c->Nf;
  if (n_dR) *n_dR = c->nD;
  return TUFRG_OK;
}

extern "C" tufrg_status tufrg_band_data(tufrg_ctx *c, double *e, tufrg_c64 *Pi) {
  if (!c) return fail(nullptr, TUFRG_E_INVAL, "null context");
  if (!is_device_ptr(e) || !is_device_ptr(Pi)) return fail(c, TUFRG_E_INVAL, "e and Pi must be device pointers");
  HIPCHK(c, hipMemcpyAsync(e, c->d_band64, sizeof(double) * c->n_o * (size_t)c->Nf, hipMemcpyDeviceToDevice, c->st));
  HIPCHK(c, launch_unpack_pi(c->n_o, c->Nf, c->d_band64 + (size_t)c->Nf * c->n_o, (double *)Pi, c->st));
  return TUFRG_OK;
}

// the loops sum Kramers pairs: six-orbital bands found paired, pairing not
// switched off, and for the matrix-core loop an even fine mesh (ky pairs)
static int pairs_active(const tufrg_ctx *c) {
  if (c->n_o != 6 || !c->bands_paired || !c->pair_enable) return 0;
  return c->prec == TUFRG_BF16X3 ? c->Lf % 2 == 0 : 1;
}

static LoopArgs loop_args(tufrg_ctx *c, double lam, int deriv, int ch_first, int n_ch) {
  LoopArgs a;
  a.n_o = c->n_o;
  a.Lq = c->Lq;
  a.n_ref = c->n_ref;
  a.Lf = c->Lf;
  a.Nq = c->Nq;
  a.ndx = c->ndx;
  a.ndy = c->ndy;
  a.nkyb = c->nkyb;
  a.nkxc = c->nkxc;
  a.kxr = c->mfma_kxr;
  a.pair = pairs_active(c);
  a.pir = c->d_pir32;
  a.pir64 = c->d_pir64;
  a.ch_first = ch_first;
  a.n_ch = n_ch;
  a.q_first = 0;
  a.n_q = c->Nq;
  a.scheme = c->scheme;
  a.deriv = deriv;
  a.prec = c->prec;
  a.lam = lam;
  if (c->n_o > 2)
    a.band = c->prec == 0 ? (const void *)c->d_bandk64 : (const void *)c->d_bandk32;
  else
    a.band = c->prec == 0 ? (const void *)c->d_band64 : (const void *)c->d_band32;
  a.kv = c->prec == 0 ? (const void *)c->d_kv64 : (const void *)c->d_kv32;
  a.tw = c->d_twf;
  a.tw32 = c->d_twf32;
  a.partial = c->d_partial;
  a.pairs = c->d_pairs;
  a.n_pairs = c->n_pairs;
  a.phy = c->prec == 0 ? (const void *)c->d_phy64 : (const void *)c->d_phy32;
  a.ekv = c->prec == 0 ? (const void *)c->d_ekv64 : (const void *)c->d_ekv32;
  a.pi4 = c->prec == 0 ? (const void *)c->d_pi4_64 : (const void *)c->d_pi4_32;
  if (c->scheme == CUT_SHELL) {
    // the kernels' divided differences are those of the fixed-temperature J
    // (regulator values at Lambda = T); the Lambda dependence and deriv are
    // in the shell factors
    a.lam = c->temp;
    a.deriv = 0;
    a.cv = c->prec == 0 ? (const void *)c->d_cv64 : (const void *)c->d_cv32;
  }
  return a;
}

static ProjArgs proj_args(tufrg_ctx *c) {
  ProjArgs a;
  a.n_o = c->n_o;
  a.n_ff = c->n_ff;
  a.B = c->B;
  a.Lq = c->Lq;
  a.Nq = c->Nq;
  a.nD = c->nD;
  a.dlist = c->d_dlist;
  a.ffgrid = c->d_ffgrid;
  a.dgrid = c->d_dgrid;
  a.ff = c->d_ff;
  a.twq = c->d_twq;
  a.ny = c->ny;
  a.phy = c->d_pphy;
  a.dtab = c->d_dtab;
  a.dslot = c->d_dtab + c->nD;
  return a;
}

static tufrg_status compute_kval(tufrg_ctx *c, double lam, int deriv) {
  // momentum shell: J of the fixed temperature in the regulator slot, the
  // shell factors at Lambda beside it
  const bool shell = c->scheme == CUT_SHELL;
  const double rl = shell ? c->temp : lam;
  const int rs = shell ? CUT_TEMPERATURE : c->scheme, rd = shell ? 0 : deriv;
  if (c->n_o == 2)
    HIPCHK(c, launch_ekv4(c->Nf, c->d_band64, rl, rs, rd, c->d_ekv64, c->d_ekv32, c->st));
  else
    HIPCHK(c, launch_kval(c->n_o * c->Nf, c->Nf, c->n_o, c->d_band64, rl, rs, rd, c->d_kv64, c->d_kv32, c->st));
  if (shell) HIPCHK(c, launch_shell_ab(c->n_o, c->Nf, c->d_band64, lam, deriv, c->d_cv64, c->d_cv32, c->st));
  return TUFRG_OK;
}

static void dfree(tufrg_ctx *c, void *p);

// the matrix-core loop's A operand for the current pairing (rebuilt when the
// pairing changed since it was computed)
static tufrg_status ensure_apre(tufrg_ctx *c) {
  const int pair = pairs_active(c);
  if (c->d_apre && c->apre_pair != pair) {
    HIPCHK(c, hipStreamSynchronize(c->st));
    dfree(c, c->d_apre);
    c->d_apre = nullptr;
  }
  if (!c->d_apre) {
    unsigned char *ap = nullptr;
    TRY(dalloc(c, &ap, loop_rb_apre_bytes(c->ndy, c->Lf, pair)));
    HIPCHK(c, launch_loop_rb_apre(c->ndy, pair, c->d_bandk32, c->d_pir32, c->d_phy32, c->Lf, ap, c->st));
    c->d_apre = ap;
    c->apre_pair = pair;
  }
  return TUFRG_OK;
}

// loops of channels [ch_first, ch_first + n_ch) and coarse q [q_first, q_first + n_q)
// (whole q_x rows) into dst, compact [n_ch][n_q][nD][no4]; regulator values
// must be current (compute_kval)
static tufrg_status loops_range_mfma(tufrg_ctx *c, double lam, int deriv, int ch_first, int n_ch, int q_first,
                                     int n_q, double *dst, const int *rows) {
  if (!c->d_hmap) {
    // half-plane point of each difference vector (the others by conjugation)
    int hx[32], hy[32];
    const int nh = loop_rb_half_points(c->ndy, hx, hy);
    std::vector<int> hm(c->nD, -1);
    for (int i = 0; i < c->nD; ++i) {
      int dx = c->dlist[2 * i], dy = c->dlist[2 * i + 1], cj = 0;
      if (dx < 0 || (dx == 0 && dy < 0)) {
        dx = -dx;
        dy = -dy;
        cj = 1;
      }
      for (int h = 0; h < nh; ++h)
        if (hx[h] == dx && hy[h] == dy) hm[i] = h | (cj << 16);
      if (hm[i] < 0) return fail(c, TUFRG_E_UNSUPPORTED, "difference vector outside the loop kernel's shape");
    }
    int *d = nullptr;
    TRY(dalloc(c, &d, hm.size()));
    HIPCHK(c, hipMemcpyAsync(d, hm.data(), hm.size() * sizeof(int), hipMemcpyHostToDevice, c->st));
    HIPCHK(c, hipStreamSynchronize(c->st));
    c->d_hmap = d;
  }
  TRY(ensure_apre(c));
  if (!c->d_yrow || !c->d_lamb) {
    // whole q_x rows per chunk, about 256 coarse q (64 groups of four); where
    // some 256..512 q make a group count that is a multiple of the
    // workgroups one XCD runs at once (one per CU), that size: the work items
    // of one kx block then start together on their XCD and read its A
    // operand from L2 in step (a quarter of the fabric traffic of a ragged
    // count on the 48 x 48 mesh)
    c->mfma_chunk = std::max(1, 256 / c->Lq) * c->Lq;
    int ncu = 0;
    if (hipDeviceGetAttribute(&ncu, hipDeviceAttributeMultiprocessorCount, c->device) != hipSuccess) {
      (void)hipGetLastError();
      ncu = 0;
    }
    const int per_xcd = ncu / 8;
    for (int m = 1; per_xcd > 0 && m * c->Lq <= 512; ++m) {
      const int nq = m * c->Lq;
      if (nq >= 256 && nq % 4 == 0 && (nq / 4) % per_xcd == 0) {
        c->mfma_chunk = nq;
        break;
      }
    }
    const size_t groups = (size_t)(c->mfma_chunk + 3) / 4;
    if (!c->d_yrow) TRY(dalloc(c, &c->d_yrow, groups * loop_rb_rowbuf_floats(c->ndy, c->Lf)));
    int hx[32], hy[32];
    const size_t nh = (size_t)loop_rb_half_points(c->ndy, hx, hy);
    TRY(dalloc(c, &c->d_lamb, 2 * (size_t)c->mfma_chunk * nh * 36 * 36));
  }
  const size_t blk = (size_t)c->nD * c->no4;
  for (int chi = 0; chi < n_ch; ++chi) {
    const int ch = ch_first + chi;
    for (int q0 = 0; q0 < n_q; q0 += c->mfma_chunk) {
      const int nq = std::min(c->mfma_chunk, n_q - q0);
      LoopArgs a = loop_args(c, lam, deriv, ch, 1);
      a.q_first = rows ? 0 : q_first + q0;
      a.n_q = nq;
      a.rows = rows ? rows + q0 / c->Lq : nullptr;
      // the loop timer covers the matrix-core kernel of each chunk
      HIPCHK(c, timer_mark(c, TUFRG_TIMER_LOOP));
      HIPCHK(c, launch_loop_rb(a, ch, c->d_apre, c->d_yrow, c->st));
      HIPCHK(c, timer_mark(c, TUFRG_TIMER_LOOP));
      HIPCHK(c, launch_loop_rb_sums(a, c->d_yrow, c->d_lamb, c->d_hmap, c->nD,
                                    dst + 2 * ((size_t)chi * n_q + q0) * blk, c->st));
    }
  }
  return TUFRG_OK;
}

static tufrg_status loops_range(tufrg_ctx *c, double lam, int deriv, int ch_first, int n_ch, int q_first, int n_q,
                                double *dst, const int *rows = nullptr) {
  if (c->prec == TUFRG_BF16X3) return loops_range_mfma(c, lam, deriv, ch_first, n_ch, q_first, n_q, dst, rows);
  if (c->n_o == 1) {
    if (rows) return fail(c, TUFRG_E_UNSUPPORTED, "sampled q rows need two or six spin-orbitals");
    HIPCHK(c, timer_mark(c, TUFRG_TIMER_LOOP));
    HIPCHK(c, launch_loop1(c->Lq, c->n_ref, c->nD, c->d_dlist, c->d_band64, c->d_kv64, c->d_twf, lam, c->scheme,
                           deriv, ch_first, n_ch, q_first, n_q, c->nkxc, c->d_partial, dst, c->st));
    HIPCHK(c, timer_mark(c, TUFRG_TIMER_LOOP));
    return TUFRG_OK;
  }
  LoopArgs a = loop_args(c, lam, deriv, ch_first, n_ch);
  a.q_first = q_first;
  a.n_q = n_q;
  a.rows = rows;
  HIPCHK(c, timer_mark(c, TUFRG_TIMER_LOOP));
  HIPCHK(c, launch_loop(a, c->st));
  HIPCHK(c, timer_mark(c, TUFRG_TIMER_LOOP));
  HIPCHK(c, launch_loop_finalize(a, c->nD, c->d_dlist, dst, c->st));
  return TUFRG_OK;
}

// loops of channels [ch_first, ch_first + n_ch) into the compact buffer
static tufrg_status compute_loops(tufrg_ctx *c, double lam, int deriv, int ch_first, int n_ch) {
  TRY(compute_kval(c, lam, deriv));
  double *dst = c->d_loop + 2 * (size_t)ch_first * c->Nq * c->nD * c->no4;
  return loops_range(c, lam, deriv, ch_first, n_ch, 0, c->Nq, dst);
}

// ---------------------------------------------------------------------------
// Autotuner of the loop kernels' launch shapes

static void dfree(tufrg_ctx *c, void *p) {
  if (!p) return;
  auto it = std::find(c->allocs.begin(), c->allocs.end(), p);
  if (it != c->allocs.end()) c->allocs.erase(it);
  (void)hipFree(p);
}

// kx chunks of the two-orbital loop kernel: whole chunks of ceil(Lf / n) rows,
// none starting at or beyond Lf; the partial sums grow with the chunks
static int normalized_kx_chunks(const tufrg_ctx *c, int n) {
  n = std::max(1, std::min(n, c->Lf));
  const int kxper = (c->Lf + n - 1) / n;
  return (c->Lf + kxper - 1) / kxper;
}

static tufrg_status set_kx_chunks(tufrg_ctx *c, int n) {
  const size_t need = 2 * 2 * (size_t)c->Nq * c->nkyb * n * c->ndx * (2 * c->ndy + 1) * c->no4;
  if (need > c->partial_cap) {
    HIPCHK(c, hipStreamSynchronize(c->st));
    dfree(c, c->d_partial);
    c->d_partial = nullptr;
    c->partial_cap = 0;
    TRY(dalloc(c, &c->d_partial, need));
    c->partial_cap = need;
  }
  c->nkxc = n;
  return TUFRG_OK;
}

static std::string tune_key(const tufrg_ctx *c) {
  hipDeviceProp_t prop;
  std::string arch = "unknown";
  int cus = 0;
  if (hipGetDeviceProperties(&prop, c->device) == hipSuccess) {
    arch = prop.gcnArchName;
    cus = prop.multiProcessorCount;
  } else {
    (void)hipGetLastError();
  }
  char buf[256];
  std::snprintf(buf, sizeof(buf),
                "%s:%dcu|n_o=%d|prec=%d|scheme=%d|Lq=%d|n_ref=%d|n_ff=%d|nD=%d|ndx=%d|ndy=%d|pairs=%d",
                arch.c_str(), cus, c->n_o, c->prec, c->scheme, c->Lq, c->n_ref, c->n_ff, c->nD, c->ndx, c->ndy,
                pairs_active(c));
  return buf;
}

// mean time of one evaluation of both loop channels at lam, after one
// untimed evaluation; repeats until about 50 ms are timed (at most 20)
static tufrg_status time_loops(tufrg_ctx *c, double lam, double *ms) {
  struct Ev {
    hipEvent_t a = nullptr, b = nullptr;
    ~Ev() {
      if (a) (void)hipEventDestroy(a);
      if (b) (void)hipEventDestroy(b);
    }
  } ev;
  HIPCHK(c, hipEventCreate(&ev.a));
  HIPCHK(c, hipEventCreate(&ev.b));
  HIPCHK(c, hipEventRecord(ev.a, c->st));
  TRY(compute_loops(c, lam, 1, 0, 2));
  HIPCHK(c, hipEventRecord(ev.b, c->st));
  HIPCHK(c, hipEventSynchronize(ev.b));
  float first = 0.f;
  HIPCHK(c, hipEventElapsedTime(&first, ev.a, ev.b));
  const int reps = (int)std::max(2.0, std::min(20.0, std::ceil(50.0 / std::max(1e-3, (double)first))));
  HIPCHK(c, hipEventRecord(ev.a, c->st));
  for (int r = 0; r < reps; ++r) TRY(compute_loops(c, lam, 1, 0, 2));
  HIPCHK(c, hipEventRecord(ev.b, c->st));
  HIPCHK(c, hipEventSynchronize(ev.b));
  float t = 0.f;
  HIPCHK(c, hipEventElapsedTime(&t, ev.a, ev.b));
  *ms = (double)t / reps;
  return TUFRG_OK;
}

extern "C" tufrg_status tufrg_autotune(tufrg_ctx *c, double lambda, const char *cache_path, tufrg_tune_result *res) {
  if (!c) return fail(nullptr, TUFRG_E_INVAL, "null context");
  if (!res) return fail(c, TUFRG_E_INVAL, "null result");
  if (!(lambda > 0.0) || !std::isfinite(lambda)) return fail(c, TUFRG_E_INVAL, "lambda must be positive");
  std::memset(res, 0, sizeof(*res));
  const bool no2 = c->n_o == 2, mx = c->prec == TUFRG_BF16X3;
  res->loop_kx_chunks = c->nkxc;
  res->mfma_kx_rows = c->mfma_kxr;
  if (!no2 && !mx) return TUFRG_OK;  // one workgroup per (q, channel): no launch shape to tune
  res->tunable = 1;
  const char *pname = no2 ? "loop_kx_chunks" : "mfma_kx_rows";
  auto apply = [&](int v) -> tufrg_status {
    if (no2) return set_kx_chunks(c, normalized_kx_chunks(c, v));
    c->mfma_kxr = std::max(1, std::min(v, 8));
    return TUFRG_OK;
  };
  const std::string key = tune_key(c);
  TuneEntries cache;
  if (cache_path) {
    std::string err;
    if (!tune_cache_read(cache_path, cache, err)) return fail(c, TUFRG_E_INVAL, err);
    auto it = cache.find(key);
    if (it != cache.end() && it->second.count(pname)) {
      TRY(apply((int)std::llround(it->second.at(pname))));
      res->from_cache = 1;
      res->loop_kx_chunks = c->nkxc;
      res->mfma_kx_rows = c->mfma_kxr;
      res->loop_ms = it->second.count("loop_ms") ? it->second.at("loop_ms") : 0.0;
      res->default_ms = it->second.count("default_ms") ? it->second.at("default_ms") : 0.0;
      return TUFRG_OK;
    }
  }
  // candidates around the default: the two-orbital kernel's kx chunking (the
  // default balances filling the chip against the L2 share of a chunk), the
  // matrix-core kernel's kx rows per work item
  const int def = no2 ? c->nkxc : c->mfma_kxr;
  std::vector<int> cand;
  if (no2) {
    for (int v : {def, def / 2, def * 2, def * 4, 1}) {
      const int n = normalized_kx_chunks(c, std::max(1, std::min(v, std::max(1, c->Lf / 8))));
      if (std::find(cand.begin(), cand.end(), n) == cand.end()) cand.push_back(n);
    }
  } else {
    for (int v : {def, 1, 2, 4})
      if (std::find(cand.begin(), cand.end(), v) == cand.end()) cand.push_back(v);
  }
  double best = INFINITY;
  int best_v = def;
  for (int v : cand) {
    TRY(apply(v));
    double ms = 0.0;
    TRY(time_loops(c, lambda, &ms));
    if (v == def) res->default_ms = ms;
    if (ms < best) {
      best = ms;
      best_v = no2 ? c->nkxc : c->mfma_kxr;
    }
  }
  TRY(apply(best_v));
  res->n_candidates = (int32_t)cand.size();
  res->loop_ms = best;
  res->loop_kx_chunks = c->nkxc;
  res->mfma_kx_rows = c->mfma_kxr;
  if (cache_path) {
    cache[key] = {{pname, (double)best_v}, {"loop_ms", best}, {"default_ms", res->default_ms}};
    std::string err;
    if (!tune_cache_write(cache_path, cache, err)) return fail(c, TUFRG_E_INVAL, err);
  }
  return TUFRG_OK;
}

extern "C" tufrg_status tufrg_pair_bands(tufrg_ctx *c, int32_t enable, int32_t *active) {
  if (!c) return fail(nullptr, TUFRG_E_INVAL, "null context");
  if (enable != 0 && enable != 1) return fail(c, TUFRG_E_INVAL, "enable must be 0 or 1");
  c->pair_enable = enable;
  // an A operand already built is rebuilt now, not inside a later flow
  if (c->d_apre) TRY(ensure_apre(c));
  if (active) *active = pairs_active(c);
  return TUFRG_OK;
}

// target scale s(Lambda): the table interpolated linearly in (ln Lambda, ln s),
// constant beyond its ends
static double sur_scale_at(const tufrg_ctx *c, double lam) {
  const std::vector<double> &x = c->sur_lnlam, &y = c->sur_lns;
  const double l = std::log(lam);
  if (x.size() == 1 || l <= x.front()) return std::exp(y.front());
  if (l >= x.back()) return std::exp(y.back());
  const size_t i = std::upper_bound(x.begin(), x.end(), l) - x.begin();
  const double t = (l - x[i - 1]) / (x[i] - x[i - 1]);
  return std::exp(y[i - 1] + t * (y[i] - y[i - 1]));
}

// network loops of all 2 Nq nD blocks into dst (compact, both channels)
static const long long SUR_CHUNK = 16384;
static tufrg_status sur_loops_internal(tufrg_ctx *c, double lam, double *dst, unsigned int *bad = nullptr) {
  const long long nb = 2LL * c->Nq * c->nD;
  const int nin = 11 + c->nD, nout = 2 * c->no4;
  if (!c->d_surX) {
    TRY(dalloc(c, &c->d_surX, (size_t)nb * nin));
    TRY(dalloc(c, &c->d_surY, (size_t)SUR_CHUNK * nout));
  }
  HIPCHK(c, timer_mark(c, TUFRG_TIMER_SURROGATE));
  HIPCHK(c, launch_sur_features(nb, nullptr, nullptr, nullptr, c->Lq, c->nD, lam, c->d_surX, c->st));
  const double s = sur_scale_at(c, lam);
  for (long long b0 = 0; b0 < nb; b0 += SUR_CHUNK) {
    const long long rows = std::min(SUR_CHUNK, nb - b0);
    TRY(mlp_forward_internal(c->sur, rows, c->d_surX + b0 * nin, c->d_surY));
    HIPCHK(c, launch_sur_scatter(rows, c->no4, s, c->d_surY, dst + b0 * nout, bad, c->st));
  }
  HIPCHK(c, timer_mark(c, TUFRG_TIMER_SURROGATE));
  return TUFRG_OK;
}

static uint64_t splitmix64(uint64_t x) {
  x += 0x9E3779B97F4A7C15ull;
  x = (x ^ (x >> 30)) * 0xBF58476D1CE4E5B9ull;
  x = (x ^ (x >> 27)) * 0x94D049BB133111EBull;
  return x ^ (x >> 31);
}

// loops of both channels for a right-hand side inside a flow with the
// surrogate: network everywhere, plain on sampled q_x rows, plain everywhere
// when the sampled error or the coupling is too large
static tufrg_status surrogate_loops(tufrg_ctx *c, double lam) {
  const tufrg_flow_opts *o = c->fopts;
  tufrg_flow_result *r = c->fres;
  const size_t blk = (size_t)c->nD * c->no4;  // complex values per (channel, q)
  if (c->cur_max > o->plain_above) {
    TRY(compute_loops(c, lam, 1, 0, 2));
    r->n_plain++;
    return TUFRG_OK;
  }
  // d_sbits: max |diff|, max |ref| of the sampled rows, and a flag set by any
  // non-finite network output (sampled or not)
  unsigned int *d_bad = (unsigned int *)(c->d_sbits + 2);
  HIPCHK(c, hipMemsetAsync(c->d_sbits, 0, 3 * sizeof(unsigned long long), c->st));
  TRY(sur_loops_internal(c, lam, c->d_loop, d_bad));
  // sampled rows: distinct q_x rows from a counter-based hash
  int nr = (int)std::llround(o->sample_frac * c->Lq);
  nr = std::max(1, std::min(c->Lq, nr));
  std::vector<int> rows;
  const uint64_t ctr = (uint64_t)(r->n_plain + r->n_surrogate);
  for (uint64_t j = 0; (int)rows.size() < nr; ++j) {
    const int row = (int)(splitmix64(o->sample_seed ^ splitmix64(ctr * 0x100000001B3ull + j)) % (uint64_t)c->Lq);
    if (std::find(rows.begin(), rows.end(), row) == rows.end()) rows.push_back(row);
  }
  // plain loops of the sampled rows in one launch: [2][nr * Lq][nD][no4]
  const size_t rowsz = 2 * (size_t)c->Lq * blk * 2;  // doubles of one sampled row, both channels
  if (nr > c->samp_rows) {
    TRY(dalloc(c, &c->d_samp, rowsz * nr));
    c->samp_rows = nr;
  }
  for (int j = 0; j < nr; ++j) c->h_rows[j] = rows[j];
  HIPCHK(c, hipMemcpyAsync(c->d_rows, c->h_rows, nr * sizeof(int), hipMemcpyHostToDevice, c->st));
  TRY(compute_kval(c, lam, 1));
  TRY(loops_range(c, lam, 1, 0, 2, 0, nr * c->Lq, c->d_samp, c->d_rows));
  auto net_at = [&](int ch, int j) { return c->d_loop + 2 * (((size_t)ch * c->Nq + (size_t)rows[j] * c->Lq) * blk); };
  auto plain_at = [&](int ch, int j) {
    return c->d_samp + 2 * (((size_t)ch * nr * c->Lq + (size_t)j * c->Lq) * blk);
  };
  for (int j = 0; j < nr; ++j)
    for (int ch = 0; ch < 2; ++ch)
      HIPCHK(c, launch_sur_compare((long long)c->Lq * blk, net_at(ch, j), plain_at(ch, j), c->d_sbits, c->st));
  HIPCHK(c, hipMemcpyAsync(c->h_sbits, c->d_sbits, 3 * sizeof(unsigned long long), hipMemcpyDeviceToHost, c->st));
  HIPCHK(c, hipStreamSynchronize(c->st));
  double dmax, rmax;
  std::memcpy(&dmax, &c->h_sbits[0], sizeof(double));
  std::memcpy(&rmax, &c->h_sbits[1], sizeof(double));
  const bool net_bad = (unsigned int)c->h_sbits[2] != 0u;
  // relative to the largest plain loop value of the sampled rows (the table
  // scale s(lam) is only the network's output unit, not a judge)
  double err = rmax > 0.0 ? dmax / rmax : (dmax > 0.0 ? INFINITY : 0.0);
  if (net_bad) err = INFINITY;
  r->max_sample_err = std::max(r->max_sample_err, err);
  if (!(err <= o->sur_tol)) {
    TRY(loops_range(c, lam, 1, 0, 2, 0, c->Nq, c->d_loop));
    r->n_plain++;
    r->n_fallback++;
    return TUFRG_OK;
  }
  for (int j = 0; j < nr; ++j)
    for (int ch = 0; ch < 2; ++ch)
      HIPCHK(c, hipMemcpyAsync(net_at(ch, j), plain_at(ch, j), 2 * sizeof(double) * c->Lq * blk,
                               hipMemcpyDeviceToDevice, c->st));
  r->n_surrogate++;
  return TUFRG_OK;
}

// projections with the buffers given: the workspace ws (ws_doubles, at least
// one qx row of the intermediate), real and G ([2][nD][B][B] complex each)
static tufrg_status project_with(tufrg_ctx *c, const double *P, const double *C, double *VP, double *VC,
                                 double *ws, size_t ws_doubles, double *real, double *G) {
  ProjArgs a = proj_args(c);
  HIPCHK(c, timer_mark(c, TUFRG_TIMER_PROJECT));
  if (c->has_c0) {
    // a non-local initial interaction enters as a static part of the C
    // channel (its D partner follows from C inside the projections)
    HIPCHK(c, launch_add(2 * (long long)c->Nq * c->B * c->B, C, c->d_c0, c->d_ceff, c->st));
    C = c->d_ceff;
  }
  if (c->has_p0) {
    // a bare vertex given by its particle-particle expansion (the band-basis
    // form of an orbital interaction) is a static part of the P channel
    HIPCHK(c, launch_add(2 * (long long)c->Nq * c->B * c->B, P, c->d_p0, c->d_peff, c->st));
    P = c->d_peff;
  }
  HIPCHK(c, launch_ft(a, P, C, ws, ws_doubles, real, c->st));
  HIPCHK(c, launch_gather(a, real, G, c->st));
  HIPCHK(c, launch_assemble(a, P, C, G, c->d_v0p, c->d_v0c, VP, VC, ws, ws_doubles, c->st));
  HIPCHK(c, timer_mark(c, TUFRG_TIMER_PROJECT));
  return TUFRG_OK;
}

static tufrg_status project_internal(tufrg_ctx *c, const double *P, const double *C, double *VP, double *VC) {
  return project_with(c, P, C, VP, VC, c->d_ftpart, c->proj_ws, c->d_real, c->d_G);
}

// dP = scale VP Lpp VP, dC = 2 scale VC Lph VC; a masked channel gets zero
static tufrg_status rhs_products(tufrg_ctx *c, const double *P, const double *C, double *dP, double *dC, double scale,
                                 unsigned mask);

static tufrg_status rhs_internal(tufrg_ctx *c, double lam, const double *P, const double *C, double *dP, double *dC,
                                 double scale, unsigned mask) {
  const size_t BB = (size_t)c->B * c->B;
  if (c->fopts && c->fopts->surrogate && (mask & 3u) == 3u) {
    TRY(surrogate_loops(c, lam));
  } else {
    if ((mask & 3u) == 3u)
      TRY(compute_loops(c, lam, 1, 0, 2));
    else if (mask & 1u)
      TRY(compute_loops(c, lam, 1, 0, 1));
    else if (mask & 2u)
      TRY(compute_loops(c, lam, 1, 1, 1));
    if (c->fres) c->fres->n_plain++;
  }
  return rhs_products(c, P, C, dP, dC, scale, mask);
}

// the right-hand side once the loops of the masked channels are at d_loop:
// projections, then the bundle products
static tufrg_status rhs_products(tufrg_ctx *c, const double *P, const double *C, double *dP, double *dC, double scale,
                                 unsigned mask) {
  const size_t BB = (size_t)c->B * c->B;
  TRY(project_internal(c, P, C, c->d_VP, c->d_VC));
  const size_t lsz = 2 * (size_t)c->Nq * c->nD * c->no4;
  HIPCHK(c, timer_mark(c, TUFRG_TIMER_BUNDLE));
  // mixed precision: the large bundles on the matrix cores
  const bool mx = c->prec == TUFRG_BF16X3 && c->B > 64;
  auto bundle = [&](const double *V, const double *L, double f, double *out) {
    return mx ? launch_bundle_bf16x3(c->n_o, c->n_ff, c->B, c->nD, c->Nq, c->d_didx, V, L, f, out, c->d_btmp,
                                     c->btmp_bytes, c->st)
              : launch_bundle(c->prec, c->n_o, c->n_ff, c->B, c->nD, c->Nq, c->d_didx, V, L, f, out, c->d_btmp,
                              c->st);
  };
  if (mask & 1u)
    HIPCHK(c, bundle(c->d_VP, c->d_loop, scale, dP));
  else
    HIPCHK(c, hipMemsetAsync(dP, 0, 2 * sizeof(double) * BB * c->Nq, c->st));
  if (mask & 2u)
    HIPCHK(c, bundle(c->d_VC, c->d_loop + lsz, 2.0 * scale, dC));
  else
    HIPCHK(c, hipMemsetAsync(dC, 0, 2 * sizeof(double) * BB * c->Nq, c->st));
  HIPCHK(c, timer_mark(c, TUFRG_TIMER_BUNDLE));
  return TUFRG_OK;
}

extern "C" tufrg_status tufrg_timing(tufrg_ctx *c, int32_t enable) {
  if (!c) return fail(nullptr, TUFRG_E_INVAL, "null context");
  HIPCHK(c, hipStreamSynchronize(c->st));
  c->timing = enable != 0;
  for (auto &t : c->timers) {
    t.used = 0;
    t.ms = 0.0;
    t.count = 0;
  }
  return TUFRG_OK;
}

extern "C" tufrg_status tufrg_timing_read(tufrg_ctx *c, int32_t timer, double *total_ms, int32_t *count) {
  if (!c) return fail(nullptr, TUFRG_E_INVAL, "null context");
  if (timer < 0 || timer >= TUFRG_TIMER_COUNT || !total_ms || !count) return fail(c, TUFRG_E_INVAL, "bad timer query");
  HIPCHK(c, hipStreamSynchronize(c->st));
  for (auto &t : c->timers) {
    for (size_t i = 0; i + 1 < t.used; i += 2) {
      float ms = 0.f;
      HIPCHK(c, hipEventElapsedTime(&ms, t.ev[i], t.ev[i + 1]));
      t.ms += ms;
      t.count += 1;
    }
    t.used = 0;
  }
  *total_ms = c->timers[timer].ms;
  *count = c->timers[timer].count;
  return TUFRG_OK;
}

extern "C" tufrg_status tufrg_bubble(tufrg_ctx *c, int32_t channel, double lambda, int32_t deriv, tufrg_c64 *L) {
  if (!c) return fail(nullptr, TUFRG_E_INVAL, "null context");
  if (channel != TUFRG_PP && channel != TUFRG_PH) return fail(c, TUFRG_E_INVAL, "channel must be PP or PH");
  if (!(lambda > 0.0) || !std::isfinite(lambda)) return fail(c, TUFRG_E_INVAL, "lambda must be positive");
  if (!is_device_ptr(L)) return fail(c, TUFRG_E_INVAL, "L must be a device pointer");
  TRY(compute_loops(c, lambda, deriv ? 1 : 0, channel, 1));
  const double *src = c->d_loop + 2 * (size_t)channel * c->Nq * c->nD * c->no4;
  HIPCHK(c, launch_loop_expand(c->n_o, c->n_ff, c->nD, c->Nq, c->d_didx, src, (double *)L, c->st));
  return TUFRG_OK;
}

extern "C" tufrg_status tufrg_basis_matrix(tufrg_ctx *c, int32_t channel, const tufrg_c64 *U, tufrg_c64 *M) {
  if (!c) return fail(nullptr, TUFRG_E_INVAL, "null context");
  if (c->n_o == 1) return fail(c, TUFRG_E_UNSUPPORTED, "one-orbital contexts run the SU(2)-reduced calls");
  if (channel != TUFRG_PP && channel != TUFRG_PH) return fail(c, TUFRG_E_INVAL, "channel must be PP or PH");
  if (!is_device_ptr(U) || !is_device_ptr(M)) return fail(c, TUFRG_E_INVAL, "U and M must be device pointers");
  // compact form [Nq][nD][n_o^4], then expanded like the loops; the row sums of
  // at most about 1 GB of coarse q at a time
  int box = 0;  // largest |component| of a dR in D
  for (int v : c->dlist) box = std::max(box, std::abs(v));
  box = box <= 2 ? 2 : 4;
  const size_t per_q = basis_rows_doubles(c->n_o, c->Lf, box, 1);
  const int q_chunk = (int)std::max<size_t>(1, std::min<size_t>(c->Nq, ((size_t)1 << 27) / per_q));
  // each buffer on its own: a failed allocation leaves the other usable and is retried next call
  if (!c->d_basis_c) TRY(dalloc(c, &c->d_basis_c, 2 * (size_t)c->Nq * c->nD * c->no4));
  if (!c->d_basis_rows) TRY(dalloc(c, &c->d_basis_rows, per_q * q_chunk));
  HIPCHK(c, launch_basis_compact(channel, c->n_o, c->Lq, c->n_ref, c->nD, box, c->d_dlist, (const double *)U,
                                 c->d_twf, c->d_basis_rows, q_chunk, c->d_basis_c, c->st));
  HIPCHK(c, launch_loop_expand(c->n_o, c->n_ff, c->nD, c->Nq, c->d_didx, c->d_basis_c, (double *)M, c->st));
  return TUFRG_OK;
}

extern "C" tufrg_status tufrg_basis_apply(tufrg_ctx *c, const tufrg_c64 *M, const tufrg_c64 *X, tufrg_c64 *Y,
                                          int32_t to_orbital) {
  if (!c) return fail(nullptr, TUFRG_E_INVAL, "null context");
  if (c->n_o == 1) return fail(c, TUFRG_E_UNSUPPORTED, "one-orbital contexts run the SU(2)-reduced calls");
  if (!is_device_ptr(M) || !is_device_ptr(X) || !is_device_ptr(Y))
    return fail(c, TUFRG_E_INVAL, "M, X and Y must be device pointers");
  const size_t n = (size_t)c->Nq * c->B * c->B;
  const uintptr_t m0 = (uintptr_t)M, m1 = m0 + n * sizeof(tufrg_c64), y0 = (uintptr_t)Y,
                  y1 = y0 + n * sizeof(tufrg_c64);
  if (y0 < m1 && m0 < y1) return fail(c, TUFRG_E_INVAL, "Y must not overlap M");
  if (!c->d_basis_tmp) TRY(dalloc(c, &c->d_basis_tmp, 2 * n));
  const double *m = (const double *)M;
  if (!to_orbital) {  // Y = M^H X M
    HIPCHK(c, launch_zgemm_batched(c->B, c->Nq, 1, 0, m, (const double *)X, c->d_basis_tmp, c->st));
    HIPCHK(c, launch_zgemm_batched(c->B, c->Nq, 0, 0, c->d_basis_tmp, m, (double *)Y, c->st));
  } else {  // Y = M X M^H
    HIPCHK(c, launch_zgemm_batched(c->B, c->Nq, 0, 0, m, (const double *)X, c->d_basis_tmp, c->st));
    HIPCHK(c, launch_zgemm_batched(c->B, c->Nq, 0, 1, c->d_basis_tmp, m, (double *)Y, c->st));
  }
  return TUFRG_OK;
}

// Symmetrised form factors: the C4v orbits of S written out by hand (the
// origin; axis shells (+-d, 0), (0, +-d); diagonal shells (+-d, +-d)), rows in
// the order A1, B1 or B2, E (x-like, y-like) per orbit, every row's first
// nonzero coefficient (in the order of S) positive.
extern "C" tufrg_status tufrg_ff_symmetrize(int32_t n_ff, const int32_t *ff_R, tufrg_c64 *W, int32_t *irrep) {
  if (n_ff < 1 || n_ff > 25 || !ff_R || !W || !irrep) return fail(nullptr, TUFRG_E_INVAL, "bad arguments");
  std::map<std::pair<int, int>, int> idx;
  for (int i = 0; i < n_ff; ++i) idx[{ff_R[2 * i], ff_R[2 * i + 1]}] = i;
  if ((int)idx.size() != n_ff) return fail(nullptr, TUFRG_E_INVAL, "duplicate form factor");
  auto at = [&](int x, int y) -> int {
    auto it = idx.find({x, y});
    return it == idx.end() ? -1 : it->second;
  };
  std::vector<double> row(n_ff);
  std::vector<bool> done(n_ff, false);
  int nrow = 0;
  auto emit = [&](int label) {
    int first = 0;
    while (first < n_ff && row[first] == 0.0) ++first;
    const double sg = row[first] < 0.0 ? -1.0 : 1.0;
    for (int i = 0; i < n_ff; ++i) W[(size_t)nrow * n_ff + i] = tufrg_c64{sg * row[i], 0.0};
    irrep[nrow++] = label;
  };
  const double h = 0.5, r2 = std::sqrt(0.5);
  for (int i0 = 0; i0 < n_ff; ++i0) {
    if (done[i0]) continue;
    const int x = ff_R[2 * i0], y = ff_R[2 * i0 + 1];
    auto set = [&](std::initializer_list<std::pair<int, double>> v) {
      std::fill(row.begin(), row.end(), 0.0);
      for (auto &p : v) row[p.first] = p.second;
    };
    if (x == 0 && y == 0) {
      done[i0] = true;
      set({{i0, 1.0}});
      emit(0);
      continue;
    }
    int m[4];
    bool axis = (x == 0 || y == 0), diag = (std::abs(x) == std::abs(y));
    if (!axis && !diag) return fail(nullptr, TUFRG_E_UNSUPPORTED, "orbits of eight form factors are not handled");
    const int d = axis ? std::abs(x) + std::abs(y) : std::abs(x);
    if (axis) {
      m[0] = at(d, 0), m[1] = at(-d, 0), m[2] = at(0, d), m[3] = at(0, -d);
    } else {
      m[0] = at(d, d), m[1] = at(-d, -d), m[2] = at(d, -d), m[3] = at(-d, d);
    }
    for (int k = 0; k < 4; ++k)
      if (m[k] < 0) return fail(nullptr, TUFRG_E_INVAL, "the form-factor set is not a union of C4v orbits");
    for (int k = 0; k < 4; ++k) done[m[k]] = true;
    set({{m[0], h}, {m[1], h}, {m[2], h}, {m[3], h}});
    emit(0);  // A1
    set({{m[0], h}, {m[1], h}, {m[2], -h}, {m[3], -h}});
    emit(axis ? 2 : 3);  // B1 (axis: cos x - cos y), B2 (diagonal: sin x sin y)
    if (axis) {
      set({{m[0], r2}, {m[1], -r2}});
      emit(4);  // x-like
      set({{m[2], r2}, {m[3], -r2}});
      emit(5);  // y-like
    } else {
      set({{m[0], h}, {m[2], h}, {m[3], -h}, {m[1], -h}});
      emit(4);  // x-like: (d,d) + (d,-d) - (-d,d) - (-d,-d)
      set({{m[0], h}, {m[3], h}, {m[2], -h}, {m[1], -h}});
      emit(5);  // y-like: (d,d) + (-d,d) - (d,-d) - (-d,-d)
    }
  }
  return TUFRG_OK;
}

extern "C" tufrg_status tufrg_ff_apply(tufrg_ctx *c, const tufrg_c64 *W, const tufrg_c64 *X, tufrg_c64 *Y,
                                       int32_t inverse) {
  if (!c) return fail(nullptr, TUFRG_E_INVAL, "null context");
  if (!W || is_device_ptr(W)) return fail(c, TUFRG_E_INVAL, "W must be a host array");
  if (!is_device_ptr(X) || !is_device_ptr(Y)) return fail(c, TUFRG_E_INVAL, "X and Y must be device pointers");
  const size_t n = (size_t)c->Nq * c->B * c->B;
  const uintptr_t x0 = (uintptr_t)X, x1 = x0 + n * sizeof(tufrg_c64), y0 = (uintptr_t)Y,
                  y1 = y0 + n * sizeof(tufrg_c64);
  if (y0 < x1 && x0 < y1) return fail(c, TUFRG_E_INVAL, "Y must not overlap X");
  const int nf = c->n_ff;
  std::vector<tufrg_c64> A((size_t)nf * nf);  // W, or W^H for the way back
  for (int i = 0; i < nf; ++i)
    for (int r = 0; r < nf; ++r) {
      const tufrg_c64 w = inverse ? W[(size_t)r * nf + i] : W[(size_t)i * nf + r];
      A[(size_t)i * nf + r] = inverse ? tufrg_c64{w.re, -w.im} : w;
    }
  if (!c->d_ffA) TRY(dalloc(c, &c->d_ffA, 2 * 25 * 25));
  HIPCHK(c, hipMemcpyAsync(c->d_ffA, A.data(), A.size() * sizeof(tufrg_c64), hipMemcpyHostToDevice, c->st));
  HIPCHK(c, launch_ff_apply(nf, c->no2, c->Nq, c->d_ffA, (const double *)X, (double *)Y, c->st));
  HIPCHK(c, hipStreamSynchronize(c->st));  // A lives on this host stack frame
  return TUFRG_OK;
}

extern "C" tufrg_status tufrg_project(tufrg_ctx *c, const tufrg_c64 *P, const tufrg_c64 *C, tufrg_c64 *VP,
                                      tufrg_c64 *VC) {
  if (!c) return fail(nullptr, TUFRG_E_INVAL, "null context");
  if (c->n_o == 1) return fail(c, TUFRG_E_UNSUPPORTED, "one-orbital contexts run the SU(2)-reduced calls");
  if (!is_device_ptr(P) || !is_device_ptr(C) || !is_device_ptr(VP) || !is_device_ptr(VC))
    return fail(c, TUFRG_E_INVAL, "P, C, VP, VC must be device pointers");
  return project_internal(c, (const double *)P, (const double *)C, (double *)VP, (double *)VC);
}

extern "C" tufrg_status tufrg_channel_d(tufrg_ctx *c, const tufrg_c64 *C, tufrg_c64 *D) {
  if (!c) return fail(nullptr, TUFRG_E_INVAL, "null context");
  if (c->n_o == 1) return fail(c, TUFRG_E_UNSUPPORTED, "one-orbital contexts run the SU(2)-reduced calls");
  if (!is_device_ptr(C) || !is_device_ptr(D)) return fail(c, TUFRG_E_INVAL, "C and D must be device pointers");
  const size_t bytes = (size_t)c->Nq * c->B * c->B * sizeof(tufrg_c64);
  const uintptr_t c0 = (uintptr_t)C, d0 = (uintptr_t)D;
  if (d0 < c0 + bytes && c0 < d0 + bytes) return fail(c, TUFRG_E_INVAL, "D must not overlap C");
  HIPCHK(c, launch_channel_d(c->n_o, c->B, c->Nq, (const double *)C, (double *)D, c->st));
  return TUFRG_OK;
}

extern "C" tufrg_status tufrg_project_static(tufrg_ctx *c, const tufrg_c64 *P, const tufrg_c64 *C, tufrg_c64 *VP,
                                             tufrg_c64 *VC) {
  if (!c) return fail(nullptr, TUFRG_E_INVAL, "null context");
  if (c->n_o == 1) return fail(c, TUFRG_E_UNSUPPORTED, "one-orbital contexts run the SU(2)-reduced calls");
  if (!is_device_ptr(P) || !is_device_ptr(C) || !is_device_ptr(VP) || !is_device_ptr(VC))
    return fail(c, TUFRG_E_INVAL, "P, C, VP, VC must be device pointers");
  int dev = -1;
  HIPCHK(c, hipGetDevice(&dev));
  if (dev != c->device) return fail(c, TUFRG_E_INVAL, "the context's device must be current");
  double *scr = g_scratch_ptr[dev];
  if (!scr) return fail(c, TUFRG_E_HIP, "static scratch not set up on this device");
  // one [2][nD][B][B] complex block each for the coefficients and the
  // gathers, the rest (at least as much, so at least one qx row of
  // [2][ny][B][B] with ny <= nD) for the transforms' intermediate
  const size_t unit = 2 * 2 * (size_t)c->nD * c->B * c->B;
  if (3 * unit > STATIC_SCRATCH_DOUBLES)
    return fail(c, TUFRG_E_UNSUPPORTED,
                "static scratch of 32 MiB holds 3 * 4 * n_dR * B^2 doubles at most; this setup needs " +
                    std::to_string(3 * unit * sizeof(double)) + " bytes");
  double *real = scr, *G = real + unit, *ws = G + unit;
  return project_with(c, (const double *)P, (const double *)C, (double *)VP, (double *)VC, ws,
                      STATIC_SCRATCH_DOUBLES - 2 * unit, real, G);
}

extern "C" tufrg_status tufrg_set_initial_c(tufrg_ctx *c, const tufrg_c64 *C0) {
  if (!c) return fail(nullptr, TUFRG_E_INVAL, "null context");
  if (c->n_o == 1) return fail(c, TUFRG_E_UNSUPPORTED, "one-orbital contexts run the SU(2)-reduced calls");
  if (!C0) {
    c->has_c0 = false;
    return TUFRG_OK;
  }
  if (!is_device_ptr(C0)) return fail(c, TUFRG_E_INVAL, "C0 must be a device pointer");
  const size_t n = 2 * (size_t)c->Nq * c->B * c->B;
  if (!c->d_c0) TRY(dalloc(c, &c->d_c0, n));
  if (!c->d_ceff) TRY(dalloc(c, &c->d_ceff, n));
  HIPCHK(c, hipMemcpyAsync(c->d_c0, C0, n * sizeof(double), hipMemcpyDeviceToDevice, c->st));
  c->has_c0 = true;
  return TUFRG_OK;
}

extern "C" tufrg_status tufrg_set_initial_p(tufrg_ctx *c, const tufrg_c64 *P0) {
  if (!c) return fail(nullptr, TUFRG_E_INVAL, "null context");
  if (c->n_o == 1) return fail(c, TUFRG_E_UNSUPPORTED, "one-orbital contexts run the SU(2)-reduced calls");
  if (!P0) {
    c->has_p0 = false;
    return TUFRG_OK;
  }
  if (!is_device_ptr(P0)) return fail(c, TUFRG_E_INVAL, "P0 must be a device pointer");
  const size_t n = 2 * (size_t)c->Nq * c->B * c->B;
  if (!c->d_p0) TRY(dalloc(c, &c->d_p0, n));
  if (!c->d_peff) TRY(dalloc(c, &c->d_peff, n));
  HIPCHK(c, hipMemcpyAsync(c->d_p0, P0, n * sizeof(double), hipMemcpyDeviceToDevice, c->st));
  c->has_p0 = true;
  return TUFRG_OK;
}

extern "C" tufrg_status tufrg_rhs(tufrg_ctx *c, double lambda, const tufrg_c64 *P, const tufrg_c64 *C, tufrg_c64 *dP,
                                  tufrg_c64 *dC) {
  if (!c) return fail(nullptr, TUFRG_E_INVAL, "null context");
  if (c->n_o == 1) return fail(c, TUFRG_E_UNSUPPORTED, "one-orbital contexts run the SU(2)-reduced calls");
  if (!(lambda > 0.0) || !std::isfinite(lambda)) return fail(c, TUFRG_E_INVAL, "lambda must be positive");
  if (!is_device_ptr(P) || !is_device_ptr(C) || !is_device_ptr(dP) || !is_device_ptr(dC))
    return fail(c, TUFRG_E_INVAL, "P, C, dP, dC must be device pointers");
  return rhs_internal(c, lambda, (const double *)P, (const double *)C, (double *)dP, (double *)dC, 1.0, 3u);
}

extern "C" tufrg_status tufrg_loops_compact(tufrg_ctx *c, double lambda, int32_t deriv, tufrg_c64 *Lc) {
  if (!c) return fail(nullptr, TUFRG_E_INVAL, "null context");
  if (!(lambda > 0.0) || !std::isfinite(lambda)) return fail(c, TUFRG_E_INVAL, "lambda must be positive");
  if (!is_device_ptr(Lc)) return fail(c, TUFRG_E_INVAL, "Lc must be a device pointer");
  TRY(compute_kval(c, lambda, deriv ? 1 : 0));
  return loops_range(c, lambda, deriv ? 1 : 0, 0, 2, 0, c->Nq, (double *)Lc);
}

extern "C" tufrg_status tufrg_dR(const tufrg_ctx *c, int32_t *dR) {
  if (!c || !dR) return fail(nullptr, TUFRG_E_INVAL, "null argument");
  for (size_t i = 0; i < c->dlist.size(); ++i) dR[i] = c->dlist[i];
  return TUFRG_OK;
}

static tufrg_status check_blocks(tufrg_ctx *c, int64_t n, const int32_t *q, const int32_t *ch, const int32_t *iD) {
  if (n < 0) return fail(c, TUFRG_E_INVAL, "negative block count");
  const bool lists = q || ch || iD;
  if (lists && (!is_device_ptr(q) || !is_device_ptr(ch) || !is_device_ptr(iD)))
    return fail(c, TUFRG_E_INVAL, "q, ch, iD must all be device pointers or all NULL");
  if (!lists && n > 2LL * c->Nq * c->nD) return fail(c, TUFRG_E_INVAL, "more blocks than 2 Nq n_dR");
  return TUFRG_OK;
}

extern "C" tufrg_status tufrg_sur_features(tufrg_ctx *c, int64_t n, const int32_t *q, const int32_t *ch,
                                          const int32_t *iD, double lambda, float *X) {
  if (!c) return fail(nullptr, TUFRG_E_INVAL, "null context");
  if (c->n_o == 1) return fail(c, TUFRG_E_UNSUPPORTED, "one-orbital contexts run the SU(2)-reduced calls");
  TRY(check_blocks(c, n, q, ch, iD));
  if (!(lambda > 0.0) || !std::isfinite(lambda)) return fail(c, TUFRG_E_INVAL, "lambda must be positive");
  if (n > 0 && !is_device_ptr(X)) return fail(c, TUFRG_E_INVAL, "X must be a device pointer");
  HIPCHK(c, launch_sur_features(n, q, ch, iD, c->Lq, c->nD, lambda, X, c->st));
  return TUFRG_OK;
}

extern "C" tufrg_status tufrg_sur_targets(tufrg_ctx *c, int64_t n, const int32_t *q, const int32_t *ch,
                                         const int32_t *iD, double scale, const tufrg_c64 *Lc, float *T,
                                         double *max_abs) {
  if (!c) return fail(nullptr, TUFRG_E_INVAL, "null context");
  if (c->n_o == 1) return fail(c, TUFRG_E_UNSUPPORTED, "one-orbital contexts run the SU(2)-reduced calls");
  TRY(check_blocks(c, n, q, ch, iD));
  if (!(scale > 0.0) || !std::isfinite(scale)) return fail(c, TUFRG_E_INVAL, "scale must be positive");
  if (n > 0 && (!is_device_ptr(Lc) || !is_device_ptr(T))) return fail(c, TUFRG_E_INVAL, "Lc, T must be device pointers");
  HIPCHK(c, launch_sur_targets(n, q, ch, iD, c->Nq, c->nD, c->no4, 1.0 / scale, (const double *)Lc, T, c->st));
  if (max_abs) {
    HIPCHK(c, hipMemsetAsync(c->d_sbits, 0, sizeof(unsigned long long), c->st));
    HIPCHK(c, launch_absmax_f32(n * 2 * c->no4, T, (unsigned int *)c->d_sbits, c->st));
    HIPCHK(c, hipMemcpyAsync(c->h_sbits, c->d_sbits, sizeof(unsigned long long), hipMemcpyDeviceToHost, c->st));
    HIPCHK(c, hipStreamSynchronize(c->st));
    float f;
    const unsigned int u = (unsigned int)(c->h_sbits[0] & 0xffffffffu);
    std::memcpy(&f, &u, sizeof(f));
    *max_abs = (double)f * scale;
  }
  return TUFRG_OK;
}

extern "C" tufrg_status tufrg_sur_attach(tufrg_ctx *c, tufrg_mlp *net, int32_t n_scale, const double *lam_tab,
                                        const double *scale_tab) {
  if (!c) return fail(nullptr, TUFRG_E_INVAL, "null context");
  if (c->n_o == 1) return fail(c, TUFRG_E_UNSUPPORTED, "one-orbital contexts run the SU(2)-reduced calls");
  if (!net) {
    c->sur = nullptr;
    return TUFRG_OK;
  }
  if (mlp_n_in(net) != 11 + c->nD || mlp_n_out(net) != 2 * c->no4)
    return fail(c, TUFRG_E_INVAL, "network widths must be 11 + n_dR inputs and 2 n_o^4 outputs");
  if (mlp_stream(net) != c->st) return fail(c, TUFRG_E_INVAL, "network and context must share one stream");
  if (n_scale < 1 || !lam_tab || !scale_tab) return fail(c, TUFRG_E_INVAL, "need a scale table");
  std::vector<std::pair<double, double>> tab;
  for (int i = 0; i < n_scale; ++i) {
    if (!(lam_tab[i] > 0.0) || !(scale_tab[i] > 0.0) || !std::isfinite(lam_tab[i]) || !std::isfinite(scale_tab[i]))
      return fail(c, TUFRG_E_INVAL, "scale table entries must be positive and finite");
    tab.emplace_back(std::log(lam_tab[i]), std::log(scale_tab[i]));
  }
  std::sort(tab.begin(), tab.end());
  for (size_t i = 1; i < tab.size(); ++i)
    if (tab[i].first == tab[i - 1].first) return fail(c, TUFRG_E_INVAL, "repeated scale in the table");
  c->sur_lnlam.clear();
  c->sur_lns.clear();
  for (auto &t : tab) {
    c->sur_lnlam.push_back(t.first);
    c->sur_lns.push_back(t.second);
  }
  c->sur = net;
  return TUFRG_OK;
}

extern "C" tufrg_status tufrg_sur_loops(tufrg_ctx *c, double lambda, tufrg_c64 *Lc) {
  if (!c) return fail(nullptr, TUFRG_E_INVAL, "null context");
  if (c->n_o == 1) return fail(c, TUFRG_E_UNSUPPORTED, "one-orbital contexts run the SU(2)-reduced calls");
  if (!c->sur) return fail(c, TUFRG_E_INVAL, "no network attached");
  if (!(lambda > 0.0) || !std::isfinite(lambda)) return fail(c, TUFRG_E_INVAL, "lambda must be positive");
  if (!is_device_ptr(Lc)) return fail(c, TUFRG_E_INVAL, "Lc must be a device pointer");
  return sur_loops_internal(c, lambda, (double *)Lc);
}

// ---------------------------------------------------------------------------
// flow

static tufrg_status read_reduce(tufrg_ctx *c, double *val, bool *bad) {
  HIPCHK(c, hipMemcpyAsync(c->h_bits, c->d_bits, sizeof(unsigned long long), hipMemcpyDeviceToHost, c->st));
  HIPCHK(c, hipMemcpyAsync(c->h_flag, c->d_flag, sizeof(unsigned int), hipMemcpyDeviceToHost, c->st));
  HIPCHK(c, hipStreamSynchronize(c->st));
  unsigned long long b = c->h_bits[0];
  double v;
  std::memcpy(&v, &b, sizeof(v));
  *val = v;
  *bad = c->h_flag[0] != 0;
  return TUFRG_OK;
}

static tufrg_status state_max(tufrg_ctx *c, const double *P, const double *C, double *m, bool *bad) {
  const long long n = (long long)c->Nq * c->B * c->B;
  HIPCHK(c, launch_clear_reduce(c->d_bits, c->d_flag, c->st));
  HIPCHK(c, launch_axpy_max(n, P, 0.0, nullptr, nullptr, c->d_bits, c->d_flag, c->st));
  HIPCHK(c, launch_axpy_max(n, C, 0.0, nullptr, nullptr, c->d_bits, c->d_flag, c->st));
  return read_reduce(c, m, bad);
}

static double lambda_c_interp(double l0, double m0, double l1, double m1, double vmax) {
  const double t = (vmax - m0) / (m1 - m0);
  return std::exp(std::log(l0) + t * (std::log(l1) - std::log(l0)));
}

// ---------------------------------------------------------------------------
// Euler steps in HIP graphs

static constexpr int MAX_GRAPH_STEPS = 64;

static double euler_lambda(const tufrg_flow_opts *o, int i) {
  if (i >= o->n_steps) return o->lambda_end;
  return o->lambda0 * std::pow(o->lambda_end / o->lambda0, (double)i / o->n_steps);
}

// workspaces of graph stepping (allocated on first use, outside any capture)
static tufrg_status graph_prepare(tufrg_ctx *c) {
  if (!c->gst) {
    if (c->st) {
      c->gst = c->st;
    } else {
      // the null stream cannot be captured: a private stream of default
      // priority, ordered against the caller's work by the flow's own
      // synchronisations
      HIPCHK(c, hipStreamCreateWithFlags(&c->gst, hipStreamDefault));
      c->own_gst = true;
    }
  }
  if (!c->d_gbits) TRY(dalloc(c, &c->d_gbits, MAX_GRAPH_STEPS));
  if (!c->d_gflag) TRY(dalloc(c, &c->d_gflag, MAX_GRAPH_STEPS));
  if (!c->h_gbits)
    HIPCHK(c, hipHostMalloc((void **)&c->h_gbits, MAX_GRAPH_STEPS * sizeof(unsigned long long), hipHostMallocDefault));
  if (!c->h_gflag)
    HIPCHK(c, hipHostMalloc((void **)&c->h_gflag, MAX_GRAPH_STEPS * sizeof(unsigned int), hipHostMallocDefault));
  const size_t ns = 2 * (size_t)c->B * c->B * c->Nq;
  if (!c->d_bkP) TRY(dalloc(c, &c->d_bkP, ns));
  if (!c->d_bkC) TRY(dalloc(c, &c->d_bkC, ns));
  return TUFRG_OK;
}

// enqueue Euler steps [i0, i0 + g) of one context on its stream, step j's max
// coupling and non-finite flag into slot j (every call is a kernel launch, so
// the sequence can be captured)
static tufrg_status enqueue_euler_steps(tufrg_ctx *c, const tufrg_flow_opts *o, double *P, double *C, int i0, int g,
                                        unsigned mask) {
  const long long ncx = (long long)c->B * c->B * c->Nq;
  for (int j = 0; j < g; ++j) {
    const double l0 = euler_lambda(o, i0 + j), l1 = euler_lambda(o, i0 + j + 1);
    TRY(rhs_internal(c, l0, P, C, c->d_dP, c->d_dC, 1.0, mask));
    HIPCHK(c, launch_clear_reduce(c->d_gbits + j, c->d_gflag + j, c->st));
    HIPCHK(c, launch_axpy_max(ncx, P, l1 - l0, c->d_dP, P, c->d_gbits + j, c->d_gflag + j, c->st));
    HIPCHK(c, launch_axpy_max(ncx, C, l1 - l0, c->d_dC, C, c->d_gbits + j, c->d_gflag + j, c->st));
  }
  return TUFRG_OK;
}

// capture g Euler steps from i0 into the context's executable graph (updated
// in place when the topology is unchanged), then launch it after saving the
// state; the slots are copied to the host and the stream synchronised
static tufrg_status run_euler_graph(tufrg_ctx *c, const tufrg_flow_opts *o, double *P, double *C, int i0, int g,
                                    unsigned mask) {
  const size_t bytes = 2 * sizeof(double) * (size_t)c->B * c->B * c->Nq;
  hipStream_t saved = c->st;
  c->st = c->gst;
  hipError_t e = hipStreamBeginCapture(c->st, hipStreamCaptureModeThreadLocal);
  if (e != hipSuccess) {
    c->st = saved;
    (void)hipGetLastError();
    return fail(c, TUFRG_E_HIP, std::string("hipStreamBeginCapture: ") + hipGetErrorString(e));
  }
  // the caller counts the steps of an accepted graph itself
  tufrg_flow_result *fres = c->fres;
  c->fres = nullptr;
  const tufrg_status s = enqueue_euler_steps(c, o, P, C, i0, g, mask);
  c->fres = fres;
  hipGraph_t graph = nullptr;
  e = hipStreamEndCapture(c->st, &graph);
  c->st = saved;
  if (s != TUFRG_OK || e != hipSuccess) {
    if (graph) (void)hipGraphDestroy(graph);
    (void)hipGetLastError();
    return s != TUFRG_OK ? s : fail(c, TUFRG_E_HIP, std::string("hipStreamEndCapture: ") + hipGetErrorString(e));
  }
  bool updated = false;
  if (c->gexec) {
    hipGraphNode_t err_node = nullptr;
    hipGraphExecUpdateResult res = hipGraphExecUpdateError;
    updated = hipGraphExecUpdate(c->gexec, graph, &err_node, &res) == hipSuccess && res == hipGraphExecUpdateSuccess;
    if (!updated) {
      (void)hipGetLastError();
      (void)hipGraphExecDestroy(c->gexec);
      c->gexec = nullptr;
    }
  }
  if (!updated) {
    e = hipGraphInstantiate(&c->gexec, graph, nullptr, nullptr, 0);
    if (e != hipSuccess) {
      c->gexec = nullptr;
      (void)hipGraphDestroy(graph);
      (void)hipGetLastError();
      return fail(c, TUFRG_E_HIP, std::string("hipGraphInstantiate: ") + hipGetErrorString(e));
    }
  }
  (void)hipGraphDestroy(graph);
  HIPCHK(c, hipMemcpyAsync(c->d_bkP, P, bytes, hipMemcpyDeviceToDevice, c->gst));
  HIPCHK(c, hipMemcpyAsync(c->d_bkC, C, bytes, hipMemcpyDeviceToDevice, c->gst));
  HIPCHK(c, hipGraphLaunch(c->gexec, c->gst));
  HIPCHK(c, hipMemcpyAsync(c->h_gbits, c->d_gbits, g * sizeof(unsigned long long), hipMemcpyDeviceToHost, c->gst));
  HIPCHK(c, hipMemcpyAsync(c->h_gflag, c->d_gflag, g * sizeof(unsigned int), hipMemcpyDeviceToHost, c->gst));
  HIPCHK(c, hipStreamSynchronize(c->gst));
  return TUFRG_OK;
}

// undo the steps of the last graph: the state saved at its start
static tufrg_status restore_graph_state(tufrg_ctx *c, double *P, double *C) {
  const size_t bytes = 2 * sizeof(double) * (size_t)c->B * c->B * c->Nq;
  HIPCHK(c, hipMemcpyAsync(P, c->d_bkP, bytes, hipMemcpyDeviceToDevice, c->gst));
  HIPCHK(c, hipMemcpyAsync(C, c->d_bkC, bytes, hipMemcpyDeviceToDevice, c->gst));
  HIPCHK(c, hipStreamSynchronize(c->gst));
  return TUFRG_OK;
}

static const double DP_C[7] = {0.0, 1.0 / 5, 3.0 / 10, 4.0 / 5, 8.0 / 9, 1.0, 1.0};
static const double DP_A[7][6] = {
    {0, 0, 0, 0, 0, 0},
    {1.0 / 5, 0, 0, 0, 0, 0},
    {3.0 / 40, 9.0 / 40, 0, 0, 0, 0},
    {44.0 / 45, -56.0 / 15, 32.0 / 9, 0, 0, 0},
    {19372.0 / 6561, -25360.0 / 2187, 64448.0 / 6561, -212.0 / 729, 0, 0},
    {9017.0 / 3168, -355.0 / 33, 46732.0 / 5247, 49.0 / 176, -5103.0 / 18656, 0},
    {35.0 / 384, 0.0, 500.0 / 1113, 125.0 / 192, -2187.0 / 6784, 11.0 / 84}};
static const double DP_B5[7] = {35.0 / 384, 0.0, 500.0 / 1113, 125.0 / 192, -2187.0 / 6784, 11.0 / 84, 0.0};
static const double DP_B4[7] = {5179.0 / 57600, 0.0, 7571.0 / 16695, 393.0 / 640, -92097.0 / 339200, 187.0 / 2100,
                                1.0 / 40};

extern "C" tufrg_status tufrg_flow(tufrg_ctx *c, const tufrg_flow_opts *o, tufrg_c64 *Pu, tufrg_c64 *Cu,
                                   tufrg_flow_result *res) {
  if (!c) return fail(nullptr, TUFRG_E_INVAL, "null context");
  if (c->n_o == 1) return fail(c, TUFRG_E_UNSUPPORTED, "one-orbital contexts run the SU(2)-reduced calls");
  if (!o || !res) return fail(c, TUFRG_E_INVAL, "null options or result");
  if (!is_device_ptr(Pu) || !is_device_ptr(Cu)) return fail(c, TUFRG_E_INVAL, "P, C must be device pointers");
  if (!(o->lambda0 > 0.0) || !(o->lambda_end > 0.0) || !(o->lambda_end < o->lambda0))
    return fail(c, TUFRG_E_INVAL, "need lambda0 > lambda_end > 0");
  if (o->n_steps < 0) return fail(c, TUFRG_E_INVAL, "n_steps must be >= 0");
  const unsigned mask = o->channel_mask & 3u;
  if (!mask) return fail(c, TUFRG_E_INVAL, "channel_mask selects no channel");
  if (o->surrogate) {
    if (!c->sur) return fail(c, TUFRG_E_INVAL, "surrogate requested but no network attached");
    if (!(o->sample_frac > 0.0 && o->sample_frac <= 1.0)) return fail(c, TUFRG_E_INVAL, "sample_frac must be in (0, 1]");
    if (!(o->sur_tol > 0.0)) return fail(c, TUFRG_E_INVAL, "sur_tol must be positive");
  }
  struct FlowGuard {
    tufrg_ctx *c;
    ~FlowGuard() {
      c->fopts = nullptr;
      c->fres = nullptr;
    }
  } guard{c};
  double *P = (double *)Pu, *C = (double *)Cu;
  const size_t BB = (size_t)c->B * c->B;
  const size_t ns = 2 * BB * c->Nq;  // doubles per state
  const long long ncx = (long long)BB * c->Nq;
  std::memset(res, 0, sizeof(*res));
  res->lambda_stop = o->lambda_end;
  double m_prev = 0.0;
  bool bad = false;
  TRY(state_max(c, P, C, &m_prev, &bad));
  if (bad) return fail(c, TUFRG_E_NONFINITE, "non-finite initial state");
  double lam_prev = o->lambda0;
  c->fopts = o;
  c->fres = res;
  c->cur_max = m_prev;

  if (o->n_steps > 0) {
    if (!c->d_dP) {
      TRY(dalloc(c, &c->d_dP, ns));
      TRY(dalloc(c, &c->d_dC, ns));
    }
    const int n = o->n_steps;
    // graph stepping: plain loops of both channels, no per-step callback or
    // timers; the first step runs directly (it allocates lazy workspaces)
    const int G = (o->graph_steps > 1 && !o->surrogate && mask == 3u && !o->on_step && !c->timing)
                      ? std::min(o->graph_steps, MAX_GRAPH_STEPS)
                      : 0;
    if (G) TRY(graph_prepare(c));
    int replay_to = -1;  // after an undone graph: direct steps up to this one
    for (int i = 0; i < n; ++i) {
      if (G && i > 0 && i > replay_to) {
        int g = std::min(G, n - i);
        if (o->max_steps > 0) g = std::min(g, o->max_steps - res->n_steps);
        if (g > 1) {
          TRY(run_euler_graph(c, o, P, C, i, g, mask));
          int stop = -1;
          for (int j = 0; j < g && stop < 0; ++j) {
            double mx;
            std::memcpy(&mx, &c->h_gbits[j], sizeof(mx));
            if (c->h_gflag[j] || mx > o->v_max) stop = j;
          }
          if (stop >= 0) {
            // a step inside the graph diverged (or went non-finite): undo the
            // graph and take its steps one by one up to that step
            TRY(restore_graph_state(c, P, C));
            replay_to = i + stop;
          } else {
            for (int j = 0; j < g; ++j) {
              double mx;
              std::memcpy(&mx, &c->h_gbits[j], sizeof(mx));
              res->n_rhs++;
              res->n_plain++;
              res->n_steps++;
              res->lambda_stop = euler_lambda(o, i + j + 1);
              res->max_coupling = mx;
              c->cur_max = mx;
              lam_prev = res->lambda_stop;
              m_prev = mx;
            }
            i += g - 1;
            if (o->max_steps > 0 && res->n_steps >= o->max_steps) break;
            continue;
          }
        }
      }
      const double l0 = euler_lambda(o, i), l1 = euler_lambda(o, i + 1);
      TRY(rhs_internal(c, l0, P, C, c->d_dP, c->d_dC, 1.0, mask));
      res->n_rhs++;
      HIPCHK(c, launch_clear_reduce(c->d_bits, c->d_flag, c->st));
      HIPCHK(c, launch_axpy_max(ncx, P, l1 - l0, c->d_dP, P, c->d_bits, c->d_flag, c->st));
      HIPCHK(c, launch_axpy_max(ncx, C, l1 - l0, c->d_dC, C, c->d_bits, c->d_flag, c->st));
      double mx;
      TRY(read_reduce(c, &mx, &bad));
      if (bad) return fail(c, TUFRG_E_NONFINITE, "non-finite state after Euler step " + std::to_string(i));
      res->n_steps++;
      res->lambda_stop = l1;
      res->max_coupling = mx;
      c->cur_max = mx;
      if (mx > o->v_max) {
        res->diverged = 1;
        res->lambda_c = lambda_c_interp(lam_prev, m_prev, l1, mx, o->v_max);
        break;
      }
      if (o->on_step && o->on_step(o->user, i, l1, mx)) {
        res->stopped_by_callback = 1;
        break;
      }
      if (o->max_steps > 0 && res->n_steps >= o->max_steps) break;
      lam_prev = l1;
      m_prev = mx;
    }
    return TUFRG_OK;
  }

  // Dormand-Prince 5(4) in l = ln Lambda, dX/dl = Lambda dX/dLambda
  while (c->d_stage.size() < 16) {  // resumes after a failed allocation
    double *p = nullptr;
    TRY(dalloc(c, &p, ns));
    c->d_stage.push_back(p);
  }
  double *kP[7], *kC[7];
  for (int j = 0; j < 7; ++j) {
    kP[j] = c->d_stage[j];
    kC[j] = c->d_stage[7 + j];
  }
  double *YP = c->d_stage[14], *YC = c->d_stage[15];
  double l = std::log(o->lambda0);
  const double l_end = std::log(o->lambda_end);
  double h = -std::fabs(o->h0 > 0 ? o->h0 : 0.05);
  TRY(rhs_internal(c, std::exp(l), P, C, kP[0], kC[0], std::exp(l), mask));
  res->n_rhs++;
  double ecoef[7];
  for (int j = 0; j < 7; ++j) ecoef[j] = DP_B5[j] - DP_B4[j];
  while (l - l_end > 1e-14) {
    if (l + h < l_end) h = l_end - l;
    for (int s = 1; s < 7; ++s) {
      HIPCHK(c, launch_lincomb((long long)ns, P, s, kP, DP_A[s], h, YP, c->st));
      HIPCHK(c, launch_lincomb((long long)ns, C, s, kC, DP_A[s], h, YC, c->st));
      const double ls = std::exp(l + DP_C[s] * h);
      TRY(rhs_internal(c, ls, YP, YC, kP[s], kC[s], ls, mask));
      res->n_rhs++;
    }
    HIPCHK(c, launch_clear_reduce(c->d_bits, c->d_flag, c->st));
    HIPCHK(c, launch_dp_error((long long)ns, P, YP, 7, kP, ecoef, h, o->rtol, o->atol, c->d_bits, c->d_flag, c->st));
    HIPCHK(c, launch_dp_error((long long)ns, C, YC, 7, kC, ecoef, h, o->rtol, o->atol, c->d_bits, c->d_flag, c->st));
    double err;
    TRY(read_reduce(c, &err, &bad));
    if (bad) return fail(c, TUFRG_E_NONFINITE, "non-finite error estimate at step " + std::to_string(res->n_steps));
    const double fac = err == 0.0 ? 5.0 : std::min(5.0, std::max(0.2, 0.9 * std::pow(err, -0.2)));
    if (err <= 1.0) {
      l += h;
      HIPCHK(c, hipMemcpyAsync(P, YP, ns * sizeof(double), hipMemcpyDeviceToDevice, c->st));
      HIPCHK(c, hipMemcpyAsync(C, YC, ns * sizeof(double), hipMemcpyDeviceToDevice, c->st));
      std::swap(kP[0], kP[6]);
      std::swap(kC[0], kC[6]);
      double mx;
      TRY(state_max(c, P, C, &mx, &bad));
      if (bad) return fail(c, TUFRG_E_NONFINITE, "non-finite state after step " + std::to_string(res->n_steps));
      const double lam = std::exp(l);
      res->n_steps++;
      res->lambda_stop = lam;
      res->max_coupling = mx;
      c->cur_max = mx;
      if (mx > o->v_max) {
        res->diverged = 1;
        res->lambda_c = lambda_c_interp(lam_prev, m_prev, lam, mx, o->v_max);
        break;
      }
      if (o->on_step && o->on_step(o->user, res->n_steps - 1, lam, mx)) {
        res->stopped_by_callback = 1;
        break;
      }
      if (o->max_steps > 0 && res->n_steps >= o->max_steps) break;
      lam_prev = lam;
      m_prev = mx;
    } else {
      res->n_reject++;
    }
    h *= fac;
    if (std::fabs(h) < 1e-12) return fail(c, TUFRG_E_STEPSIZE, "step size underflow");
  }
  if (l - l_end <= 1e-14) res->lambda_stop = o->lambda_end;
  return TUFRG_OK;
}

// ---------------------------------------------------------------------------
// SU(2)-reduced flows (one orbital per site)

static tufrg_status su2_prepare(tufrg_ctx *c) {
  const size_t BB = (size_t)c->B * c->B, st = 2 * BB * c->Nq, rs = 2 * 2 * (size_t)c->nD * BB;
  if (!c->d_s_px) TRY(dalloc(c, &c->d_s_px, st));
  if (!c->d_s_rA) TRY(dalloc(c, &c->d_s_rA, rs));
  if (!c->d_s_rB) TRY(dalloc(c, &c->d_s_rB, rs));
  if (!c->d_s_G3) TRY(dalloc(c, &c->d_s_G3, 2 * 3 * (size_t)c->nD * BB));
  if (!c->d_s_Vd) TRY(dalloc(c, &c->d_s_Vd, st));
  if (!c->d_s_Vax) TRY(dalloc(c, &c->d_s_Vax, st));
  return TUFRG_OK;
}

// (dp, dc, dd) of the reduced state (p, c, d) at scale lam: one-band loops,
// the reduced projected vertices a~, c~, d~ (the q -> rho transforms of p, c,
// p^x and d, the gathers, the assembly with the onsite v), a~^x, the products
static tufrg_status su2_rhs_internal(tufrg_ctx *c, double lam, const double *p, const double *cc, const double *d,
                                     double *dp, double *dc, double *dd) {
  TRY(su2_prepare(c));
  TRY(compute_loops(c, lam, 1, 0, 2));
  ProjArgs a = proj_args(c);
  HIPCHK(c, timer_mark(c, TUFRG_TIMER_PROJECT));
  HIPCHK(c, launch_su2_exch(c->n_ff, c->Nq, c->Lq, c->d_ff, c->d_fneg, c->d_twq, p, c->d_s_px, c->st));
  HIPCHK(c, launch_ft(a, p, cc, c->d_ftpart, c->proj_ws, c->d_s_rA, c->st));
  HIPCHK(c, launch_ft(a, c->d_s_px, d, c->d_ftpart, c->proj_ws, c->d_s_rB, c->st));
  HIPCHK(c, launch_su2_gather(c->B, c->nD, c->d_ff, c->d_dlist, c->d_ffgrid, c->d_dgrid, c->d_s_rA, c->d_s_rB,
                              c->d_s_G3, c->st));
  // a~ and c~ from (p, c) with the gathers 0, 1; d~ from d with gather 2 (v in every (0,0) entry)
  HIPCHK(c, launch_assemble(a, p, cc, c->d_s_G3, c->d_v0p, c->d_v0c, c->d_VP, c->d_VC, c->d_ftpart, c->proj_ws,
                            c->st));
  HIPCHK(c, launch_assemble(a, d, d, c->d_s_G3 + 2 * 2 * (size_t)c->nD * c->B * c->B, c->d_v0p, c->d_v0p,
                            c->d_s_Vd, nullptr, c->d_ftpart, c->proj_ws, c->st, 1));
  HIPCHK(c, launch_su2_exch(c->n_ff, c->Nq, c->Lq, c->d_ff, c->d_fneg, c->d_twq, c->d_VP, c->d_s_Vax, c->st));
  HIPCHK(c, timer_mark(c, TUFRG_TIMER_PROJECT));
  HIPCHK(c, timer_mark(c, TUFRG_TIMER_BUNDLE));
  HIPCHK(c, launch_su2_bundle(c->B, c->Nq, c->nD, c->d_didx, c->d_loop, c->d_VP, c->d_s_Vax, c->d_VC, c->d_s_Vd, 1.0,
                              dp, dc, dd, c->st));
  HIPCHK(c, timer_mark(c, TUFRG_TIMER_BUNDLE));
  return TUFRG_OK;
}

static tufrg_status su2_state_check(tufrg_ctx *c, const void *const *arrs, int n) {
  if (c->n_o != 1) return fail(c, TUFRG_E_UNSUPPORTED, "the SU(2)-reduced calls need a one-orbital context");
  for (int i = 0; i < n; ++i)
    if (!is_device_ptr(arrs[i])) return fail(c, TUFRG_E_INVAL, "every state array must be device memory");
  return TUFRG_OK;
}

extern "C" tufrg_status tufrg_su2_rhs(tufrg_ctx *c, double lambda, const tufrg_c64 *p, const tufrg_c64 *cc,
                                      const tufrg_c64 *d, tufrg_c64 *dp, tufrg_c64 *dc, tufrg_c64 *dd) {
  if (!c) return fail(nullptr, TUFRG_E_INVAL, "null context");
  if (!(lambda > 0.0) || !std::isfinite(lambda)) return fail(c, TUFRG_E_INVAL, "lambda must be positive");
  const void *arrs[6] = {p, cc, d, dp, dc, dd};
  TRY(su2_state_check(c, arrs, 6));
  return su2_rhs_internal(c, lambda, (const double *)p, (const double *)cc, (const double *)d, (double *)dp,
                          (double *)dc, (double *)dd);
}

extern "C" tufrg_status tufrg_su2_flow(tufrg_ctx *c, const tufrg_flow_opts *o, tufrg_c64 *pu, tufrg_c64 *cu,
                                       tufrg_c64 *du, tufrg_flow_result *res) {
  if (!c) return fail(nullptr, TUFRG_E_INVAL, "null context");
  if (!o || !res) return fail(c, TUFRG_E_INVAL, "null options or result");
  const void *arrs[3] = {pu, cu, du};
  TRY(su2_state_check(c, arrs, 3));
  if (!(o->lambda0 > 0.0) || !(o->lambda_end > 0.0) || !(o->lambda_end < o->lambda0))
    return fail(c, TUFRG_E_INVAL, "need lambda0 > lambda_end > 0");
  if (o->n_steps < 1) return fail(c, TUFRG_E_UNSUPPORTED, "the SU(2)-reduced flow takes Euler steps (n_steps >= 1)");
  if (o->surrogate || (o->channel_mask & 3u) != 3u || o->graph_steps > 1)
    return fail(c, TUFRG_E_UNSUPPORTED, "the SU(2)-reduced flow runs plain loops, all channels, no graphs");
  double *p = (double *)pu, *cc = (double *)cu, *d = (double *)du;
  const long long ncx = (long long)c->Nq * c->B * c->B;
  std::memset(res, 0, sizeof(*res));
  res->lambda_stop = o->lambda_end;
  if (!c->d_dP) {
    TRY(dalloc(c, &c->d_dP, 2 * (size_t)ncx));
    TRY(dalloc(c, &c->d_dC, 2 * (size_t)ncx));
  }
  if (!c->d_s_dd) TRY(dalloc(c, &c->d_s_dd, 2 * (size_t)ncx));
  auto maxof = [&](double h, const double *dx1, const double *dx2, const double *dx3, double *m, bool *bad) {
    HIPCHK(c, launch_clear_reduce(c->d_bits, c->d_flag, c->st));
    HIPCHK(c, launch_axpy_max(ncx, p, h, dx1, dx1 ? p : nullptr, c->d_bits, c->d_flag, c->st));
    HIPCHK(c, launch_axpy_max(ncx, cc, h, dx2, dx2 ? cc : nullptr, c->d_bits, c->d_flag, c->st));
    HIPCHK(c, launch_axpy_max(ncx, d, h, dx3, dx3 ? d : nullptr, c->d_bits, c->d_flag, c->st));
    return read_reduce(c, m, bad);
  };
  double m_prev = 0.0;
  bool bad = false;
  TRY(maxof(0.0, nullptr, nullptr, nullptr, &m_prev, &bad));
  if (bad) return fail(c, TUFRG_E_NONFINITE, "non-finite initial state");
  double lam_prev = o->lambda0;
  for (int i = 0; i < o->n_steps; ++i) {
    const double l0 = euler_lambda(o, i), l1 = euler_lambda(o, i + 1);
    TRY(su2_rhs_internal(c, l0, p, cc, d, c->d_dP, c->d_dC, c->d_s_dd));
    res->n_rhs++;
    res->n_plain++;
    double mx;
    TRY(maxof(l1 - l0, c->d_dP, c->d_dC, c->d_s_dd, &mx, &bad));
    if (bad) return fail(c, TUFRG_E_NONFINITE, "non-finite state after Euler step " + std::to_string(i));
    res->n_steps++;
    res->lambda_stop = l1;
    res->max_coupling = mx;
    if (mx > o->v_max) {
      res->diverged = 1;
      res->lambda_c = lambda_c_interp(lam_prev, m_prev, l1, mx, o->v_max);
      break;
    }
    if (o->on_step && o->on_step(o->user, i, l1, mx)) {
      res->stopped_by_callback = 1;
      break;
    }
    if (o->max_steps > 0 && res->n_steps >= o->max_steps) break;
    lam_prev = l1;
    m_prev = mx;
  }
  return TUFRG_OK;
}

// ---------------------------------------------------------------------------
// batches of independent instances (lockstep Euler)

struct tufrg_batch {
  std::vector<tufrg_ctx *> ctx;
  std::vector<hipStream_t> streams;  // owned, default priority
  std::string err;
  // lockstep steps in HIP graphs: the executable graph and the fork/join events
  hipGraphExec_t gexec = nullptr;
  std::vector<hipEvent_t> events;
  // fused loop launches: instance descriptors (pinned host and device) and
  // the join/fork events around them
  No2Inst *desc_h = nullptr, *desc_d = nullptr;
  std::vector<hipEvent_t> fev;
};

static thread_local std::string g_batch_err;

static tufrg_status bfail(tufrg_batch *b, tufrg_status s, const std::string &m) {
  if (b)
    b->err = m;
  else
    g_batch_err = m;
  return s;
}

static void batch_free(tufrg_batch *b) {
  if (b->gexec) (void)hipGraphExecDestroy(b->gexec);
  b->gexec = nullptr;
  for (hipEvent_t e : b->events) (void)hipEventDestroy(e);
  b->events.clear();
  for (hipEvent_t e : b->fev) (void)hipEventDestroy(e);
  b->fev.clear();
  if (b->desc_h) (void)hipHostFree(b->desc_h);
  if (b->desc_d) (void)hipFree(b->desc_d);
  b->desc_h = nullptr;
  b->desc_d = nullptr;
  for (tufrg_ctx *c : b->ctx) tufrg_destroy(c);
  for (hipStream_t s : b->streams) (void)hipStreamDestroy(s);
  b->ctx.clear();
  b->streams.clear();
}

extern "C" const char *tufrg_batch_last_error(const tufrg_batch *b) {
  return b ? b->err.c_str() : g_batch_err.c_str();
}

extern "C" tufrg_status tufrg_batch_create(int32_t n_inst, const tufrg_model *models, const tufrg_setup *setups,
                                           int32_t n_streams, tufrg_batch **out) {
  if (!out) return bfail(nullptr, TUFRG_E_INVAL, "null output pointer");
  *out = nullptr;
  if (n_inst < 1 || !models || !setups) return bfail(nullptr, TUFRG_E_INVAL, "need n_inst >= 1 models and setups");
  if (n_streams < 1 || n_streams > 8) return bfail(nullptr, TUFRG_E_INVAL, "n_streams must be in [1, 8]");
  for (int i = 0; i < n_inst; ++i)
    if (models[i].n_orb == 1)
      return bfail(nullptr, TUFRG_E_UNSUPPORTED, "batches run spinful instances (n_orb = 2 or 6)");
  tufrg_batch *b = new tufrg_batch();
  for (int i = 0; i < std::min(n_streams, n_inst); ++i) {
    hipStream_t s;
    if (hipStreamCreateWithFlags(&s, hipStreamNonBlocking) != hipSuccess) {
      (void)hipGetLastError();
      batch_free(b);
      delete b;
      return bfail(nullptr, TUFRG_E_HIP, "hipStreamCreate failed");
    }
    b->streams.push_back(s);
  }
  for (int i = 0; i < n_inst; ++i) {
    tufrg_ctx *c = nullptr;
    const tufrg_status s = tufrg_create(&models[i], &setups[i], b->streams[i % b->streams.size()], &c);
    if (s != TUFRG_OK) {
      const std::string m = "instance " + std::to_string(i) + ": " + tufrg_last_error(nullptr);
      batch_free(b);
      delete b;
      return bfail(nullptr, s, m);
    }
    b->ctx.push_back(c);
  }
  *out = b;
  return TUFRG_OK;
}

extern "C" tufrg_status tufrg_batch_destroy(tufrg_batch *b) {
  if (!b) return TUFRG_OK;
  batch_free(b);
  delete b;
  return TUFRG_OK;
}

extern "C" tufrg_status tufrg_batch_dims(const tufrg_batch *b, int32_t inst, int32_t *B, int32_t *Nq, int32_t *Nf,
                                         int32_t *n_dR) {
  if (!b || inst < 0 || inst >= (int)b->ctx.size()) return bfail(nullptr, TUFRG_E_INVAL, "bad instance");
  return tufrg_dims(b->ctx[inst], B, Nq, Nf, n_dR);
}

extern "C" tufrg_status tufrg_batch_flow(tufrg_batch *b, const tufrg_flow_opts *o, tufrg_c64 *const *P,
                                         tufrg_c64 *const *C, tufrg_flow_result *res) {
  if (!b) return bfail(nullptr, TUFRG_E_INVAL, "null batch");
  if (!o || !P || !C || !res) return bfail(b, TUFRG_E_INVAL, "null argument");
  if (o->n_steps <= 0) return bfail(b, TUFRG_E_UNSUPPORTED, "batched flows are lockstep Euler (n_steps > 0)");
  if (o->surrogate) return bfail(b, TUFRG_E_UNSUPPORTED, "no surrogate in batched flows");
  if (!(o->lambda0 > 0.0) || !(o->lambda_end > 0.0) || !(o->lambda_end < o->lambda0))
    return bfail(b, TUFRG_E_INVAL, "need lambda0 > lambda_end > 0");
  const unsigned mask = o->channel_mask & 3u;
  if (!mask) return bfail(b, TUFRG_E_INVAL, "channel_mask selects no channel");
  const int n = (int)b->ctx.size();
  for (int i = 0; i < n; ++i)
    if (!is_device_ptr(P[i]) || !is_device_ptr(C[i])) return bfail(b, TUFRG_E_INVAL, "P, C must be device pointers");
  auto inst_fail = [&](int i) {
    return bfail(b, TUFRG_E_HIP, "instance " + std::to_string(i) + ": " + b->ctx[i]->err);
  };
  // the caller's writes to P, C are complete before the instances' streams start
  if (hipDeviceSynchronize() != hipSuccess) {
    (void)hipGetLastError();
    return bfail(b, TUFRG_E_HIP, "hipDeviceSynchronize failed");
  }
  std::vector<char> active(n, 1);
  std::vector<double> m_prev(n, 0.0), lam_prev(n, o->lambda0);
  for (int i = 0; i < n; ++i) {
    std::memset(&res[i], 0, sizeof(res[i]));
    res[i].lambda_stop = o->lambda0;
    bool bad = false;
    if (state_max(b->ctx[i], (const double *)P[i], (const double *)C[i], &m_prev[i], &bad) != TUFRG_OK)
      return inst_fail(i);
    if (bad) return bfail(b, TUFRG_E_NONFINITE, "non-finite initial state of instance " + std::to_string(i));
  }
  const int ns = o->n_steps;
  // one lockstep step of every active instance: enqueue, one wait for all,
  // then the stop tests
  // fused loop launches (asked for): every instance two-orbital in one
  // precision, both channels, no graphs (the work items and partial sums of
  // each instance are those of its own launch)
  bool fused = o->fused_loops && mask == 3u && !(o->graph_steps > 1);
  for (int i = 0; i < n && fused; ++i)
    fused = b->ctx[i]->n_o == 2 && b->ctx[i]->prec == b->ctx[0]->prec && !b->ctx[i]->timing;
  if (o->fused_loops && !fused)
    return bfail(b, TUFRG_E_UNSUPPORTED,
                 "fused loop launches need two-orbital instances of one precision, both channels and no graphs");
  if (fused) {
    if (!b->desc_h && hipHostMalloc((void **)&b->desc_h, n * sizeof(No2Inst), hipHostMallocDefault) != hipSuccess) {
      (void)hipGetLastError();
      b->desc_h = nullptr;
      return bfail(b, TUFRG_E_NOMEM, "hipHostMalloc of the loop descriptors failed");
    }
    if (!b->desc_d && hipMalloc((void **)&b->desc_d, n * sizeof(No2Inst)) != hipSuccess) {
      (void)hipGetLastError();
      b->desc_d = nullptr;
      return bfail(b, TUFRG_E_NOMEM, "hipMalloc of the loop descriptors failed");
    }
    while (b->fev.size() < b->streams.size()) {
      hipEvent_t e;
      if (hipEventCreateWithFlags(&e, hipEventDisableTiming) != hipSuccess) {
        (void)hipGetLastError();
        return bfail(b, TUFRG_E_HIP, "hipEventCreate failed");
      }
      b->fev.push_back(e);
    }
    for (int i = 0; i < n; ++i)
      if (!b->ctx[i]->d_dP) {
        tufrg_ctx *c = b->ctx[i];
        const size_t ns2 = 2 * (size_t)c->B * c->B * c->Nq;
        if (dalloc(c, &c->d_dP, ns2) != TUFRG_OK || dalloc(c, &c->d_dC, ns2) != TUFRG_OK) return inst_fail(i);
      }
  }
  // the loops of every active instance at l0 in fused launches on the first
  // stream, after each instance's regulator values on its own stream; then
  // each instance's stream waits for them
  auto fused_loops = [&](double l0) -> tufrg_status {
    std::vector<LoopArgs> la;
    for (int i = 0; i < n; ++i) {
      if (!active[i]) continue;
      if (compute_kval(b->ctx[i], l0, 1) != TUFRG_OK) return inst_fail(i);
      la.push_back(loop_args(b->ctx[i], l0, 1, 0, 2));
    }
    hipStream_t s0 = b->streams[0];
    for (size_t k = 1; k < b->streams.size(); ++k)
      if (hipEventRecord(b->fev[k], b->streams[k]) != hipSuccess || hipStreamWaitEvent(s0, b->fev[k], 0) != hipSuccess) {
        (void)hipGetLastError();
        return bfail(b, TUFRG_E_HIP, "stream join failed");
      }
    if (launch_loop_batch(la.data(), (int)la.size(), b->desc_h, b->desc_d, s0) != hipSuccess) {
      (void)hipGetLastError();
      return bfail(b, TUFRG_E_HIP, "fused loop launch failed");
    }
    if (hipEventRecord(b->fev[0], s0) != hipSuccess) {
      (void)hipGetLastError();
      return bfail(b, TUFRG_E_HIP, "hipEventRecord failed");
    }
    for (size_t k = 1; k < b->streams.size(); ++k)
      if (hipStreamWaitEvent(b->streams[k], b->fev[0], 0) != hipSuccess) {
        (void)hipGetLastError();
        return bfail(b, TUFRG_E_HIP, "stream fork failed");
      }
    int j = 0;
    for (int i = 0; i < n; ++i) {
      if (!active[i]) continue;
      tufrg_ctx *c = b->ctx[i];
      if (launch_loop_finalize(la[j++], c->nD, c->d_dlist, c->d_loop, c->st) != hipSuccess) {
        (void)hipGetLastError();
        return bfail(b, TUFRG_E_HIP, "instance " + std::to_string(i) + ": loop finalize failed");
      }
    }
    return TUFRG_OK;
  };
  auto direct_step = [&](int s) -> tufrg_status {
    const double l0 = euler_lambda(o, s), l1 = euler_lambda(o, s + 1);
    if (fused) {
      const tufrg_status fs = fused_loops(l0);
      if (fs != TUFRG_OK) return fs;
    }
    for (int i = 0; i < n; ++i) {
      if (!active[i]) continue;
      tufrg_ctx *c = b->ctx[i];
      double *Pi = (double *)P[i], *Ci = (double *)C[i];
      const long long ncx = (long long)c->B * c->B * c->Nq;
      if ((fused ? rhs_products(c, Pi, Ci, c->d_dP, c->d_dC, 1.0, mask)
                 : rhs_internal(c, l0, Pi, Ci, c->d_dP, c->d_dC, 1.0, mask)) != TUFRG_OK)
        return inst_fail(i);
      if (launch_clear_reduce(c->d_bits, c->d_flag, c->st) != hipSuccess ||
          launch_axpy_max(ncx, Pi, l1 - l0, c->d_dP, Pi, c->d_bits, c->d_flag, c->st) != hipSuccess ||
          launch_axpy_max(ncx, Ci, l1 - l0, c->d_dC, Ci, c->d_bits, c->d_flag, c->st) != hipSuccess ||
          hipMemcpyAsync(c->h_bits, c->d_bits, sizeof(unsigned long long), hipMemcpyDeviceToHost, c->st) !=
              hipSuccess ||
          hipMemcpyAsync(c->h_flag, c->d_flag, sizeof(unsigned int), hipMemcpyDeviceToHost, c->st) != hipSuccess) {
        (void)hipGetLastError();
        return bfail(b, TUFRG_E_HIP, "instance " + std::to_string(i) + ": launch failed");
      }
      res[i].n_rhs++;
      res[i].n_plain++;
    }
    for (hipStream_t st : b->streams)
      if (hipStreamSynchronize(st) != hipSuccess) {
        (void)hipGetLastError();
        return bfail(b, TUFRG_E_HIP, "stream synchronisation failed");
      }
    for (int i = 0; i < n; ++i) {
      if (!active[i]) continue;
      tufrg_ctx *c = b->ctx[i];
      double mx;
      std::memcpy(&mx, &c->h_bits[0], sizeof(mx));
      if (c->h_flag[0]) return bfail(b, TUFRG_E_NONFINITE, "non-finite state of instance " + std::to_string(i));
      res[i].n_steps++;
      res[i].lambda_stop = l1;
      res[i].max_coupling = mx;
      if (mx > o->v_max) {
        res[i].diverged = 1;
        res[i].lambda_c = lambda_c_interp(lam_prev[i], m_prev[i], l1, mx, o->v_max);
        active[i] = 0;
        continue;
      }
      if (o->max_steps > 0 && res[i].n_steps >= o->max_steps) active[i] = 0;
      lam_prev[i] = l1;
      m_prev[i] = mx;
    }
    return TUFRG_OK;
  };
  for (int i = 0; i < n; ++i) {
    tufrg_ctx *c = b->ctx[i];
    const size_t ns_d = 2 * (size_t)c->B * c->B * c->Nq;
    if (!c->d_dP && (dalloc(c, &c->d_dP, ns_d) != TUFRG_OK || dalloc(c, &c->d_dC, ns_d) != TUFRG_OK))
      return bfail(b, TUFRG_E_NOMEM, "instance " + std::to_string(i) + ": " + c->err);
  }
  // lockstep steps in HIP graphs: every active instance's steps captured
  // across the batch's streams (fork from the first stream, join back)
  const int G = (o->graph_steps > 1 && mask == 3u) ? std::min(o->graph_steps, MAX_GRAPH_STEPS) : 0;
  if (G) {
    for (int i = 0; i < n; ++i)
      if (graph_prepare(b->ctx[i]) != TUFRG_OK) return bfail(b, TUFRG_E_NOMEM, "instance " + std::to_string(i) + ": " + b->ctx[i]->err);
    while (b->events.size() < 2 * b->streams.size()) {
      hipEvent_t e;
      if (hipEventCreateWithFlags(&e, hipEventDisableTiming) != hipSuccess) {
        (void)hipGetLastError();
        return bfail(b, TUFRG_E_HIP, "hipEventCreate failed");
      }
      b->events.push_back(e);
    }
  }
  auto hipok = [&](hipError_t e, const char *what) -> bool {
    if (e == hipSuccess) return true;
    (void)hipGetLastError();
    bfail(b, TUFRG_E_HIP, std::string(what) + ": " + hipGetErrorString(e));
    return false;
  };
  int replay_to = -1;
  for (int s = 0; s < ns;) {
    if (G && s > 0 && s > replay_to) {
      int g = std::min(G, ns - s);
      if (o->max_steps > 0)
        for (int i = 0; i < n; ++i)
          if (active[i]) g = std::min(g, o->max_steps - res[i].n_steps);
      if (g > 1) {
        hipStream_t s0 = b->streams[0];
        if (!hipok(hipStreamBeginCapture(s0, hipStreamCaptureModeThreadLocal), "hipStreamBeginCapture"))
          return TUFRG_E_HIP;
        bool ok = hipok(hipEventRecord(b->events[0], s0), "hipEventRecord");
        for (size_t k = 1; ok && k < b->streams.size(); ++k)
          ok = hipok(hipStreamWaitEvent(b->streams[k], b->events[0], 0), "hipStreamWaitEvent");
        int bad_inst = -1;
        for (int i = 0; ok && i < n; ++i)
          if (active[i] && enqueue_euler_steps(b->ctx[i], o, (double *)P[i], (double *)C[i], s, g, mask) != TUFRG_OK) {
            bad_inst = i;
            ok = false;
          }
        for (size_t k = 1; ok && k < b->streams.size(); ++k)
          ok = hipok(hipEventRecord(b->events[k], b->streams[k]), "hipEventRecord") &&
               hipok(hipStreamWaitEvent(s0, b->events[k], 0), "hipStreamWaitEvent");
        hipGraph_t graph = nullptr;
        const hipError_t ee = hipStreamEndCapture(s0, &graph);
        if (!ok || ee != hipSuccess) {
          if (graph) (void)hipGraphDestroy(graph);
          (void)hipGetLastError();
          if (bad_inst >= 0) return inst_fail(bad_inst);
          return b->err.empty() ? bfail(b, TUFRG_E_HIP, "graph capture failed") : TUFRG_E_HIP;
        }
        bool updated = false;
        if (b->gexec) {
          hipGraphNode_t en = nullptr;
          hipGraphExecUpdateResult ur = hipGraphExecUpdateError;
          updated = hipGraphExecUpdate(b->gexec, graph, &en, &ur) == hipSuccess && ur == hipGraphExecUpdateSuccess;
          if (!updated) {
            (void)hipGetLastError();
            (void)hipGraphExecDestroy(b->gexec);
            b->gexec = nullptr;
          }
        }
        if (!updated && !hipok(hipGraphInstantiate(&b->gexec, graph, nullptr, nullptr, 0), "hipGraphInstantiate")) {
          b->gexec = nullptr;
          (void)hipGraphDestroy(graph);
          return TUFRG_E_HIP;
        }
        (void)hipGraphDestroy(graph);
        // save the states, run the graph, read every instance's step slots
        for (int i = 0; i < n; ++i) {
          if (!active[i]) continue;
          tufrg_ctx *c = b->ctx[i];
          const size_t bytes = 2 * sizeof(double) * (size_t)c->B * c->B * c->Nq;
          if (!hipok(hipMemcpyAsync(c->d_bkP, P[i], bytes, hipMemcpyDeviceToDevice, s0), "hipMemcpyAsync") ||
              !hipok(hipMemcpyAsync(c->d_bkC, C[i], bytes, hipMemcpyDeviceToDevice, s0), "hipMemcpyAsync"))
            return TUFRG_E_HIP;
        }
        if (!hipok(hipGraphLaunch(b->gexec, s0), "hipGraphLaunch")) return TUFRG_E_HIP;
        for (int i = 0; i < n; ++i) {
          if (!active[i]) continue;
          tufrg_ctx *c = b->ctx[i];
          if (!hipok(hipMemcpyAsync(c->h_gbits, c->d_gbits, g * sizeof(unsigned long long), hipMemcpyDeviceToHost,
                                    s0), "hipMemcpyAsync") ||
              !hipok(hipMemcpyAsync(c->h_gflag, c->d_gflag, g * sizeof(unsigned int), hipMemcpyDeviceToHost, s0),
                     "hipMemcpyAsync"))
            return TUFRG_E_HIP;
        }
        if (!hipok(hipStreamSynchronize(s0), "hipStreamSynchronize")) return TUFRG_E_HIP;
        int stop = -1;
        for (int i = 0; i < n; ++i) {
          if (!active[i]) continue;
          for (int j = 0; j < g; ++j) {
            double mx;
            std::memcpy(&mx, &b->ctx[i]->h_gbits[j], sizeof(mx));
            if (b->ctx[i]->h_gflag[j] || mx > o->v_max) {
              stop = stop < 0 ? j : std::min(stop, j);
              break;
            }
          }
        }
        if (stop >= 0) {
          // undo the graph's steps of every instance and take them one by one
          for (int i = 0; i < n; ++i) {
            if (!active[i]) continue;
            tufrg_ctx *c = b->ctx[i];
            const size_t bytes = 2 * sizeof(double) * (size_t)c->B * c->B * c->Nq;
            if (!hipok(hipMemcpyAsync(P[i], c->d_bkP, bytes, hipMemcpyDeviceToDevice, s0), "hipMemcpyAsync") ||
                !hipok(hipMemcpyAsync(C[i], c->d_bkC, bytes, hipMemcpyDeviceToDevice, s0), "hipMemcpyAsync"))
              return TUFRG_E_HIP;
          }
          if (!hipok(hipStreamSynchronize(s0), "hipStreamSynchronize")) return TUFRG_E_HIP;
          replay_to = s + stop;
          continue;
        }
        for (int i = 0; i < n; ++i) {
          if (!active[i]) continue;
          for (int j = 0; j < g; ++j) {
            double mx;
            std::memcpy(&mx, &b->ctx[i]->h_gbits[j], sizeof(mx));
            res[i].n_rhs++;
            res[i].n_plain++;
            res[i].n_steps++;
            res[i].lambda_stop = euler_lambda(o, s + j + 1);
            res[i].max_coupling = mx;
            lam_prev[i] = res[i].lambda_stop;
            m_prev[i] = mx;
          }
          if (o->max_steps > 0 && res[i].n_steps >= o->max_steps) active[i] = 0;
        }
        s += g;
        if (std::none_of(active.begin(), active.end(), [](char a) { return a != 0; })) break;
        continue;
      }
    }
    TRY(direct_step(s));
    ++s;
    if (std::none_of(active.begin(), active.end(), [](char a) { return a != 0; })) break;
  }
  return TUFRG_OK;
}
