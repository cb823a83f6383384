// C ABI of the LDG-Stokes library: setup (host hierarchy + device upload),
// the V-cycle driver (Algorithm 1) and the outer iterations.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <chrono>
#include <cmath>
#include <cstdio>
#include <cstdlib>
#include <cstring>
#include <memory>
#include <stdexcept>
#include <string>
#include <type_traits>
#include <vector>

#include "build.hpp"
#include "host.hpp"
#include "implicit.hpp"
#include "learned_internal.hpp"

namespace ldgs {
void assemble_rhs_host(const ldgs_problem& P, const Geometry& g, const Basis& B, const Level& L,
                       const ldgs_rhs_data& data, double* out);
}

using namespace ldgs;

namespace {

struct Fail {
  ldgs_status st;
  std::string msg;
};

#define HIPCHK(call)                                                              \
  do {                                                                            \
    hipError_t e_ = (call);                                                       \
    if (e_ != hipSuccess) throw Fail{LDGS_E_HIP, std::string(#call) + ": " + hipGetErrorString(e_)}; \
  } while (0)

#define LCHK(call)                                                                \
  do {                                                                            \
    int r_ = (call);                                                              \
    if (r_ == 2) throw Fail{LDGS_E_UNSUPPORTED, std::string(#call) + ": no kernel for this d/p"}; \
    if (r_ != 0) throw Fail{LDGS_E_HIP, std::string(#call) + ": launch failed"};  \
  } while (0)

template <typename T>
struct PrecLevel {
  DevLevel<T> view{};            // the V-cycle's (possibly scaled) operator
  DevLevel<T> unscaled{};        // same data, no scaling (finest level, outer residual)
  const void* inv = nullptr;     // colour-major, column-major blocks
  int inv_kind = 0;              // 0 double, 1 float, 2 bf16
  int* elems = nullptr;          // colour-major element ids
  std::vector<int64_t> col_off;  // colour offsets (elements)
  std::vector<int64_t> col_reg;  // per colour: leading elements whose evaluation touches no interphase face
  bool parity = false;           // parity colouring, each colour in increasing order (kernels compute the ids)
  size_t inv_stride = 0;         // entries per element in the inverse layout
  const T* ainv_sh = nullptr;    // set when every element has the same block: its inverse, k-major (a[k nb + row])
  const void* ainv_tiles = nullptr;   // the same inverse in the symmetric tile layout (one element's worth)
  int ainv_tiles_kind = 0;            // 0 double, 1 float
  T* rbuf = nullptr;             // colour residuals for the shared-inverse pass ([largest colour][nb])
  T* x = nullptr;                // level work vectors (levels >= 1)
  T* b = nullptr;
};

template <typename T>
struct PrecStore {
  bool built = false;           // full V-cycle data
  bool ops = false;             // operator data uploaded
  std::vector<PrecLevel<T>> lv;
};

}  // namespace

struct ldgs_ctx {
  ldgs_problem P{};
  Geometry g;
  Basis B;
  Tab1D tab{};
  std::vector<Level> levels;
  std::string err;
  bool host_only = false;
  hipStream_t stream = nullptr;
  int vprec = 0;
  int k0 = 1;
  int small_grid = 4096;       // see LaunchCfg; LDGS_SMALL_GRID overrides (tests)
  bool shared_inverse = true;  // one inverse per level with equal blocks; LDGS_SHARED_INVERSE=0 disables
  bool use_graph = true;       // V-cycles replayed from captured HIP graphs; LDGS_GRAPH=0 disables
  bool device_setup = true;    // per-element block inverses assembled and inverted on the GPU; LDGS_DEVICE_SETUP=0: host
  // colour passes with per-element inverses as two launches (residual, then
  // the streamed product) on 3D levels; LDGS_SPLIT_PASS=0/1 overrides
  int split_pass = -1;
  // split colour passes of at least overlap_min elements run in overlap_chunks
  // chunks: the residuals of chunk k + 1 (LDS- and issue-bound) on the main
  // stream beside the streamed product of chunk k (HBM-bound) on a second
  // stream; elements of one colour do not couple, so the chunks' residuals do
  // not read what the products write.  LDGS_OVERLAP=<chunks> (1: off) and
  // LDGS_OVERLAP_MIN=<elements> override
  int overlap_chunks = 8;
  int64_t overlap_min = 131072;
  hipStream_t side = nullptr;
  hipEvent_t ov_fork = nullptr, ov_join = nullptr;
  std::vector<hipEvent_t> ov_prod;   // end of each chunk's product (side stream)
  bool ov_chain = true;              // chain the chunks across colours; LDGS_OVERLAP_CHAIN=0 disables
  // one-inverse updates (FP32 and FP64) of colours of at least mfma_min elements on the
  // matrix cores (0: never); LDGS_MFMA=0 disables, LDGS_MFMA_MIN overrides
  // the size (tests)
  int64_t mfma_min = 8192;
  // one-inverse colours of fewer elements than this run as one launch (the
  // evaluation and the product with the level's inverse in one kernel)
  // instead of a residual launch and an update launch; LDGS_FUSE_SHARED_MAX
  // overrides (0: never)
  int64_t fuse_shared_max = 4096;
  std::vector<int> kernel_offsets;
  bool rotations = false;            // the rigid rotations belong to the kernel (stress walls)
  PrecStore<double> s64;
  PrecStore<float> s32;      // float arithmetic, float inverses
  PrecStore<float> s16;      // float arithmetic, bf16 inverses (shares operator data with s32)
  double* d_pinv = nullptr;
  double* d_Ac = nullptr;            // bottom operator (dense), for the refinement step
  double *d_bt0 = nullptr, *d_bt1 = nullptr, *d_bt2 = nullptr;   // bottom temporaries
  int64_t Nc = 0;
  std::vector<double> h_pinv, h_eig, h_Ac;
  // finest-size work vectors
  double *w_b = nullptr, *w_x = nullptr, *w_r = nullptr, *w_z = nullptr, *w_part = nullptr;
  float *w_b32 = nullptr, *w_x32 = nullptr;
  double* d_dscale0 = nullptr;      // finest-level scaling (double) for user <-> scaled
  std::vector<double*> kry;         // FGMRES basis storage
  // learned correction
  bool net_loaded = false;
  NetShape ns{};
  float* d_net = nullptr;           // padded FP32 parameters
  uint16_t* d_netbf = nullptr;      // BF16 copy
  double c_net[2] = {1.0, 1.0};
  float* d_logmu = nullptr;         // finest-level log10 of the element mean of mu
  double* d_sums = nullptr;         // [2] sums of squares (velocity, pressure)
  double *w_xold = nullptr, *w_zl = nullptr, *w_r64b = nullptr, *w_dx = nullptr, *w_adx64 = nullptr;
  float *w_r32 = nullptr, *w_adx32 = nullptr;
  double* d_mr = nullptr;           // [3] minimal-residual sums r'.q, q.q and the step w
  int64_t learned_steps = 0;        // corrections applied (diagnostics)
  bool learned_full_step = false;   // LDGS_LEARNED_FULL_STEP=1 at setup: w = 1 instead of the minimal-residual step
  double* w_rf64 = nullptr;         // fine residual scratch of the split residual + restriction (small grids)
  float* w_rf32 = nullptr;
  double *w_cb = nullptr, *w_cx = nullptr, *w_ce = nullptr;
  int* d_orig = nullptr;
  int64_t d_orig_cap = 0;
  // optional timing of the finest-level colour passes (HIP events on the
  // stream): one event pair around all colour passes of a sweep
  struct ProfEv {
    hipEvent_t e0, e1;
    int passes;                  // colour passes between the two events
  };
  int prof = 0;                  // time every prof-th finest sweep (0: off)
  int64_t prof_count = 0;
  std::vector<ProfEv> prof_ev;
  std::vector<hipEvent_t> ev_pool;
  size_t ev_used = 0;
  std::vector<void*> allocs;
  // a stream of the library's own when the caller gives none (the legacy
  // null stream cannot be captured into a graph); calls order it after the
  // caller's null-stream work and the null stream after it (join events)
  hipEvent_t join_in = nullptr, join_out = nullptr;
  // captured V-cycles, one per (precision, zero guess); cycles timed with
  // event pairs are launched directly
  struct CycleGraph {
    int vp;
    bool zero_x;
    hipGraphExec_t exec;
  };
  std::vector<CycleGraph> graphs;
  ~ldgs_ctx() {
    // nothing may still use the storage when it goes back to its owner (a
    // caching allocator hands it out again at once)
    if (!host_only) (void)hipStreamSynchronize(stream);
    if (side) (void)hipStreamSynchronize(side);
    for (auto& g : graphs) (void)hipGraphExecDestroy(g.exec);
    for (hipEvent_t e : ev_pool) (void)hipEventDestroy(e);
    for (void* p : allocs) {
      if (P.dev_free) P.dev_free(p, P.alloc_user);
      else (void)hipFree(p);
    }
    if (side) (void)hipStreamDestroy(side);
    for (hipEvent_t e : ov_prod) (void)hipEventDestroy(e);
    if (ov_fork) (void)hipEventDestroy(ov_fork);
    if (ov_join) (void)hipEventDestroy(ov_join);
    if (join_in) (void)hipEventDestroy(join_in);
    if (join_out) (void)hipEventDestroy(join_out);
    if (stream_owned && stream) (void)hipStreamDestroy(stream);
  }
  bool stream_owned = false;
  // implicitly defined mesh (circle level set): explicit element blocks on
  // every level, host data in imp, device arrays per level in idev
  std::unique_ptr<ImpHier> imp;
  struct ImpDev {
    int64_t NE = 0;
    int *rowptr = nullptr, *cols = nullptr, *parent = nullptr, *kid_ptr = nullptr, *kids = nullptr;
    std::vector<int*> elems;
    std::vector<int64_t> ncnt;
    double *blk64 = nullptr, *inv64 = nullptr, *I64 = nullptr, *b64 = nullptr, *x64 = nullptr, *r64 = nullptr;
    float *blk32 = nullptr, *inv32 = nullptr, *I32 = nullptr, *b32 = nullptr, *x32 = nullptr, *r32 = nullptr;
  };
  std::vector<ImpDev> idev;
  double* d_kernel = nullptr;       // fine kernel vector (unit norm)
  double* d_dinv0 = nullptr;        // fine per-element 1 / (alpha, beta)
  bool imp64 = false, imp32 = false;
  int64_t ndof() const {
    if (imp) return imp->lv.empty() ? 0 : imp->lv[0].NE * imp->nb;
    return levels.empty() ? 0 : levels[0].NE * g.nb;
  }
};

namespace {

// Device storage of the context: from the caller's allocator when it gave
// one (dev_alloc / dev_free of ldgs_problem), else hipMalloc.  Every block is
// returned when the context is destroyed.
template <typename T>
T* dalloc(ldgs_ctx* c, size_t count) {
  void* p = nullptr;
  if (count == 0) count = 1;
  const size_t bytes = count * sizeof(T);
  if (c->P.dev_alloc) {
    p = c->P.dev_alloc(bytes, c->P.alloc_user);
    if (!p) throw Fail{LDGS_E_NOMEM, "dev_alloc returned NULL for " + std::to_string(bytes) + " bytes"};
    if (((uintptr_t)p & 255u) != 0) {
      c->P.dev_free(p, c->P.alloc_user);
      throw Fail{LDGS_E_ARG, "dev_alloc returned a block that is not 256-byte aligned"};
    }
  } else {
    hipError_t e = hipMalloc(&p, bytes);
    if (e != hipSuccess) throw Fail{LDGS_E_NOMEM, std::string("hipMalloc: ") + hipGetErrorString(e)};
  }
  c->allocs.push_back(p);
  return (T*)p;
}

// Orders the library's own stream (used when the caller gave none) after the
// work the caller queued on the null stream before the call, and the null
// stream after the work of the call.
struct Join {
  ldgs_ctx* c;
  explicit Join(ldgs_ctx* c_) : c(c_) {
    if (c && c->stream_owned) {
      HIPCHK(hipEventRecord(c->join_in, nullptr));
      HIPCHK(hipStreamWaitEvent(c->stream, c->join_in, 0));
    }
  }
  ~Join() {
    if (c && c->stream_owned) {
      (void)hipEventRecord(c->join_out, c->stream);
      (void)hipStreamWaitEvent(nullptr, c->join_out, 0);
    }
  }
};

template <typename T>
T* upload(ldgs_ctx* c, const double* src, size_t n) {
  T* d = dalloc<T>(c, n);
  if (n == 0) return d;
  if constexpr (std::is_same_v<T, double>) {
    HIPCHK(hipMemcpy(d, src, n * sizeof(T), hipMemcpyHostToDevice));
  } else {
    // converted in pieces on all host threads
    const size_t piece = (size_t)1 << 24;
    std::vector<T> tmp(std::min(piece, n));
    for (size_t o = 0; o < n; o += piece) {
      const int64_t cnt = (int64_t)std::min(piece, n - o);
#pragma omp parallel for schedule(static)
      for (int64_t i = 0; i < cnt; ++i) tmp[i] = (T)src[o + i];
      HIPCHK(hipMemcpy(d + o, tmp.data(), cnt * sizeof(T), hipMemcpyHostToDevice));
    }
  }
  return d;
}

template <typename T>
T* upload(ldgs_ctx* c, const std::vector<double>& src) {
  return upload<T>(c, src.data(), src.size());
}

bool stress_walls(const ldgs_problem& P) { return P.bc[0] == LDGS_STRESS; }

// trivial kernel (bottom-solver footnote): periodic steady: constant velocity
// components and pressure; stress walls, steady: constant velocity components
// and, in viscous-stress form, the d(d-1)/2 rigid rotations (none when
// unsteady); otherwise the constant pressure
int kernel_dim(const ldgs_problem& P) {
  const bool steady = !(P.delta > 0.0);
  if (stress_walls(P)) return steady ? P.dim + (P.form ? P.dim * (P.dim - 1) / 2 : 0) : 0;
  bool per = true;
  for (int j = 0; j < P.dim; ++j) per = per && P.bc[j] == LDGS_PERIODIC;
  return (per && steady) ? P.dim + 1 : 1;
}

void fill_defaults(ldgs_problem& P) {
  static const double tab_std[2][5] = {{0.19, 0.10, 0.086, 0.019, 0.031}, {0.12, 0.088, 0.084, 0, 0}};
  static const double tab_vs[2][5] = {{0.14, 0.046, 0.034, 0.0095, 0.011}, {0.12, 0.039, 0.040, 0, 0}};
  if (!(P.tau > 0)) P.tau = (P.form ? tab_vs : tab_std)[P.dim - 2][P.degree - 1];
  if (!(P.tau0 > 0)) P.tau0 = 0.5 * P.degree;
  if (!(P.tau_u_bdry_C > 0)) P.tau_u_bdry_C = 10.0;
  if (!(P.tau_u_inter_C > 0)) P.tau_u_inter_C = (P.levelset_kind == LDGS_LEVELSET_CIRCLE || P.levelset_kind == LDGS_LEVELSET_DISK) ? 8.0 : 3.0;
  if (P.q_cut <= 0) P.q_cut = 8;
  if (P.nu1 <= 0) P.nu1 = 3;
  if (P.nu2 <= 0) P.nu2 = 3;
  if (P.coarsest_n <= 0) P.coarsest_n = (P.dim == 2) ? 4 : 2;
}

bool pow2(int v) { return v > 0 && (v & (v - 1)) == 0; }

void validate(const ldgs_problem& P) {
  if (P.dim != 2 && P.dim != 3) throw Fail{LDGS_E_ARG, "dim must be 2 or 3"};
  if (P.degree < 1 || P.degree > 3) throw Fail{LDGS_E_ARG, "degree must be 1..3"};
  if (P.dim == 3 && P.degree > 2) throw Fail{LDGS_E_UNSUPPORTED, "3D supports p <= 2"};
  if (!pow2(P.n) || !pow2(P.coarsest_n) || P.coarsest_n < 2 || P.coarsest_n > P.n)
    throw Fail{LDGS_E_ARG, "n and coarsest_n must be powers of two with 2 <= coarsest_n <= n"};
  if (P.form != 0 && P.form != 1) throw Fail{LDGS_E_ARG, "form"};
  int nstress = 0;
  for (int j = 0; j < P.dim; ++j) {
    if (P.bc[j] != LDGS_PERIODIC && P.bc[j] != LDGS_DIRICHLET && P.bc[j] != LDGS_STRESS)
      throw Fail{LDGS_E_ARG, "bc"};
    nstress += P.bc[j] == LDGS_STRESS;
  }
  if (nstress != 0 && nstress != P.dim)
    throw Fail{LDGS_E_UNSUPPORTED, "stress boundary conditions must be given on every axis"};
  if (P.levelset_kind == LDGS_LEVELSET_CIRCLE || P.levelset_kind == LDGS_LEVELSET_DISK) {
    if (P.dim != 2 || P.bc[0] != LDGS_DIRICHLET || P.bc[1] != LDGS_DIRICHLET)
      throw Fail{LDGS_E_UNSUPPORTED, "circle level sets: 2D problems with Dirichlet walls"};
    if (P.delta > 0.0 && P.rho.kind != LDGS_FIELD_CONST && P.rho.kind != LDGS_FIELD_PHASE_CONST)
      throw Fail{LDGS_E_UNSUPPORTED, "circle level sets: density constant or constant per phase"};
    if (P.delta > 0.0 && !(P.rho.params && P.rho.params[0] > 0 &&
                           (P.rho.kind == LDGS_FIELD_CONST || P.rho.params[1] > 0)))
      throw Fail{LDGS_E_ARG, "rho must be positive"};
    if (!(P.levelset_params[0] > 0.0)) throw Fail{LDGS_E_ARG, "circle radius must be positive"};
    if (P.vprec == LDGS_V_FP32_BF16BLK || (P.build_precisions & 4))
      throw Fail{LDGS_E_UNSUPPORTED, "BF16-stored blocks are not built on implicitly defined meshes"};
    if (P.q_cut > 32) throw Fail{LDGS_E_ARG, "q_cut"};
  } else if (P.levelset_kind != LDGS_LEVELSET_NONE) {
    if (P.levelset_kind != LDGS_LEVELSET_BOX) throw Fail{LDGS_E_ARG, "levelset_kind"};
    if (!P.host_only && P.dim != 2) throw Fail{LDGS_E_UNSUPPORTED, "interphase faces are supported in 2D"};
  }
  if (P.delta > 0.0 && !(P.levelset_kind == LDGS_LEVELSET_CIRCLE || P.levelset_kind == LDGS_LEVELSET_DISK)) {
    if (P.rho.kind != LDGS_FIELD_CONST || P.mu.kind != LDGS_FIELD_CONST)
      throw Fail{LDGS_E_UNSUPPORTED, "unsteady problems need constant mu and rho"};
    if (!(P.rho.params && P.rho.params[0] > 0)) throw Fail{LDGS_E_ARG, "rho must be positive"};
  }
  if (P.mu.kind < 0 || P.mu.kind > LDGS_FIELD_CALLBACK) throw Fail{LDGS_E_ARG, "mu kind"};
  if (P.mu.kind != LDGS_FIELD_CALLBACK && !P.mu.params) throw Fail{LDGS_E_ARG, "mu params"};
  if (P.mu.kind == LDGS_FIELD_CALLBACK && !P.mu.fn) throw Fail{LDGS_E_ARG, "mu callback"};
  if (P.vprec < 0 || P.vprec > 2) throw Fail{LDGS_E_ARG, "vprec"};
  if ((P.dev_alloc == nullptr) != (P.dev_free == nullptr))
    throw Fail{LDGS_E_ARG, "dev_alloc and dev_free must be given together"};
  if (P.coloring < 0 || P.coloring > 3) throw Fail{LDGS_E_ARG, "coloring"};
}

// smoothed levels: colouring, blocks, inverses
int log2i(int v) {
  int l = 0;
  while ((1 << l) < v) ++l;
  return l;
}

void build_smoother_host(ldgs_ctx* c) {
  const int d = c->g.d;
  for (size_t l = 0; l + 1 < c->levels.size(); ++l) {
    Level& L = c->levels[l];
    int scheme = c->P.coloring;
    int64_t bad = -1;
    if (scheme == LDGS_COLOR_AUTO) {
      const int order[3] = {LDGS_COLOR_RED_BLACK, LDGS_COLOR_PARITY, LDGS_COLOR_MOD3};
      scheme = -1;
      for (int s : order)
        if (colouring_is_proper(L, d, s, c->P.form, &bad)) { scheme = s; break; }
      if (scheme < 0) throw Fail{LDGS_E_COLORING, "no proper colouring found"};
    } else if (!colouring_is_proper(L, d, scheme, c->P.form, &bad)) {
      throw Fail{LDGS_E_COLORING, "colouring couples two elements of one colour at element " + std::to_string(bad) +
                                       " on level " + std::to_string(l)};
    }
    set_colouring(L, d, scheme);
  }
}

// stride of the axis-k coordinate in the face numbering of axis k (axis 0
// fastest; every axis before k has n entries)
int64_t face_stride(int n, int k) {
  int64_t s = 1;
  for (int j = 0; j < k; ++j) s *= n;
  return s;
}

template <typename T>
DevLevel<T> make_view(ldgs_ctx* c, const Level& L, bool with_scale) {
  DevLevel<T> v{};
  const int d = c->g.d, mt = c->g.mt, nq = c->g.nq;
  bool iface = false;
  for (int k = 0; k < d; ++k)
    for (unsigned char t : L.faces[k].type) iface = iface || t == F_INTER;
  v.iface = iface ? 1 : 0;
  v.stress = stress_walls(c->P) ? 1 : 0;
  v.n = L.n;
  v.hinv = (T)(1.0 / L.h);
  for (int k = 0; k < 3; ++k) {
    if (k < d) {
      const FaceSet& fs = L.faces[k];
      v.nf[k] = fs.nfk;
      // without interphase faces the kernels derive face types and lifting
      // weights from the position (intraphase inside, Dirichlet at
      // non-periodic walls); check that the level matches
      if (iface) {
        // interphase faces: 2D only (extended stencil), data from the tables
        if (d != 2) throw Fail{LDGS_E_UNSUPPORTED, "interphase faces are supported in 2D"};
      } else for (int64_t id = 0; id < fs.count; ++id) {
        const int64_t f = (id / face_stride(L.n, k)) % fs.nfk;
        const bool wall = fs.nfk != L.n && (f == 0 || f == L.n);
        const bool stress = wall && c->P.bc[k] == LDGS_STRESS;
        unsigned char want = F_INTRA;
        if (fs.nfk != L.n && f == 0) want = F_DIR_LO;
        if (fs.nfk != L.n && f == L.n) want = F_DIR_HI;
        if (stress) want = F_NONE;
        const double wl = fs.w[2 * id], wr = fs.w[2 * id + 1];
        const double wl_want = want == F_DIR_HI ? 1.0 : 0.0, wr_want = (want == F_DIR_HI || stress) ? 0.0 : 1.0;
        if (fs.type[id] != want || wl != wl_want || wr != wr_want)
          throw Fail{LDGS_E_UNSUPPORTED, "face types other than intraphase, Dirichlet and stress walls are not supported on the GPU"};
      }
      unsigned char* ft = dalloc<unsigned char>(c, fs.count);
      HIPCHK(hipMemcpy(ft, fs.type.data(), fs.count, hipMemcpyHostToDevice));
      v.ftype[k] = ft;
      v.fw[k] = upload<T>(c, fs.w);
      v.fT[k] = upload<T>(c, fs.T);
    } else {
      v.nf[k] = 0;
      v.ftype[k] = nullptr;
      v.fw[k] = nullptr;
      v.fT[k] = nullptr;
    }
  }
  int lg = 0;
  while ((1 << lg) < L.n) ++lg;
  v.lgn = lg;
  v.mmu = L.mu_is_const ? nullptr : upload<T>(c, L.mmu);
  v.rmu = nullptr;
  v.rmuh = nullptr;
  if (!L.mu_is_const) {
    // (e0^T)_k M_mu and (e1^T)_k M_mu: low- and high-face trace rows of the
    // mass block along axis k
    const int M = c->g.p + 1;
    auto rows = [&](const double* ev) {
      std::vector<double> R((size_t)L.NE * d * mt * nq, 0.0);
#pragma omp parallel for schedule(static)
      for (int64_t e = 0; e < L.NE; ++e) {
        const double* Me = L.mmu.data() + (size_t)e * nq * nq;
        for (int k = 0; k < d; ++k) {
          int lo = 1;
          for (int j = 0; j < k; ++j) lo *= M;
          double* Rk = R.data() + ((size_t)e * d + k) * mt * nq;
          for (int t = 0; t < mt; ++t)
            for (int cc = 0; cc < M; ++cc) {
              const int a = t % lo + lo * cc + lo * M * (t / lo);
              const double w = ev[cc];
              for (int b = 0; b < nq; ++b) Rk[t * nq + b] += w * Me[a * nq + b];
            }
        }
      }
      return R;
    };
    v.rmu = upload<T>(c, rows(c->tab.e0));
    if (v.iface) v.rmuh = upload<T>(c, rows(c->tab.e1));
  }
  v.mu_const = (T)L.mu_c;
  v.rho_delta = (T)L.rho_delta;
  v.dscale = (with_scale && !L.dscale.empty()) ? upload<T>(c, L.dscale) : nullptr;
  v.gamma = c->P.form;
  return v;
}

template <typename T>
void upload_ops(ldgs_ctx* c, PrecStore<T>& S, bool all_levels) {
  size_t nl = all_levels ? c->levels.size() : 1;
  S.lv.resize(c->levels.size());
  for (size_t l = 0; l < nl; ++l) {
    S.lv[l].view = make_view<T>(c, c->levels[l], true);
    S.lv[l].unscaled = S.lv[l].view;
    S.lv[l].unscaled.dscale = nullptr;
    if (l > 0) {
      int64_t n = c->levels[l].NE * c->g.nb;
      S.lv[l].x = dalloc<T>(c, n);
      S.lv[l].b = dalloc<T>(c, n);
    }
  }
  S.ops = true;
}

// entries of one element's inverse in the smoother's symmetric tile layout
// (see sym_tiles): inv is row-major nb x nb; its symmetric part is stored, out
// receives sym_tile_off(TR, NTILE) values
static void arrange_inverse(const double* inv, int nb, int bytes, double* out) {
  const SymTiles L = sym_tiles(nb, bytes);
  auto sym = [&](int r, int c) {
    return (r < nb && c < nb) ? 0.5 * (inv[(size_t)r * nb + c] + inv[(size_t)c * nb + r]) : 0.0;
  };
  for (int i = 0; i < L.TR; ++i)
    for (int j = i; j < L.TR; ++j) {
      const int t = i * L.TR - i * (i - 1) / 2 + (j - i);
      const int nblk = i == j ? SYM_DBLOCKS : 64;
      double* o = out + sym_tile_off(L.TR, t);
      for (int r = 0; r < 16; ++r)
        for (int cb = 0; cb < 4; ++cb) {
          if (i == j && cb < r / 4) continue;       // below the diagonal: not stored
          const int slot = i == j ? sym_dslot(r, cb) : 4 * r + cb;
          for (int v = 0; v < 4; ++v) {
            const int h = v / L.EL, u = v % L.EL;
            o[((size_t)h * nblk + slot) * L.EL + u] = sym(16 * i + r, 16 * j + 4 * cb + v);
          }
        }
    }
}

static uint16_t to_bf16(double d) {
  float f = (float)d;
  uint32_t u;
  std::memcpy(&u, &f, 4);
  u += 0x7fffu + ((u >> 16) & 1u);   // round to nearest even
  return (uint16_t)(u >> 16);
}

// true when the evaluation of E uses an interphase face: a face of E or of E + e_j
bool touches_interphase(const Level& L, int d, int64_t E) {
  int c[3] = {0, 0, 0};
  int64_t r = E;
  for (int j = 0; j < d; ++j) {
    c[j] = (int)(r % L.n);
    r /= L.n;
  }
  for (int fi = 0; fi <= d; ++fi) {
    int cf[3] = {c[0], c[1], c[2]};
    if (fi > 0) {
      const int j = fi - 1;
      int v = cf[j] + 1;
      if (v >= L.n) {
        if (L.faces[j].nfk != L.n) continue;   // beyond a wall
        v -= L.n;
      }
      cf[j] = v;
    }
    for (int k = 0; k < d; ++k)
      for (int side = 0; side < 2; ++side) {
        int f = cf[k] + side;
        if (L.faces[k].nfk == L.n) f %= L.n;
        if (L.faces[k].type[face_id(L, d, k, cf, f)] == F_INTER) return true;
      }
  }
  return false;
}

// inverse blocks of all smoothed levels into the stores that need them
// True when every diagonal block of the level is the same matrix: constant
// viscosity, all faces intraphase (periodic grid) with equal weights and
// penalty blocks, one phase and one scaling.  The blocks are then translation
// invariant; three elements' blocks are compared as a check.
static bool uniform_blocks(const ldgs_ctx* c, const Level& L) {
  if (!L.mu_is_const || L.NE < 1) return false;
  for (int k = 0; k < c->g.d; ++k) {
    const FaceSet& F = L.faces[k];
    for (unsigned char t : F.type)
      if (t != F_INTRA) return false;
    auto constant = [](const std::vector<double>& v, size_t stride) {
      for (size_t i = stride; i < v.size(); ++i)
        if (v[i] != v[i % stride]) return false;
      return true;
    };
    const size_t mt2 = (size_t)c->g.mt * c->g.mt;
    if (!constant(F.w, 2) || !constant(F.T, mt2) || !constant(F.Tmu, mt2) || !constant(F.Trho, mt2)) return false;
  }
  for (size_t i = 1; i < L.chi.size(); ++i)
    if (L.chi[i] != L.chi[0]) return false;
  for (size_t i = 2; i < L.dscale.size(); ++i)
    if (L.dscale[i] != L.dscale[i % 2]) return false;
  const int nb = c->g.nb;
  std::vector<double> A0((size_t)nb * nb), A1((size_t)nb * nb);
  host_diag_block(L, c->g, c->B, c->P.form, 0, A0.data());
  for (int64_t E : {L.NE / 2 + 1, L.NE - 1}) {
    if (E >= L.NE) continue;
    host_diag_block(L, c->g, c->B, c->P.form, E, A1.data());
    for (size_t i = 0; i < A0.size(); ++i)
      if (std::fabs(A1[i] - A0[i]) > 1e-13 * (std::fabs(A0[i]) + 1.0)) return false;
  }
  return true;
}

// Device buffers needed during setup only: drawn like the context's own
// storage (caller's allocator or hipMalloc) and returned at scope exit, after
// the stream has drained.
struct TempDev {
  ldgs_ctx* c;
  std::vector<void*> p;
  explicit TempDev(ldgs_ctx* c_) : c(c_) {}
  template <typename T>
  T* get(size_t count) {
    const size_t bytes = (count ? count : 1) * sizeof(T);
    void* q = nullptr;
    if (c->P.dev_alloc) {
      q = c->P.dev_alloc(bytes, c->P.alloc_user);
      if (!q) throw Fail{LDGS_E_NOMEM, "dev_alloc returned NULL for " + std::to_string(bytes) + " bytes"};
    } else {
      hipError_t e = hipMalloc(&q, bytes);
      if (e != hipSuccess) throw Fail{LDGS_E_NOMEM, std::string("hipMalloc: ") + hipGetErrorString(e)};
    }
    p.push_back(q);
    return (T*)q;
  }
  ~TempDev() {
    (void)hipStreamSynchronize(c->stream);
    for (void* q : p) {
      if (c->P.dev_free) c->P.dev_free(q, c->P.alloc_user);
      else (void)hipFree(q);
    }
  }
};

// Inverses of the diagonal blocks of level l on the device (section 3; K7),
// colour by colour: the FP64 blocks from n_b colour residuals of unit
// vectors, FP64 Gauss-Jordan inverses of the equilibrated blocks, their
// symmetric parts into the tile layout of each precision.
void device_inverses(ldgs_ctx* c, size_t l, const std::vector<int64_t>& off, const int* elems, bool parity,
                     double* inv64, float* inv32, uint16_t* inv16, size_t st64, size_t st32, size_t st16) {
  const Level& L = c->levels[l];
  const int nb = c->g.nb;
  const DevLevel<double>& view = c->s64.lv[l].view;
  int64_t maxc = 0;
  for (int col = 0; col < L.ncol; ++col) maxc = std::max(maxc, off[col + 1] - off[col]);
  TempDev tmp(c);
  double* x = tmp.get<double>((size_t)L.NE * nb);
  double* b0 = tmp.get<double>((size_t)L.NE * nb);
  double* r = tmp.get<double>((size_t)maxc * nb);
  double* blk = tmp.get<double>((size_t)maxc * nb * nb);
  int* nsing = tmp.get<int>(1);
  LCHK(launch_fill<double>(c->stream, L.NE * nb, 0.0, x));
  LCHK(launch_fill<double>(c->stream, L.NE * nb, 0.0, b0));
  HIPCHK(hipMemsetAsync(nsing, 0, sizeof(int), c->stream));
  LaunchCfg cfg{c->g.d, c->g.p, c->stream, c->small_grid};
  for (int col = 0; col < L.ncol; ++col) {
    const int64_t o = off[col], cnt = off[col + 1] - o;
    if (cnt == 0) continue;
    for (int j = 0; j < nb; ++j) {
      LCHK(launch_set_unit(c->stream, cnt, elems + o, nb, j, x));
      LCHK(launch_colour_residual<double>(cfg, view, c->tab, elems + o, parity ? col : -1, cnt, b0, x, r));
      LCHK(launch_take_column(c->stream, cnt, nb, j, r, blk));
    }
    LCHK(launch_set_unit(c->stream, cnt, elems + o, nb, nb, x));   // x back to zero
    LCHK(launch_block_inverse(c->stream, cnt, nb, blk, nsing));
    if (inv64) LCHK(launch_arrange_sym(c->stream, cnt, nb, blk, inv64 + o * st64, 8, (int64_t)st64));
    if (inv32) LCHK(launch_arrange_sym(c->stream, cnt, nb, blk, inv32 + o * st32, 4, (int64_t)st32));
    if (inv16) LCHK(launch_arrange_sym(c->stream, cnt, nb, blk, inv16 + o * st16, 2, (int64_t)st16));
  }
  int h_sing = 0;
  HIPCHK(hipMemcpyAsync(&h_sing, nsing, sizeof(int), hipMemcpyDeviceToHost, c->stream));
  HIPCHK(hipStreamSynchronize(c->stream));
  if (h_sing > 0)
    throw Fail{LDGS_E_SINGULAR_BLOCK, std::to_string(h_sing) + " singular element blocks on level " + std::to_string(l)};
}

void build_inverses(ldgs_ctx* c, bool need64, bool need32, bool need16) {
  const int nb = c->g.nb;
  const size_t nb2 = (size_t)nb * nb;
  const int trs = sym_tiles(nb, 4).TR;
  const size_t st64 = (size_t)sym_tile_off(trs, sym_tiles(nb, 8).NTILE);
  const size_t st32 = (size_t)sym_tile_off(trs, sym_tiles(nb, 4).NTILE);
  const size_t st16 = (size_t)sym_tile_off(trs, sym_tiles(nb, 2).NTILE);
  for (size_t l = 0; l + 1 < c->levels.size(); ++l) {
    Level& L = c->levels[l];
    std::vector<int64_t> off(L.ncol + 1, 0);
    for (int col = 0; col < L.ncol; ++col) off[col + 1] = off[col] + (int64_t)L.elems[col].size();
    // colour-major element order; on levels with interphase faces each colour
    // lists first the elements the regular kernel can evaluate, then the rest
    std::vector<int> order;
    order.reserve(L.NE);
    std::vector<int64_t> reg(L.ncol, 0);
    bool iface = false;
    for (int k = 0; k < c->g.d; ++k)
      for (unsigned char t : L.faces[k].type) iface = iface || t == F_INTER;
    for (int col = 0; col < L.ncol; ++col) {
      std::vector<int> rest;
      for (int E : L.elems[col]) {
        if (iface && touches_interphase(L, c->g.d, E)) rest.push_back(E);
        else order.push_back(E);
      }
      reg[col] = (int64_t)L.elems[col].size() - (int64_t)rest.size();
      order.insert(order.end(), rest.begin(), rest.end());
    }
    // parity colouring with each colour in increasing order: the kernels
    // compute element ids from the launch index instead of reading them
    bool parity = !iface;
    {
      const int lgn = log2i(L.n), lgh = lgn - 1, hm = (1 << lgh) - 1;
      for (int col = 0; col < L.ncol && parity; ++col)
        for (int64_t i = 0; i < off[col + 1] - off[col] && parity; ++i) {
          int64_t E = 0;
          for (int k = 0; k < c->g.d; ++k) E |= ((((i >> (k * lgh)) & hm) << 1) | ((col >> k) & 1)) << (k * lgn);
          parity = order[off[col] + i] == E;
        }
    }
    if (L.uniform) {
      // one inverse for the level, held dense (FP64 for the FP64 cycle, FP32
      // for both the FP32 and the BF16-inverse cycles: nothing to stream)
      std::vector<double> A(nb2), inv(nb2);
      host_diag_block(L, c->g, c->B, c->P.form, 0, A.data());
      if (!block_inverse(nb, A.data(), inv.data(), 1e-14))
        throw Fail{LDGS_E_SINGULAR_BLOCK, "singular element block 0 on level " + std::to_string(l)};
      auto kmajor = [&](int bytes) {
        std::vector<double> t((size_t)shared_inverse_rows(nb, bytes) * nb, 0.0);
        for (int r = 0; r < nb; ++r)
          for (int k = 0; k < nb; ++k) t[(size_t)k * nb + r] = inv[(size_t)r * nb + k];
        return t;
      };
      int64_t maxc = 0;
      for (int col = 0; col < L.ncol; ++col) maxc = std::max(maxc, off[col + 1] - off[col]);
      double* dense_inv = upload<double>(c, inv);
      int* elems = dalloc<int>(c, L.NE);
      HIPCHK(hipMemcpy(elems, order.data(), order.size() * sizeof(int), hipMemcpyHostToDevice));
      auto set = [&](auto& S) {
        using T = std::remove_pointer_t<decltype(S.lv[l].x)>;
        PrecLevel<T>& pl = S.lv[l];
        pl.ainv_sh = upload<T>(c, kmajor((int)sizeof(T)));
        // the symmetric tile layout of the same inverse, for the one-launch pass
        const int tb = (int)sizeof(T);
        const size_t st = (size_t)sym_tile_off(trs, sym_tiles(nb, tb).NTILE);
        void* tiles = tb == 8 ? (void*)dalloc<double>(c, st) : (void*)dalloc<float>(c, st);
        LCHK(launch_arrange_sym(c->stream, 1, nb, dense_inv, tiles, tb, (int64_t)st));
        pl.ainv_tiles = tiles;
        pl.ainv_tiles_kind = tb == 8 ? 0 : 1;
        pl.rbuf = dalloc<T>(c, (size_t)maxc * nb);
        pl.inv = nullptr;
        pl.elems = elems;
        pl.col_off = off;
        pl.col_reg = reg;
        pl.inv_stride = 0;
        pl.parity = parity;
      };
      if (need64) set(c->s64);
      if (need32) set(c->s32);
      if (need16) set(c->s16);
      continue;
    }
    double* inv64 = need64 ? dalloc<double>(c, L.NE * st64) : nullptr;
    float* inv32 = need32 ? dalloc<float>(c, L.NE * st32) : nullptr;
    uint16_t* inv16 = need16 ? dalloc<uint16_t>(c, L.NE * st16) : nullptr;
    int* elems = dalloc<int>(c, L.NE);
    HIPCHK(hipMemcpy(elems, order.data(), order.size() * sizeof(int), hipMemcpyHostToDevice));
    const int64_t CH = c->device_setup ? 0 : 8192;
    if (c->device_setup) device_inverses(c, l, off, elems, parity, inv64, inv32, inv16, st64, st32, st16);
    std::vector<double> b64, b32, b16;
    std::vector<float> h32;
    std::vector<uint16_t> h16;
    for (int64_t p0 = 0; CH > 0 && p0 < L.NE; p0 += CH) {
      const int64_t cnt = std::min(CH, L.NE - p0);
      if (need64) b64.assign(cnt * st64, 0.0);
      if (need32) b32.assign(cnt * st32, 0.0);
      if (need16) b16.assign(cnt * st16, 0.0);
      int failed = -1;
#pragma omp parallel
      {
        std::vector<double> A(nb2), inv(nb2);
#pragma omp for schedule(dynamic, 16)
        for (int64_t i = 0; i < cnt; ++i) {
          const int64_t E = order[p0 + i];
          host_diag_block(L, c->g, c->B, c->P.form, E, A.data());
          if (!block_inverse(nb, A.data(), inv.data(), 1e-14)) {
#pragma omp critical
            failed = (int)E;
            continue;
          }
          if (need64) arrange_inverse(inv.data(), nb, 8, b64.data() + i * st64);
          if (need32) arrange_inverse(inv.data(), nb, 4, b32.data() + i * st32);
          if (need16) arrange_inverse(inv.data(), nb, 2, b16.data() + i * st16);
        }
      }
      if (failed >= 0)
        throw Fail{LDGS_E_SINGULAR_BLOCK, "singular element block " + std::to_string(failed) + " on level " +
                                              std::to_string(l)};
      if (inv64) HIPCHK(hipMemcpy(inv64 + p0 * st64, b64.data(), cnt * st64 * sizeof(double), hipMemcpyHostToDevice));
      if (inv32) {
        h32.assign(b32.begin(), b32.end());
        HIPCHK(hipMemcpy(inv32 + p0 * st32, h32.data(), cnt * st32 * sizeof(float), hipMemcpyHostToDevice));
      }
      if (inv16) {
        h16.resize(b16.size());
        for (size_t i = 0; i < b16.size(); ++i) h16[i] = to_bf16(b16[i]);
        HIPCHK(hipMemcpy(inv16 + p0 * st16, h16.data(), cnt * st16 * sizeof(uint16_t), hipMemcpyHostToDevice));
      }
    }
    if (c->split_pass && !iface) {
      int64_t maxc = 0;
      for (int col = 0; col < L.ncol; ++col) maxc = std::max(maxc, off[col + 1] - off[col]);
      if (need64) c->s64.lv[l].rbuf = dalloc<double>(c, (size_t)maxc * nb);
      if (need32 || need16) {
        float* rb = dalloc<float>(c, (size_t)maxc * nb);
        if (need32) c->s32.lv[l].rbuf = rb;
        if (need16) c->s16.lv[l].rbuf = rb;
      }
    }
    if (need64) { c->s64.lv[l].inv = inv64; c->s64.lv[l].inv_kind = 0; c->s64.lv[l].elems = elems; c->s64.lv[l].col_off = off; c->s64.lv[l].col_reg = reg; c->s64.lv[l].inv_stride = st64; c->s64.lv[l].parity = parity; }
    if (need32) { c->s32.lv[l].inv = inv32; c->s32.lv[l].inv_kind = 1; c->s32.lv[l].elems = elems; c->s32.lv[l].col_off = off; c->s32.lv[l].col_reg = reg; c->s32.lv[l].inv_stride = st32; c->s32.lv[l].parity = parity; }
    if (need16) { c->s16.lv[l].inv = inv16; c->s16.lv[l].inv_kind = 2; c->s16.lv[l].elems = elems; c->s16.lv[l].col_off = off; c->s16.lv[l].col_reg = reg; c->s16.lv[l].inv_stride = st16; c->s16.lv[l].parity = parity; }
  }
}

// Bottom solver (footnote to the bottom solver, section 3): eigendecomposition
// with the k0 smallest-magnitude eigenvalues snapped to zero, taken of the
// Jacobi-equilibrated operator D A D (D = |diag A|^{-1/2}); the solve matrix
// is D (D A D)^+ D, a generalized inverse of A on range(A).
void build_bottom(ldgs_ctx* c) {
  Level& L = c->levels.back();
  const int64_t N = L.NE * c->g.nb;
  c->Nc = N;
  std::vector<double> A((size_t)N * N), e(N, 0.0), col(N);
  for (int64_t j = 0; j < N; ++j) {
    e[j] = 1.0;
    host_apply(L, c->g, c->B, c->P.form, e.data(), col.data());
    e[j] = 0.0;
    for (int64_t i = 0; i < N; ++i) A[(size_t)i * N + j] = col[i];
  }
  c->h_Ac = A;
  std::vector<double> dg(N);
  for (int64_t i = 0; i < N; ++i) {
    double a = std::fabs(A[(size_t)i * N + i]);
    if (!(a > 0.0)) throw Fail{LDGS_E_SINGULAR_BLOCK, "zero diagonal entry in the bottom operator"};
    dg[i] = 1.0 / std::sqrt(a);
  }
  for (int64_t i = 0; i < N; ++i)
    for (int64_t j = i; j < N; ++j) {
      double s = 0.5 * (A[(size_t)i * N + j] + A[(size_t)j * N + i]) * dg[i] * dg[j];
      A[(size_t)i * N + j] = s;
      A[(size_t)j * N + i] = s;
    }
  std::vector<double> lam;
  sym_eigen((int)N, A, lam);
  c->h_eig = lam;
  std::vector<int64_t> idx(N);
  for (int64_t i = 0; i < N; ++i) idx[i] = i;
  std::sort(idx.begin(), idx.end(), [&](int64_t a, int64_t b) { return std::fabs(lam[a]) < std::fabs(lam[b]); });
  double lmax = std::fabs(lam[idx[N - 1]]);
  if (!(std::fabs(lam[idx[c->k0]]) > 1e-8 * lmax))
    throw Fail{LDGS_E_SINGULAR_BLOCK, "bottom operator has more near-zero eigenvalues than the trivial kernel"};
  std::vector<double> inv(N, 0.0);
  for (int64_t q = c->k0; q < N; ++q) inv[idx[q]] = 1.0 / lam[idx[q]];
  c->h_pinv.assign((size_t)N * N, 0.0);
  // D V diag(inv) V^T D
#pragma omp parallel for schedule(static)
  for (int64_t i = 0; i < N; ++i) {
    double* row = &c->h_pinv[(size_t)i * N];
    for (int64_t q = 0; q < N; ++q) {
      double viq = A[(size_t)i * N + q] * inv[q];
      if (viq == 0.0) continue;
      for (int64_t j = 0; j < N; ++j) row[j] += viq * A[(size_t)j * N + q];
    }
    for (int64_t j = 0; j < N; ++j) row[j] *= dg[i] * dg[j];
  }
}

void check_ctx(ldgs_ctx* c, bool device) {
  if (!c) throw Fail{LDGS_E_ARG, "null context"};
  if (device && c->host_only) throw Fail{LDGS_E_UNSUPPORTED, "context was built host_only"};
}

ldgs_status handle(ldgs_ctx* c, const Fail& f) {
  if (c) c->err = f.msg;
  return f.st;
}

// ---------------------------------------------------------------------------
// the V-cycle (Algorithm 1) on one precision store
// ---------------------------------------------------------------------------
hipEvent_t next_event(ldgs_ctx* c) {
  if (c->ev_used == c->ev_pool.size()) {
    hipEvent_t e;
    HIPCHK(hipEventCreate(&e));
    c->ev_pool.push_back(e);
  }
  return c->ev_pool[c->ev_used++];
}

template <typename T>
T* rf_scratch(ldgs_ctx* c) {
  if constexpr (sizeof(T) == 8) return c->w_rf64;
  else return c->w_rf32;
}

// Chunked colour passes of one level chained across colours (and sweeps):
// while the products of one colour's last chunks still run on the side
// stream, the next colour's first residual chunks start on the main stream.
// pending: the side stream holds products the main stream has not joined.
struct OvChain {
  bool pending = false;
  int l = -1;
  const void* x = nullptr;
  int64_t ch = 0;
  int64_t nch = 0;
};

// the main stream waits for every product queued on the side stream
void ov_join(ldgs_ctx* c, OvChain* chain) {
  if (!chain || !chain->pending) return;
  HIPCHK(hipEventRecord(c->ov_join, c->side));
  HIPCHK(hipStreamWaitEvent(c->stream, c->ov_join, 0));
  chain->pending = false;
}

// chain: null for a single pass (joined at its end); else the state of the
// passes before it, left pending for the caller to join with ov_join
template <typename T>
void smooth_colour(ldgs_ctx* c, PrecStore<T>& S, int l, int col, const T* b, T* x, OvChain* chain = nullptr) {
  LaunchCfg cfg{c->g.d, c->g.p, c->stream, c->small_grid};
  PrecLevel<T>& pl = S.lv[l];
  const size_t esz = pl.inv_kind == 0 ? 8 : (pl.inv_kind == 1 ? 4 : 2);
  int64_t o = pl.col_off[col], cnt = pl.col_off[col + 1] - o;
  const void* inv = (const char*)pl.inv + o * pl.inv_stride * esz;
  const int64_t nreg = pl.col_reg.empty() ? cnt : pl.col_reg[col];
  const int pcol = pl.parity ? col : -1;
  const bool chunked = !pl.ainv_sh && c->split_pass && pl.rbuf && !pl.view.iface && c->side &&
                       c->overlap_chunks > 1 && cnt >= c->overlap_min;
  if (!chunked) ov_join(c, chain);
  if (pl.ainv_sh && pl.ainv_tiles && cnt < c->fuse_shared_max) {
    // one inverse for the level, small colour: one launch, every element's
    // product with the same tiles (latency-bound launches: half of them)
    LCHK(launch_smooth_colour<T>(cfg, pl.view, c->tab, pl.elems + o, pcol, cnt, pl.ainv_tiles, pl.ainv_tiles_kind, b,
                                 x, true));
  } else if (pl.ainv_sh) {
    // one inverse for the level: residuals of the colour, then the shared update
    LCHK(launch_colour_residual<T>(cfg, pl.view, c->tab, pl.elems + o, pcol, cnt, b, x, pl.rbuf));
    LCHK(launch_shared_update<T>(c->stream, cnt, c->g.nb, pl.ainv_sh, pl.rbuf, pl.elems + o, x, 0, nullptr, 0,
                                 c->mfma_min));
  } else if (c->split_pass && pl.rbuf && !pl.view.iface) {
    if (chunked) {
      // chunk k's product on the side stream after chunk k's residuals, beside
      // the residuals of chunk k + 1
      LaunchCfg cfg_side = cfg;
      cfg_side.stream = c->side;
      const int64_t ch = (cnt + c->overlap_chunks - 1) / c->overlap_chunks;
      const int64_t nch = (cnt + ch - 1) / ch;
      // Chained after the previous colour's chunks (same level, x and chunk
      // bounds; parity colours only): the residuals of chunk q read x of the
      // previous colour only at positions within +-H of the chunk, H = 2 (n/2)^(d-1)
      // (each half-grid coordinate of a stencil neighbour differs by at most
      // one, or wraps on a periodic axis below the slowest), so they wait for
      // that colour's products up to the chunk holding position (q+1) ch - 1 + H,
      // all of them when the slowest axis is periodic.  Waiting for a later
      // chunk also orders the previous colour's reads of r chunk q before
      // this colour's residuals overwrite it (one side stream, in order).
      const bool chained = chain && chain->pending && chain->l == l && chain->x == (const void*)x &&
                           chain->ch == ch && chain->nch == nch && pcol >= 0;
      if (chain && chain->pending && !chained) ov_join(c, chain);
      const int64_t half = int64_t(1) << (pl.view.lgn - 1);
      int64_t H = 2;
      for (int k = 0; k + 1 < c->g.d; ++k) H *= half;
      const bool wrap = c->P.bc[c->g.d - 1] == LDGS_PERIODIC;
      for (int64_t q = 0; q < nch; ++q) {
        const int64_t lo = q * ch, n = std::min(ch, cnt - lo);
        if (chained) {
          const int64_t j = wrap ? nch - 1 : std::min(nch - 1, (lo + ch - 1 + H) / ch);
          HIPCHK(hipStreamWaitEvent(c->stream, c->ov_prod[j], 0));
        }
        LCHK(launch_colour_residual<T>(cfg, pl.view, c->tab, pl.elems + o, pcol, n, b, x, pl.rbuf, lo));
        HIPCHK(hipEventRecord(c->ov_fork, c->stream));
        HIPCHK(hipStreamWaitEvent(c->side, c->ov_fork, 0));
        LCHK(launch_apply_inverse<T>(cfg_side, pl.view.lgn, pl.elems + o, pcol, n, inv, pl.inv_kind, pl.rbuf, x, lo));
        HIPCHK(hipEventRecord(c->ov_prod[q], c->side));
      }
      if (chain) {
        chain->pending = true;
        chain->l = l;
        chain->x = (const void*)x;
        chain->ch = ch;
        chain->nch = nch;
      } else {
        HIPCHK(hipEventRecord(c->ov_join, c->side));
        HIPCHK(hipStreamWaitEvent(c->stream, c->ov_join, 0));
      }
    } else {
      // residuals of the colour, then the streamed product with the inverses
      LCHK(launch_colour_residual<T>(cfg, pl.view, c->tab, pl.elems + o, pcol, cnt, b, x, pl.rbuf));
      LCHK(launch_apply_inverse<T>(cfg, pl.view.lgn, pl.elems + o, pcol, cnt, inv, pl.inv_kind, pl.rbuf, x));
    }
  } else
  // (split only large launches: on coarse levels the second launch would cost
  // more than the extended stencil)
  if (!pl.view.iface || nreg == cnt || cnt < c->small_grid) {
    LCHK(launch_smooth_colour<T>(cfg, pl.view, c->tab, pl.elems + o, pcol, cnt, inv, pl.inv_kind, b, x));
  } else {
    // elements away from the interfaces: regular kernel; the rest: the
    // extended-stencil variant (the two ranges of one colour are uncoupled)
    DevLevel<T> regular = pl.view;
    regular.iface = 0;
    if (nreg > 0) LCHK(launch_smooth_colour<T>(cfg, regular, c->tab, pl.elems + o, -1, nreg, inv, pl.inv_kind, b, x));
    const void* inv_i = (const char*)inv + nreg * pl.inv_stride * esz;
    LCHK(launch_smooth_colour<T>(cfg, pl.view, c->tab, pl.elems + o + nreg, -1, cnt - nreg, inv_i, pl.inv_kind, b, x));
  }
}

// First colour pass from x = 0 (x need not be initialised): x_E = Ainv_E b_E
// on colour 0, every other element set to zero, in one launch.
template <typename T>
void first_colour(ldgs_ctx* c, PrecStore<T>& S, int l, const T* b, T* x) {
  LaunchCfg cfg{c->g.d, c->g.p, c->stream, c->small_grid};
  PrecLevel<T>& pl = S.lv[l];
  const int64_t cnt = pl.col_off[1], nzero = c->levels[l].NE - cnt;
  const int pcol = pl.parity ? 0 : -1;
  if (pl.ainv_sh)
    LCHK(launch_shared_update<T>(c->stream, cnt, c->g.nb, pl.ainv_sh, b, pl.elems, x, 1, pl.elems + cnt, nzero,
                                 c->mfma_min));
  else
    LCHK(launch_first_colour<T>(cfg, log2i(c->levels[l].n), pl.elems, pcol, cnt, pl.inv, pl.inv_kind, b, x,
                                pl.elems + cnt, nzero));
}

// sweeps of colour passes; zero_x: x is taken as zero on entry (and need not
// be initialised)
template <typename T>
void smooth(ldgs_ctx* c, PrecStore<T>& S, int l, const T* b, T* x, int sweeps, bool zero_x = false) {
  if (zero_x && sweeps == 0) LCHK(launch_fill<T>(c->stream, c->levels[l].NE * c->g.nb, (T)0, x));
  const int ncol = c->levels[l].ncol;
  OvChain chain;
  for (int s = 0; s < sweeps; ++s) {
    const bool first = zero_x && s == 0;
    // finest level, profiling on: every prof-th sweep whose passes all
    // evaluate the operator (not the one that starts from the zero guess)
    const bool timed = c->prof > 0 && l == 0 && !first && (c->prof_count++ % c->prof) == 0;
    hipEvent_t e0 = nullptr, e1 = nullptr;
    if (timed) {
      // a timed sweep holds its own passes only
      ov_join(c, &chain);
      e0 = next_event(c);
      e1 = next_event(c);
      HIPCHK(hipEventRecord(e0, c->stream));
    }
    for (int col = 0; col < ncol; ++col) {
      if (first && col == 0) {
        ov_join(c, &chain);
        first_colour(c, S, l, b, x);
      } else {
        smooth_colour(c, S, l, col, b, x, c->ov_chain ? &chain : nullptr);
      }
    }
    if (timed) {
      ov_join(c, &chain);
      HIPCHK(hipEventRecord(e1, c->stream));
      c->prof_ev.push_back({e0, e1, ncol});
    }
  }
  ov_join(c, &chain);
}

// Least-squares bottom solve x = A_c^+ b (footnote to the bottom solver):
// the eigendecomposition pseudo-inverse, applied in FP64 with one step of
// iterative refinement, x = y + A_c^+ (b - A_c y) with y = A_c^+ b.
template <typename T>
void bottom_solve(ldgs_ctx* c, const T* b, T* x) {
  const int64_t N = c->Nc;
  const double* b64;
  if constexpr (sizeof(T) == 8) {
    b64 = (const double*)b;
  } else {
    LCHK(launch_cast_f2d_add(c->stream, N, (const float*)b, c->d_bt0, 0));
    b64 = c->d_bt0;
  }
  LCHK((launch_dense_mv<double, double>(c->stream, N, c->d_pinv, b64, nullptr, 1.0, c->d_bt1)));
  LCHK((launch_dense_mv<double, double>(c->stream, N, c->d_Ac, c->d_bt1, b64, -1.0, c->d_bt2)));
  LCHK((launch_dense_mv<double, T>(c->stream, N, c->d_pinv, c->d_bt2, c->d_bt1, 1.0, x)));
}

// ---------------------------------------------------------------------------
// implicitly defined meshes: device data and the V-cycle on explicit blocks

int* upload_int(ldgs_ctx* c, const std::vector<int>& v) {
  int* d = dalloc<int>(c, v.size());
  if (!v.empty()) HIPCHK(hipMemcpy(d, v.data(), v.size() * sizeof(int), hipMemcpyHostToDevice));
  return d;
}

void imp_device(ldgs_ctx* c) {
  const ImpHier& H = *c->imp;
  const int mask = (1 << c->P.vprec) | c->P.build_precisions;
  c->imp64 = mask & 1;
  c->imp32 = (mask & 2) != 0;
  const size_t nl = H.lv.size();
  c->idev.assign(nl, ldgs_ctx::ImpDev{});
  for (size_t l = 0; l < nl; ++l) {
    const ImpLevel& L = H.lv[l];
    ldgs_ctx::ImpDev& D = c->idev[l];
    D.NE = L.NE;
    const int64_t N = L.NE * H.nb;
    D.rowptr = upload_int(c, L.rowptr);
    D.cols = upload_int(c, L.cols);
    // the FP64 finest operator always (outer residual and products)
    if (c->imp64 || l == 0) D.blk64 = upload<double>(c, L.blk.data(), L.blk.size());
    if (c->imp32) D.blk32 = upload<float>(c, L.blk.data(), L.blk.size());
    if (l + 1 < nl) {
      if (c->imp64) D.inv64 = upload<double>(c, L.inv.data(), L.inv.size());
      if (c->imp32) D.inv32 = upload<float>(c, L.inv.data(), L.inv.size());
      D.parent = upload_int(c, L.parent);
      if (c->imp64) D.I64 = upload<double>(c, L.Iblk);
      if (c->imp32) D.I32 = upload<float>(c, L.Iblk);
      for (const auto& e : L.elems) {
        D.elems.push_back(upload_int(c, e));
        D.ncnt.push_back((int64_t)e.size());
      }
    }
    if (l > 0) {
      D.kid_ptr = upload_int(c, L.kid_ptr);
      D.kids = upload_int(c, L.kids);
      if (c->imp64) {
        D.b64 = dalloc<double>(c, N);
        D.x64 = dalloc<double>(c, N);
      }
      if (c->imp32) {
        D.b32 = dalloc<float>(c, N);
        D.x32 = dalloc<float>(c, N);
      }
    }
    if (l + 1 < nl) {
      if (c->imp64) D.r64 = dalloc<double>(c, N);
      if (c->imp32) D.r32 = dalloc<float>(c, N);
    }
  }
  c->d_pinv = upload<double>(c, H.pinv);
  c->d_Ac = upload<double>(c, H.Ac);
  c->d_bt0 = dalloc<double>(c, c->Nc);
  c->d_bt1 = dalloc<double>(c, c->Nc);
  c->d_bt2 = dalloc<double>(c, c->Nc);
  const int64_t N = c->ndof();
  c->w_b = dalloc<double>(c, N);
  c->w_x = dalloc<double>(c, N);
  c->w_r = dalloc<double>(c, N);
  c->w_z = dalloc<double>(c, N);
  c->w_part = dalloc<double>(c, 1024);
  if (c->imp32) {
    c->w_b32 = dalloc<float>(c, N);
    c->w_x32 = dalloc<float>(c, N);
  }
  c->d_kernel = upload<double>(c, H.kernel);
  if (c->P.diag_scaling) {
    const std::vector<double>& ds = H.lv[0].dscale;
    std::vector<double> inv(ds.size());
    for (size_t i = 0; i < ds.size(); ++i) inv[i] = 1.0 / ds[i];
    c->d_dscale0 = upload<double>(c, ds);
    c->d_dinv0 = upload<double>(c, inv);
  }
  c->s64.built = c->imp64;
  c->s32.built = c->imp32;
  HIPCHK(hipDeviceSynchronize());
}

template <typename T>
struct ImpArrays;
template <>
struct ImpArrays<double> {
  static const double* blk(const ldgs_ctx::ImpDev& D) { return D.blk64; }
  static const double* inv(const ldgs_ctx::ImpDev& D) { return D.inv64; }
  static const double* I(const ldgs_ctx::ImpDev& D) { return D.I64; }
  static double* b(ldgs_ctx::ImpDev& D) { return D.b64; }
  static double* x(ldgs_ctx::ImpDev& D) { return D.x64; }
  static double* r(ldgs_ctx::ImpDev& D) { return D.r64; }
};
template <>
struct ImpArrays<float> {
  static const float* blk(const ldgs_ctx::ImpDev& D) { return D.blk32; }
  static const float* inv(const ldgs_ctx::ImpDev& D) { return D.inv32; }
  static const float* I(const ldgs_ctx::ImpDev& D) { return D.I32; }
  static float* b(ldgs_ctx::ImpDev& D) { return D.b32; }
  static float* x(ldgs_ctx::ImpDev& D) { return D.x32; }
  static float* r(ldgs_ctx::ImpDev& D) { return D.r32; }
};

template <typename T>
void imp_colour(ldgs_ctx* c, int l, int col, const T* b, T* x) {
  using A = ImpArrays<T>;
  ldgs_ctx::ImpDev& D = c->idev[l];
  LCHK(launch_bsr_colour<T>(c->stream, c->imp->nb, D.ncnt[col], D.elems[col], D.rowptr, D.cols, A::blk(D),
                            A::inv(D), b, x));
}

// sweeps of colour passes on level l; on the finest level with pass timing
// on, every prof-th sweep is bracketed by an event pair
template <typename T>
void imp_smooth(ldgs_ctx* c, int l, const T* b, T* x, int sweeps) {
  const int ncol = (int)c->idev[l].elems.size();
  for (int s = 0; s < sweeps; ++s) {
    const bool timed = c->prof > 0 && l == 0 && (c->prof_count++ % c->prof) == 0;
    hipEvent_t e0 = nullptr, e1 = nullptr;
    if (timed) {
      e0 = next_event(c);
      e1 = next_event(c);
      HIPCHK(hipEventRecord(e0, c->stream));
    }
    for (int col = 0; col < ncol; ++col) imp_colour<T>(c, l, col, b, x);
    if (timed) {
      HIPCHK(hipEventRecord(e1, c->stream));
      c->prof_ev.push_back({e0, e1, ncol});
    }
  }
}

template <typename T>
void imp_cycle(ldgs_ctx* c, int l, const T* b, T* x, bool zero_x) {
  using A = ImpArrays<T>;
  const int bottom = (int)c->idev.size() - 1;
  if (l == bottom) {
    bottom_solve(c, b, x);
    return;
  }
  ldgs_ctx::ImpDev& D = c->idev[l];
  ldgs_ctx::ImpDev& C = c->idev[l + 1];
  const int nb = c->imp->nb;
  if (zero_x) LCHK(launch_fill<T>(c->stream, D.NE * nb, (T)0, x));
  imp_smooth<T>(c, l, b, x, c->P.nu1);
  LCHK(launch_bsr_residual<T>(c->stream, nb, D.NE, D.rowptr, D.cols, A::blk(D), b, x, A::r(D), nullptr));
  LCHK(launch_bsr_restrict<T>(c->stream, nb, C.NE, C.kid_ptr, C.kids, A::I(D), A::r(D), A::b(C)));
  imp_cycle<T>(c, l + 1, A::b(C), A::x(C), true);
  LCHK(launch_bsr_prolong<T>(c->stream, nb, D.NE, D.parent, A::I(D), A::x(C), x));
  imp_smooth<T>(c, l, b, x, c->P.nu2);
}

// V-cycle on level l; zero_x: x is taken as zero on entry (the coarse levels'
// corrections, and the finest level inside the outer iterations)
template <typename T>
void cycle(ldgs_ctx* c, PrecStore<T>& S, int l, const T* b, T* x, bool zero_x) {
  const int bottom = (int)c->levels.size() - 1;
  LaunchCfg cfg{c->g.d, c->g.p, c->stream, c->small_grid};
  if (l == bottom) {
    bottom_solve(c, b, x);    // overwrites x
    return;
  }
  smooth(c, S, l, b, x, c->P.nu1, zero_x);
  PrecLevel<T>& nx = S.lv[l + 1];
  LCHK(launch_residual_restrict<T>(cfg, S.lv[l].view, c->tab, b, x, nx.b, rf_scratch<T>(c)));
  cycle(c, S, l + 1, nx.b, nx.x, true);
  LCHK(launch_prolong_add<T>(cfg, c->levels[l].n, c->tab, nx.x, x));
  smooth(c, S, l, b, x, c->P.nu2);
}

// One V-cycle on the context's finest work vectors, replayed from a captured
// graph (captured on first use: the launch sequence and every pointer are
// fixed after setup).  A replay takes the host about half the time of the
// ~170 stream launches of a cycle; on the benchmark problem the GPU is the
// slower side either way.  Any failure to capture falls back to direct
// launches for the context's life.
// Runs launch() (one V-cycle's launches on c->stream) from a graph captured
// on first use for the key (vp, zero_x); timed cycles (pass timing on) and
// contexts whose capture failed launch directly.
template <class Launch>
void run_captured(ldgs_ctx* c, int vp, bool zero_x, Launch&& launch) {
  // timed cycles are launched directly: events recorded inside a captured
  // graph cannot be timed from the host
  if (!c->use_graph || c->prof > 0) {
    launch();
    return;
  }
  ldgs_ctx::CycleGraph* g = nullptr;
  for (auto& e : c->graphs)
    if (e.vp == vp && e.zero_x == zero_x) g = &e;
  if (!g) {
    hipGraph_t graph = nullptr;
    if (hipStreamBeginCapture(c->stream, hipStreamCaptureModeThreadLocal) != hipSuccess) {
      (void)hipGetLastError();
      c->use_graph = false;
      launch();
      return;
    }
    try {
      launch();
    } catch (...) {
      (void)hipStreamEndCapture(c->stream, &graph);
      if (graph) (void)hipGraphDestroy(graph);
      (void)hipGetLastError();
      throw;
    }
    hipGraphExec_t exec = nullptr;
    const bool ok = hipStreamEndCapture(c->stream, &graph) == hipSuccess && graph &&
                    hipGraphInstantiate(&exec, graph, nullptr, nullptr, 0) == hipSuccess;
    if (graph) (void)hipGraphDestroy(graph);
    if (!ok) {
      (void)hipGetLastError();
      c->use_graph = false;
      launch();
      return;
    }
    c->graphs.push_back({vp, zero_x, exec});
    g = &c->graphs.back();
  }
  HIPCHK(hipGraphLaunch(g->exec, c->stream));
}

template <typename T>
void run_cycle(ldgs_ctx* c, PrecStore<T>& S, int vp, T* b, T* x, bool zero_x) {
  run_captured(c, vp, zero_x, [&]() { cycle<T>(c, S, 0, b, x, zero_x); });
}

const double* dscale0(ldgs_ctx* c) { return c->P.diag_scaling ? c->d_dscale0 : nullptr; }

// x <- V(b, x) on user (unscaled, FP64) vectors in precision vp.
// If zero_x, x is taken as zero on entry (and overwritten).
// add: x += V(b, 0) instead (with zero_x)
void vcycle_user(ldgs_ctx* c, int vp, const double* b, double* x, bool zero_x, bool add = false) {
  const double* ds = dscale0(c);
  if (c->imp) {
    const int64_t NE = c->imp->lv[0].NE;
    const int nb = c->imp->nb, nvel = 2 * c->imp->nq;
    if (vp == LDGS_V_FP64) {
      if (!c->imp64) throw Fail{LDGS_E_UNSUPPORTED, "FP64 V-cycle not built"};
      LCHK((launch_scale_cast<double, double>(c->stream, NE, nb, nvel, ds, b, c->w_b, 0, 0)));
      if (!zero_x) LCHK((launch_scale_cast<double, double>(c->stream, NE, nb, nvel, ds, x, c->w_x, 1, 0)));
      run_captured(c, vp, zero_x, [&]() { imp_cycle<double>(c, 0, c->w_b, c->w_x, zero_x); });
      LCHK((launch_scale_cast<double, double>(c->stream, NE, nb, nvel, ds, c->w_x, x, 0, add ? 1 : 0)));
    } else if (vp == LDGS_V_FP32) {
      if (!c->imp32) throw Fail{LDGS_E_UNSUPPORTED, "FP32 V-cycle not built"};
      LCHK((launch_scale_cast<double, float>(c->stream, NE, nb, nvel, ds, b, c->w_b32, 0, 0)));
      if (!zero_x) LCHK((launch_scale_cast<double, float>(c->stream, NE, nb, nvel, ds, x, c->w_x32, 1, 0)));
      run_captured(c, vp, zero_x, [&]() { imp_cycle<float>(c, 0, c->w_b32, c->w_x32, zero_x); });
      LCHK((launch_scale_cast<float, double>(c->stream, NE, nb, nvel, ds, c->w_x32, x, 0, add ? 1 : 0)));
    } else {
      throw Fail{LDGS_E_UNSUPPORTED, "BF16-stored blocks are not built on implicitly defined meshes"};
    }
    return;
  }
  const int64_t NE = c->levels[0].NE;
  const int nb = c->g.nb, nvel = c->g.d * c->g.nq;
  if (vp == LDGS_V_FP64) {
    if (!c->s64.built) throw Fail{LDGS_E_UNSUPPORTED, "FP64 V-cycle not built"};
    LCHK((launch_scale_cast<double, double>(c->stream, NE, nb, nvel, ds, b, c->w_b, 0, 0)));
    if (!zero_x) LCHK((launch_scale_cast<double, double>(c->stream, NE, nb, nvel, ds, x, c->w_x, 1, 0)));
    run_cycle<double>(c, c->s64, vp, c->w_b, c->w_x, zero_x);
    LCHK((launch_scale_cast<double, double>(c->stream, NE, nb, nvel, ds, c->w_x, x, 0, add ? 1 : 0)));
  } else {
    PrecStore<float>& S = (vp == LDGS_V_FP32) ? c->s32 : c->s16;
    if (!S.built) throw Fail{LDGS_E_UNSUPPORTED, "requested V-cycle precision not built"};
    LCHK((launch_scale_cast<double, float>(c->stream, NE, nb, nvel, ds, b, c->w_b32, 0, 0)));
    if (!zero_x) LCHK((launch_scale_cast<double, float>(c->stream, NE, nb, nvel, ds, x, c->w_x32, 1, 0)));
    run_cycle<float>(c, S, vp, c->w_b32, c->w_x32, zero_x);
    LCHK((launch_scale_cast<float, double>(c->stream, NE, nb, nvel, ds, c->w_x32, x, 0, add ? 1 : 0)));
  }
}

// z += V(r, 0) in precision vp (r, z user vectors)
void precond_add(ldgs_ctx* c, int vp, const double* r, double* z) {
  vcycle_user(c, vp, r, z, true, true);   // the final unscaling cast adds into z
}

double host_sum_partials(ldgs_ctx* c, int nblk) {
  std::vector<double> h(nblk);
  HIPCHK(hipMemcpyAsync(h.data(), c->w_part, nblk * sizeof(double), hipMemcpyDeviceToHost, c->stream));
  HIPCHK(hipStreamSynchronize(c->stream));
  double s = 0.0;
  for (double v : h) s += v;
  return s;
}

double dot(ldgs_ctx* c, const double* x, const double* y) {
  const int nblk = 512;
  LCHK(launch_dot_partial(c->stream, c->ndof(), x, y, c->w_part, nblk));
  return host_sum_partials(c, nblk);
}

// Modified Gram-Schmidt of w against V[0..j]: h[i] = <w, V[i]>, w -= h[i] V[i]
// in turn; returns ||w||.  Each update is fused with the next inner product
// (the last with ||w||^2), which sums exactly as the separate launches do.
double mgs(ldgs_ctx* c, double* const* V, int j, double* w, double* h) {
  const int nblk = 512;
  double hij = dot(c, w, V[0]);
  for (int i = 0; i <= j; ++i) {
    h[i] = hij;
    LCHK(launch_axpy_dot_partial(c->stream, c->ndof(), -hij, V[i], w, i < j ? V[i + 1] : nullptr, c->w_part, nblk));
    hij = host_sum_partials(c, nblk);
  }
  return std::sqrt(hij);
}

void residual_fine(ldgs_ctx* c, const double* b, const double* x, double* r) {
  if (c->imp) {
    const ldgs_ctx::ImpDev& D = c->idev[0];
    LCHK(launch_bsr_residual<double>(c->stream, c->imp->nb, D.NE, D.rowptr, D.cols, D.blk64, b, x, r, c->d_dinv0));
    return;
  }
  LaunchCfg cfg{c->g.d, c->g.p, c->stream, c->small_grid};
  LCHK(launch_residual<double>(cfg, c->s64.lv[0].unscaled, c->tab, b, x, r, 0));
}

// y = A x with the unscaled finest operator
void apply_fine(ldgs_ctx* c, const double* x, double* y) {
  if (c->imp) {
    const ldgs_ctx::ImpDev& D = c->idev[0];
    LCHK(launch_bsr_residual<double>(c->stream, c->imp->nb, D.NE, D.rowptr, D.cols, D.blk64, nullptr, x, y,
                                     c->d_dinv0));
    return;
  }
  LaunchCfg cfg{c->g.d, c->g.p, c->stream, c->small_grid};
  LCHK(launch_residual<double>(cfg, c->s64.lv[0].unscaled, c->tab, nullptr, x, y, 1));
}

void project_kernel(ldgs_ctx* c, double* v) {
  if (c->imp) {
    // the constant pressure: v -= K (K^T v), K of unit norm
    const int nblk = 512;
    LCHK(launch_dot_partial(c->stream, c->ndof(), c->d_kernel, v, c->w_part, nblk));
    const double w = host_sum_partials(c, nblk);
    LCHK(launch_axpy(c->stream, c->ndof(), -w, c->d_kernel, v));
    return;
  }
  const Level& L = c->levels[0];
  const int64_t NE = L.NE;
  const int nblk = 256;
  for (int off : c->kernel_offsets) {
    LCHK(launch_strided_sum_partial(c->stream, NE, c->g.nb, off, v, c->w_part, nblk));
    double mean = host_sum_partials(c, nblk) / (double)NE;
    LCHK(launch_strided_add(c->stream, NE, c->g.nb, off, -mean, v));
  }
  if (c->rotations) {
    // rotation (x_a - 1/2) e_b - (x_b - 1/2) e_a, a < b: per element the mean
    // coefficient m(E) = x_a(centre) - 1/2 and the linear coefficient h / (2
    // sqrt 3) (times the common factor h^{d/2}), of u_b, and minus those of
    // x_b in u_a; orthogonal to the translations and to each other
    const int d = c->g.d, n = L.n;
    const double lin = L.h / (2.0 * std::sqrt(3.0));
    double cc = 0.0;   // sum over elements of m(E)^2 along one axis, times n^{d-1}
    for (int i = 0; i < n; ++i) {
      const double m = (i + 0.5) * L.h - 0.5;
      cc += m * m;
    }
    cc *= (double)NE / n;
    const double rr = 2.0 * (cc + (double)NE * lin * lin);
    for (int a = 0; a < d; ++a)
      for (int b = a + 1; b < d; ++b) {
        LCHK(launch_rotation_dot_partial(c->stream, d, c->g.p, log2i(n), L.h, a, b, v, c->w_part, nblk));
        const double w = host_sum_partials(c, nblk) / rr;
        LCHK(launch_rotation_axpy(c->stream, d, c->g.p, log2i(n), L.h, a, b, -w, v));
      }
  }
}

// ---------------------------------------------------------------------------
// learned correction
// ---------------------------------------------------------------------------
int periodic_mask(const ldgs_problem& P) {
  int m = 0;
  for (int k = 0; k < P.dim; ++k)
    if (P.bc[k] == LDGS_PERIODIC) m |= 1 << k;
  return m;
}

// flat host layout <-> padded device layout
void net_pack(const NetShape& s, const float* flat, std::vector<float>& pad) {
  const int H = NET_H;
  pad.assign(s.total, 0.f);
  const float* q = flat;
  for (int h = 0; h < H; ++h)
    for (int o = 0; o < s.noff; ++o)
      for (int c = 0; c < s.ch; ++c) pad[s.oW1 + (int64_t)h * s.k1p + o * s.chp + c] = *q++;
  for (int h = 0; h < H; ++h) pad[s.ob1 + h] = *q++;
  for (int i = 0; i < H * H; ++i) pad[s.oW2 + i] = *q++;
  for (int h = 0; h < H; ++h) pad[s.ob2 + h] = *q++;
  for (int o = 0; o < s.nb; ++o)
    for (int h = 0; h < H; ++h) pad[s.oW3 + (int64_t)o * H + h] = *q++;
  for (int o = 0; o < s.nb; ++o) pad[s.ob3 + o] = *q++;
}
// per-context buffers of the correction (allocated once)
void learned_buffers(ldgs_ctx* c) {
  if (c->d_logmu) return;
  const Level& L = c->levels[0];
  const int nq = c->g.nq;
  std::vector<float> lm(L.NE);
  for (int64_t e = 0; e < L.NE; ++e)
    lm[e] = (float)std::log10(L.mu_is_const ? L.mu_c : L.mmu[(size_t)e * nq * nq]);
  c->d_logmu = dalloc<float>(c, L.NE);
  HIPCHK(hipMemcpy(c->d_logmu, lm.data(), lm.size() * sizeof(float), hipMemcpyHostToDevice));
  c->d_sums = dalloc<double>(c, 2);
  c->d_mr = dalloc<double>(c, 3);
  const int64_t N = c->ndof();
  c->w_xold = dalloc<double>(c, N);
  c->w_zl = dalloc<double>(c, N);
}

NetDev net_dev(ldgs_ctx* c) { return NetDev{c->d_net, c->d_netbf}; }

constexpr int SUMSQ_BLK = 512;

// out = base + N(r') with r' = (b - A x) of the V-cycle's finest level as it
// stands after the last cycle (scaled variables; unscaled inside the kernel)
// Minimal-residual correction after a V-cycle: out = z + w dx with
// dx = N(r'), r' = b - A z the residual the cycle leaves (its own precision and
// variables), and w = <r', A dx> / ||A dx||^2 in those variables (the diagonally
// scaled system when the scaling is on), so that ||r' - w A dx|| <= ||r'||.
// z is the cycle's result in user variables; its internal copies of b and z
// (w_b/w_x or w_b32/w_x32) must be those of the cycle just run.  out may be z.
void learned_minres(ldgs_ctx* c, int vp, const double* z, double* out) {
  LaunchCfg cfg{c->g.d, c->g.p, c->stream, c->small_grid};
  const Level& L = c->levels[0];
  const int64_t NE = L.NE, N = c->ndof();
  const int nb = c->g.nb, nvel = c->g.d * c->g.nq;
  const double* ds = dscale0(c);
  const double cu = (double)NE * nvel, cp = (double)NE * (nb - nvel);
  if (!c->w_dx) c->w_dx = dalloc<double>(c, N);
  const bool full = c->learned_full_step;
  if (vp == LDGS_V_FP64) {
    if (!c->w_r64b) c->w_r64b = dalloc<double>(c, N);
    if (!c->w_adx64) c->w_adx64 = dalloc<double>(c, N);
    LCHK(launch_residual<double>(cfg, c->s64.lv[0].view, c->tab, c->w_b, c->w_x, c->w_r64b, 0));
    LCHK(launch_field_sumsq<double>(c->stream, NE, nb, nvel, c->w_r64b, ds, c->w_part, SUMSQ_BLK, c->d_sums));
    LCHK(launch_net_apply<double>(c->stream, c->g.d, c->g.p, L.n, log2i(L.n), periodic_mask(c->P), c->w_r64b, ds,
                                  c->d_logmu, c->d_sums, cu, cp, c->c_net[0], c->c_net[1], net_dev(c), nullptr,
                                  c->w_dx));
    if (!full) {
      // A dx in the cycle's variables (w_x is free once r' is formed)
      LCHK((launch_scale_cast<double, double>(c->stream, NE, nb, nvel, ds, c->w_dx, c->w_x, 1, 0)));
      LCHK(launch_residual<double>(cfg, c->s64.lv[0].view, c->tab, nullptr, c->w_x, c->w_adx64, 1));
      LCHK(launch_minres_sums<double>(c->stream, N, c->w_r64b, c->w_adx64, c->w_part, SUMSQ_BLK, c->d_mr));
    }
  } else {
    PrecStore<float>& S = (vp == LDGS_V_FP32) ? c->s32 : c->s16;
    if (!c->w_r32) c->w_r32 = dalloc<float>(c, N);
    if (!c->w_adx32) c->w_adx32 = dalloc<float>(c, N);
    LCHK(launch_residual<float>(cfg, S.lv[0].view, c->tab, c->w_b32, c->w_x32, c->w_r32, 0));
    LCHK(launch_field_sumsq<float>(c->stream, NE, nb, nvel, c->w_r32, ds, c->w_part, SUMSQ_BLK, c->d_sums));
    LCHK(launch_net_apply<float>(c->stream, c->g.d, c->g.p, L.n, log2i(L.n), periodic_mask(c->P), c->w_r32, ds,
                                 c->d_logmu, c->d_sums, cu, cp, c->c_net[0], c->c_net[1], net_dev(c), nullptr,
                                 c->w_dx));
    if (!full) {
      LCHK((launch_scale_cast<double, float>(c->stream, NE, nb, nvel, ds, c->w_dx, c->w_x32, 1, 0)));
      LCHK(launch_residual<float>(cfg, S.lv[0].view, c->tab, nullptr, c->w_x32, c->w_adx32, 1));
      LCHK(launch_minres_sums<float>(c->stream, N, c->w_r32, c->w_adx32, c->w_part, SUMSQ_BLK, c->d_mr));
    }
  }
  LCHK(launch_minres_update(c->stream, N, full ? nullptr : c->d_mr, z, c->w_dx, out));
  ++c->learned_steps;
}

// RAII device buffers for the context-free training entry point
struct DevBufs {
  std::vector<void*> p;
  template <typename T>
  T* get(size_t n) {
    void* q = nullptr;
    hipError_t e = hipMalloc(&q, (n ? n : 1) * sizeof(T));
    if (e != hipSuccess) throw Fail{LDGS_E_NOMEM, std::string("hipMalloc: ") + hipGetErrorString(e)};
    p.push_back(q);
    return (T*)q;
  }
  ~DevBufs() {
    for (void* q : p) (void)hipFree(q);
  }
};

// device buffers of one training run: FP32 master parameters and their BF16
// copy (padded layout), gradient, Adam moments, per-step losses, batch order
struct TrainBufs {
  float* w;
  uint16_t* wbf;
  float* g;
  float* m;
  float* v;
  double* dl;
  int* ord;
};

NetShape check_train_args(const ldgs_train_args* a, const float* params) {
  if (!a || !params || !a->feat || !a->targ || !a->order) throw Fail{LDGS_E_ARG, "null argument"};
  if ((a->dim != 2 && a->dim != 3) || a->degree < 1 || a->degree > (a->dim == 2 ? 3 : 2))
    throw Fail{LDGS_E_UNSUPPORTED, "dim/degree"};
  if (a->hidden != NET_H) throw Fail{LDGS_E_UNSUPPORTED, "hidden width must be 16"};
  if (!pow2(a->crop) || a->crop < 4) throw Fail{LDGS_E_ARG, "crop must be a power of two >= 4"};
  if (a->batch < 1 || a->steps < 0 || a->ncrops < 1) throw Fail{LDGS_E_ARG, "batch/steps/ncrops"};
  if (!(a->c_vel > 0) || !(a->c_pre > 0) || !(a->lr > 0)) throw Fail{LDGS_E_ARG, "scales and lr must be positive"};
  for (int64_t i = 0; i < (int64_t)a->steps * a->batch; ++i)
    if (a->order[i] < 0 || a->order[i] >= a->ncrops) throw Fail{LDGS_E_ARG, "order index out of range"};
  return net_shape(a->dim, a->degree);
}

// Host flat parameter layout <-> padded device layout, copied directly
// between host and device memory (2D copies place each first-layer row
// group at its padded offset; the padding itself must be zero beforehand).
void net_upload(const NetShape& s, const float* flat, float* dev, hipStream_t st) {
  const int H = NET_H;
  const size_t f = sizeof(float);
  for (int h = 0; h < H; ++h)
    HIPCHK(hipMemcpy2DAsync(dev + s.oW1 + (int64_t)h * s.k1p, s.chp * f, flat + (int64_t)h * s.noff * s.ch, s.ch * f,
                            s.ch * f, s.noff, hipMemcpyHostToDevice, st));
  const float* q = flat + (int64_t)H * s.noff * s.ch;
  HIPCHK(hipMemcpyAsync(dev + s.ob1, q, (2 * H + H * H) * f, hipMemcpyHostToDevice, st));   // b1 | W2 | b2
  q += 2 * H + H * H;
  HIPCHK(hipMemcpyAsync(dev + s.oW3, q, (size_t)s.nb * H * f, hipMemcpyHostToDevice, st));
  q += (int64_t)s.nb * H;
  HIPCHK(hipMemcpyAsync(dev + s.ob3, q, s.nb * f, hipMemcpyHostToDevice, st));
}
void net_download(const NetShape& s, const float* dev, float* flat, hipStream_t st) {
  const int H = NET_H;
  const size_t f = sizeof(float);
  for (int h = 0; h < H; ++h)
    HIPCHK(hipMemcpy2DAsync(flat + (int64_t)h * s.noff * s.ch, s.ch * f, dev + s.oW1 + (int64_t)h * s.k1p, s.chp * f,
                            s.ch * f, s.noff, hipMemcpyDeviceToHost, st));
  float* q = flat + (int64_t)H * s.noff * s.ch;
  HIPCHK(hipMemcpyAsync(q, dev + s.ob1, (2 * H + H * H) * f, hipMemcpyDeviceToHost, st));
  q += 2 * H + H * H;
  HIPCHK(hipMemcpyAsync(q, dev + s.oW3, (size_t)s.nb * H * f, hipMemcpyDeviceToHost, st));
  q += (int64_t)s.nb * H;
  HIPCHK(hipMemcpyAsync(q, dev + s.ob3, s.nb * f, hipMemcpyDeviceToHost, st));
}

// The training loop on given device buffers: Adam on the FP32 master
// weights, forward/backward in BF16 with FP32 accumulation.  Every buffer is
// initialised here (parameters uploaded over a zeroed padding, gradient,
// moments and losses zero-filled by kernels).
void train_run(const ldgs_train_args* a, const NetShape& ns, const TrainBufs& T, float* params, double* loss_out,
               float* grad0_out) {
  hipStream_t st = (hipStream_t)a->hip_stream;
  const int nsteps = a->steps > 0 ? a->steps : 1;
  LCHK(launch_fill<float>(st, ns.total, 0.f, T.w));
  net_upload(ns, params, T.w, st);
  HIPCHK(hipMemcpyAsync(T.ord, a->order, (size_t)std::max(a->steps, 1) * a->batch * sizeof(int),
                        hipMemcpyHostToDevice, st));
  LCHK(launch_to_bf16(st, ns.total, T.w, T.wbf));
  LCHK(launch_fill<float>(st, ns.total, 0.f, T.m));
  LCHK(launch_fill<float>(st, ns.total, 0.f, T.v));
  LCHK(launch_fill<double>(st, nsteps, 0.0, T.dl));
  int64_t Cd = 1;
  for (int k = 0; k < a->dim; ++k) Cd *= a->crop;
  const double inv_count = 1.0 / ((double)a->batch * Cd * ns.nb);
  const int steps_run = (a->steps == 0 && grad0_out) ? 1 : a->steps;
  for (int s = 0; s < steps_run; ++s) {
    LCHK(launch_fill<float>(st, ns.total, 0.f, T.g));
    LCHK(launch_train_grad(st, a->dim, a->degree, a->crop, log2i(a->crop), a->batch, T.ord + (int64_t)s * a->batch,
                           a->feat, a->targ, a->c_vel, a->c_pre, inv_count, NetDev{T.w, T.wbf}, T.g, T.dl + s));
    if (s == 0 && grad0_out) net_download(ns, T.g, grad0_out, st);
    if (a->steps == 0) break;
    const int t = s + 1;
    const float bc1 = (float)(1.0 / (1.0 - std::pow((double)a->beta1, t)));
    const float bc2 = (float)(1.0 / (1.0 - std::pow((double)a->beta2, t)));
    LCHK(launch_adam(st, ns.total, T.w, T.wbf, T.g, T.m, T.v, a->lr, a->beta1, a->beta2, a->eps, bc1, bc2));
  }
  net_download(ns, T.w, params, st);
  if (loss_out && a->steps > 0)
    HIPCHK(hipMemcpyAsync(loss_out, T.dl, (size_t)a->steps * sizeof(double), hipMemcpyDeviceToHost, st));
  HIPCHK(hipStreamSynchronize(st));
  if (loss_out)
    for (int s = 0; s < a->steps; ++s) loss_out[s] *= inv_count;
}

}  // namespace

// ===========================================================================
extern "C" {

const char* ldgs_status_str(ldgs_status s) {
  switch (s) {
    case LDGS_OK: return "ok";
    case LDGS_E_ARG: return "invalid argument";
    case LDGS_E_UNSUPPORTED: return "unsupported";
    case LDGS_E_NOMEM: return "out of memory";
    case LDGS_E_HIP: return "HIP error";
    case LDGS_E_SINGULAR_BLOCK: return "singular block";
    case LDGS_E_COLORING: return "improper colouring";
    case LDGS_E_NOT_CONVERGED: return "not converged";
    case LDGS_E_NONFINITE: return "non-finite value";
  }
  return "unknown status";
}

static thread_local std::string g_setup_error;

const char* ldgs_last_error(const ldgs_ctx* ctx) { return ctx ? ctx->err.c_str() : g_setup_error.c_str(); }

ldgs_status ldgs_setup(const ldgs_problem* prob, ldgs_ctx** out) {
  if (!prob || !out) return LDGS_E_ARG;
  *out = nullptr;
  std::unique_ptr<ldgs_ctx> c(new ldgs_ctx());
  try {
    c->P = *prob;
    fill_defaults(c->P);
    validate(c->P);
    const ldgs_problem& P = c->P;
    c->host_only = P.host_only != 0;
    c->g.set(P.dim, P.degree);
    c->B.init(P.degree);
    c->tab = c->B.tab();
    c->vprec = P.vprec;
    if (const char* sg = std::getenv("LDGS_SMALL_GRID")) {
      const long v = std::strtol(sg, nullptr, 10);
      if (v >= 1) c->small_grid = (int)v;
    }
    if (const char* si = std::getenv("LDGS_SHARED_INVERSE")) c->shared_inverse = std::strtol(si, nullptr, 10) != 0;
    if (const char* fs = std::getenv("LDGS_LEARNED_FULL_STEP")) c->learned_full_step = std::strtol(fs, nullptr, 10) != 0;
    if (const char* gr = std::getenv("LDGS_GRAPH")) c->use_graph = std::strtol(gr, nullptr, 10) != 0;
    if (const char* ds = std::getenv("LDGS_DEVICE_SETUP")) c->device_setup = std::strtol(ds, nullptr, 10) != 0;
    if (const char* sp = std::getenv("LDGS_SPLIT_PASS")) c->split_pass = std::strtol(sp, nullptr, 10) != 0;
    if (c->split_pass < 0) c->split_pass = P.dim == 3 ? 1 : 0;
    if (const char* ov = std::getenv("LDGS_OVERLAP")) {
      const long v = std::strtol(ov, nullptr, 10);
      if (v >= 1 && v <= 64) c->overlap_chunks = (int)v;
    }
    if (const char* oc = std::getenv("LDGS_OVERLAP_CHAIN")) c->ov_chain = std::strtol(oc, nullptr, 10) != 0;
    if (const char* om = std::getenv("LDGS_OVERLAP_MIN")) {
      const long v = std::strtol(om, nullptr, 10);
      if (v >= 1) c->overlap_min = v;
    }
    if (const char* mm = std::getenv("LDGS_MFMA_MIN")) {
      const long v = std::strtol(mm, nullptr, 10);
      if (v >= 1) c->mfma_min = v;
    }
    if (const char* fs = std::getenv("LDGS_FUSE_SHARED_MAX")) c->fuse_shared_max = std::strtol(fs, nullptr, 10);
    if (const char* mf = std::getenv("LDGS_MFMA"))
      if (std::strtol(mf, nullptr, 10) == 0) c->mfma_min = 0;
    // LDGS_SETUP_TIMING=1: wall time of each setup phase on stderr
    const bool timing = std::getenv("LDGS_SETUP_TIMING") && std::strtol(std::getenv("LDGS_SETUP_TIMING"), nullptr, 10);
    auto tmark = std::chrono::steady_clock::now();
    auto phase = [&](const char* what) {
      if (!timing) return;
      const auto now = std::chrono::steady_clock::now();
      std::fprintf(stderr, "[ldgs setup] %-28s %8.3f s\n", what, std::chrono::duration<double>(now - tmark).count());
      tmark = now;
    };
    if (P.levelset_kind == LDGS_LEVELSET_CIRCLE || P.levelset_kind == LDGS_LEVELSET_DISK) {
      // implicitly defined mesh: explicit element blocks on every level
      c->k0 = 1;
      c->imp.reset(new ImpHier());
      try {
        imp_build(P, *c->imp);
      } catch (const std::runtime_error& ex) {
        const std::string m = ex.what();
        const ldgs_status st = m.find("colouring") != std::string::npos  ? LDGS_E_COLORING
                               : m.find("singular") != std::string::npos ? LDGS_E_SINGULAR_BLOCK
                                                                         : LDGS_E_ARG;
        throw Fail{st, m};
      }
      phase("implicit hierarchy");
      c->Nc = c->imp->Nc;
      c->h_pinv = c->imp->pinv;
      c->h_eig = c->imp->eig;
      if (!c->host_only) {
        if (P.hip_stream) {
          c->stream = (hipStream_t)P.hip_stream;
        } else {
          HIPCHK(hipStreamCreate(&c->stream));
          c->stream_owned = true;
          HIPCHK(hipEventCreateWithFlags(&c->join_in, hipEventDisableTiming));
          HIPCHK(hipEventCreateWithFlags(&c->join_out, hipEventDisableTiming));
        }
        imp_device(c.get());
        phase("implicit upload");
      }
      g_setup_error.clear();
      *out = c.release();
      return LDGS_OK;
    }
    c->k0 = kernel_dim(P);
    if (stress_walls(P)) {
      // constant velocity components; the rotations are projected separately
      if (c->k0 > 0)
        for (int i = 0; i < P.dim; ++i) c->kernel_offsets.push_back(i * c->g.nq);
      c->rotations = c->k0 > P.dim;
    } else if (c->k0 == 1) {
      c->kernel_offsets = {P.dim * c->g.nq};
    } else {
      for (int i = 0; i <= P.dim; ++i) c->kernel_offsets.push_back(i * c->g.nq);
    }
    // hierarchy
    c->levels.emplace_back();
    build_fine_level(P, c->g, c->B, c->levels[0]);
    phase("fine level");
    while (c->levels.back().n > P.coarsest_n) {
      Level C;
      coarsen_level(P, c->g, c->B, c->levels.back(), C);
      c->levels.push_back(std::move(C));
    }
    phase("coarse levels");
    if (P.diag_scaling)
      for (Level& L : c->levels) set_scaling(L, c->g);
    build_smoother_host(c.get());
    phase("colouring");
    if (c->shared_inverse)
      for (size_t l = 0; l + 1 < c->levels.size(); ++l) c->levels[l].uniform = uniform_blocks(c.get(), c->levels[l]);
    build_bottom(c.get());
    phase("bottom solver");
    if (!c->host_only) {
      if (P.hip_stream) {
        c->stream = (hipStream_t)P.hip_stream;
      } else {
        HIPCHK(hipStreamCreate(&c->stream));
        c->stream_owned = true;
        HIPCHK(hipEventCreateWithFlags(&c->join_in, hipEventDisableTiming));
        HIPCHK(hipEventCreateWithFlags(&c->join_out, hipEventDisableTiming));
      }
      if (c->split_pass && c->overlap_chunks > 1) {
        HIPCHK(hipStreamCreateWithFlags(&c->side, hipStreamNonBlocking));
        HIPCHK(hipEventCreateWithFlags(&c->ov_fork, hipEventDisableTiming));
        HIPCHK(hipEventCreateWithFlags(&c->ov_join, hipEventDisableTiming));
        c->ov_prod.resize(c->overlap_chunks);
        for (auto& e : c->ov_prod) HIPCHK(hipEventCreateWithFlags(&e, hipEventDisableTiming));
      }
      int mask = (1 << P.vprec) | P.build_precisions;
      bool n64 = mask & 1, n32 = mask & 2, n16 = mask & 4;
      // the finest FP64 operator always (outer residual); every level's when
      // the block inverses are built on the device (from the FP64 operator)
      upload_ops<double>(c.get(), c->s64, n64 || c->device_setup);
      if (n32 || n16) {
        upload_ops<float>(c.get(), c->s32, true);
        c->s16.lv = c->s32.lv;                       // same operator data and work vectors
        for (auto& l : c->s16.lv) l.inv = nullptr;
        c->s16.ops = true;
      }
      phase("operator upload");
      build_inverses(c.get(), n64, n32, n16);
      phase("block inverses");
      {
        // scratch of the split residual + restriction: the largest level that
        // uses it (coarse grid below small_grid elements; every level in 3D)
        int64_t rf = 0;
        for (size_t l = 0; l + 1 < c->levels.size(); ++l)
          if (c->levels[l + 1].NE < c->small_grid || c->g.d == 3) rf = std::max(rf, c->levels[l].NE * c->g.nb);
        if (rf > 0) {
          c->w_rf64 = dalloc<double>(c.get(), rf);
          if (n32 || n16) c->w_rf32 = dalloc<float>(c.get(), rf);
        }
      }
      c->s64.built = n64;
      c->s32.built = n32;
      c->s16.built = n16;
      c->d_pinv = upload<double>(c.get(), c->h_pinv);
      c->d_Ac = upload<double>(c.get(), c->h_Ac);
      c->d_bt0 = dalloc<double>(c.get(), c->Nc);
      c->d_bt1 = dalloc<double>(c.get(), c->Nc);
      c->d_bt2 = dalloc<double>(c.get(), c->Nc);
      const int64_t N = c->ndof();
      c->w_b = dalloc<double>(c.get(), N);
      c->w_x = dalloc<double>(c.get(), N);
      c->w_r = dalloc<double>(c.get(), N);
      c->w_z = dalloc<double>(c.get(), N);
      c->w_part = dalloc<double>(c.get(), 1024);
      if (n32 || n16) {
        c->w_b32 = dalloc<float>(c.get(), N);
        c->w_x32 = dalloc<float>(c.get(), N);
      }
      if (P.diag_scaling) c->d_dscale0 = upload<double>(c.get(), c->levels[0].dscale);
      HIPCHK(hipDeviceSynchronize());
      phase("work vectors");
    }
  } catch (const Fail& f) {
    g_setup_error = f.msg;
    return f.st;
  } catch (const std::bad_alloc&) {
    g_setup_error = "host allocation failed";
    return LDGS_E_NOMEM;
  } catch (const std::exception& ex) {
    g_setup_error = ex.what();
    return LDGS_E_ARG;
  }
  g_setup_error.clear();
  *out = c.release();
  return LDGS_OK;
}

ldgs_status ldgs_destroy(ldgs_ctx* ctx) {
  delete ctx;
  return LDGS_OK;
}

ldgs_status ldgs_num_dofs(const ldgs_ctx* ctx, int64_t* ndof) {
  if (!ctx || !ndof) return LDGS_E_ARG;
  *ndof = ctx->ndof();
  return LDGS_OK;
}

ldgs_status ldgs_level_info(const ldgs_ctx* ctx, int level, int* n_l, int* n_levels, int* n_colours) {
  if (ctx && ctx->imp) {
    if (level < 0 || level >= (int)ctx->imp->lv.size()) return LDGS_E_ARG;
    if (n_l) *n_l = ctx->imp->lv[level].n;
    if (n_levels) *n_levels = (int)ctx->imp->lv.size();
    if (n_colours) *n_colours = ctx->imp->lv[level].ncol;
    return LDGS_OK;
  }
  if (!ctx || level < 0 || level >= (int)ctx->levels.size()) return LDGS_E_ARG;
  if (n_l) *n_l = ctx->levels[level].n;
  if (n_levels) *n_levels = (int)ctx->levels.size();
  if (n_colours) *n_colours = ctx->levels[level].ncol;
  return LDGS_OK;
}

ldgs_status ldgs_level_shared_inverse(const ldgs_ctx* ctx, int level, int* shared) {
  if (ctx && ctx->imp && shared) {
    if (level < 0 || level >= (int)ctx->imp->lv.size()) return LDGS_E_ARG;
    *shared = 0;
    return LDGS_OK;
  }
  if (!ctx || !shared || level < 0 || level >= (int)ctx->levels.size()) return LDGS_E_ARG;
  *shared = ctx->levels[level].uniform ? 1 : 0;
  return LDGS_OK;
}

ldgs_status ldgs_assemble_rhs(ldgs_ctx* ctx, const ldgs_rhs_data* data, double* b) {
  try {
    check_ctx(ctx, false);
    if (!data || !b) throw Fail{LDGS_E_ARG, "null argument"};
    std::vector<double> hb(ctx->ndof());
    if (ctx->imp) imp_rhs(ctx->P, *ctx->imp, *data, hb.data());
    else assemble_rhs_host(ctx->P, ctx->g, ctx->B, ctx->levels[0], *data, hb.data());
    if (ctx->host_only) std::memcpy(b, hb.data(), hb.size() * sizeof(double));
    else HIPCHK(hipMemcpy(b, hb.data(), hb.size() * sizeof(double), hipMemcpyHostToDevice));
    return LDGS_OK;
  } catch (const Fail& f) {
    return handle(ctx, f);
  }
}

ldgs_status ldgs_apply(ldgs_ctx* ctx, const double* x, double* y) {
  try {
    check_ctx(ctx, true);
    Join join_(ctx);
    if (!x || !y || x == y) throw Fail{LDGS_E_ARG, "x, y must be distinct non-null"};
    apply_fine(ctx, x, y);
    return LDGS_OK;
  } catch (const Fail& f) {
    return handle(ctx, f);
  }
}

ldgs_status ldgs_residual(ldgs_ctx* ctx, const double* b, const double* x, double* r, double* norm2) {
  try {
    check_ctx(ctx, true);
    Join join_(ctx);
    if (!b || !x) throw Fail{LDGS_E_ARG, "null argument"};
    double* rr = r ? r : ctx->w_r;
    residual_fine(ctx, b, x, rr);
    if (norm2) *norm2 = std::sqrt(dot(ctx, rr, rr));
    return LDGS_OK;
  } catch (const Fail& f) {
    return handle(ctx, f);
  }
}

ldgs_status ldgs_vcycle(ldgs_ctx* ctx, const double* b, double* x) {
  try {
    check_ctx(ctx, true);
    Join join_(ctx);
    if (!b || !x) throw Fail{LDGS_E_ARG, "null argument"};
    vcycle_user(ctx, ctx->vprec, b, x, false);
    return LDGS_OK;
  } catch (const Fail& f) {
    return handle(ctx, f);
  }
}

ldgs_status ldgs_graph_count(const ldgs_ctx* ctx, int* n_graphs) {
  if (!ctx || !n_graphs) return LDGS_E_ARG;
  *n_graphs = ctx->use_graph ? (int)ctx->graphs.size() : 0;
  return LDGS_OK;
}

ldgs_status ldgs_set_vprec(ldgs_ctx* ctx, int vprec) {
  if (!ctx || vprec < 0 || vprec > 2) return LDGS_E_ARG;
  bool ok = (vprec == 0 && ctx->s64.built) || (vprec == 1 && ctx->s32.built) || (vprec == 2 && ctx->s16.built);
  if (!ok) {
    ctx->err = "precision not built at setup";
    return LDGS_E_UNSUPPORTED;
  }
  ctx->vprec = vprec;
  return LDGS_OK;
}

ldgs_status ldgs_set_learned(ldgs_ctx* ctx, const ldgs_net* net) {
  try {
    check_ctx(ctx, true);
    if (ctx->imp) throw Fail{LDGS_E_UNSUPPORTED, "no learned correction on implicitly defined meshes"};
    Join join_(ctx);
    if (!net) {
      ctx->net_loaded = false;
      return LDGS_OK;
    }
    if (net->dim != ctx->P.dim || net->degree != ctx->P.degree) throw Fail{LDGS_E_ARG, "network dim/degree mismatch"};
    if (net->hidden != NET_H) throw Fail{LDGS_E_UNSUPPORTED, "network hidden width must be 16"};
    const NetShape ns = net_shape(ctx->P.dim, ctx->P.degree);
    if (!net->params || net->nparams != ns.flat_total)
      throw Fail{LDGS_E_ARG, "network parameter count: expected " + std::to_string(ns.flat_total)};
    if (!(net->c_vel > 0) || !(net->c_pre > 0)) throw Fail{LDGS_E_ARG, "output scales must be positive"};
    for (int64_t i = 0; i < ns.flat_total; ++i)
      if (!std::isfinite(net->params[i])) throw Fail{LDGS_E_NONFINITE, "network parameters"};
    learned_buffers(ctx);
    if (!ctx->d_net) {
      ctx->d_net = dalloc<float>(ctx, ns.total);
      ctx->d_netbf = dalloc<uint16_t>(ctx, ns.total);
    }
    std::vector<float> pad;
    net_pack(ns, net->params, pad);
    HIPCHK(hipMemcpy(ctx->d_net, pad.data(), pad.size() * sizeof(float), hipMemcpyHostToDevice));
    LCHK(launch_to_bf16(ctx->stream, ns.total, ctx->d_net, ctx->d_netbf));
    HIPCHK(hipStreamSynchronize(ctx->stream));
    ctx->ns = ns;
    ctx->c_net[0] = net->c_vel;
    ctx->c_net[1] = net->c_pre;
    ctx->net_loaded = true;
    return LDGS_OK;
  } catch (const Fail& f) {
    return handle(ctx, f);
  }
}

ldgs_status ldgs_learned_correction(ldgs_ctx* ctx, const double* r, double* dx) {
  try {
    check_ctx(ctx, true);
    if (ctx->imp) throw Fail{LDGS_E_UNSUPPORTED, "no learned correction on implicitly defined meshes"};
    Join join_(ctx);
    if (!r || !dx) throw Fail{LDGS_E_ARG, "null argument"};
    if (!ctx->net_loaded) throw Fail{LDGS_E_ARG, "no network loaded"};
    const Level& L = ctx->levels[0];
    const int nb = ctx->g.nb, nvel = ctx->g.d * ctx->g.nq;
    LCHK(launch_field_sumsq<double>(ctx->stream, L.NE, nb, nvel, r, nullptr, ctx->w_part, SUMSQ_BLK, ctx->d_sums));
    LCHK(launch_net_apply<double>(ctx->stream, ctx->g.d, ctx->g.p, L.n, log2i(L.n), periodic_mask(ctx->P), r, nullptr,
                                  ctx->d_logmu, ctx->d_sums, (double)L.NE * nvel, (double)L.NE * (nb - nvel),
                                  ctx->c_net[0], ctx->c_net[1], net_dev(ctx), nullptr, dx));
    return LDGS_OK;
  } catch (const Fail& f) {
    return handle(ctx, f);
  }
}

ldgs_status ldgs_learned_collect(ldgs_ctx* ctx, const double* xstar, int ncycles, int crop, int ncrops,
                                 const int* origins, uint16_t* feat, uint16_t* targ, double* stats) {
  try {
    check_ctx(ctx, true);
    if (ctx->imp) throw Fail{LDGS_E_UNSUPPORTED, "no learned correction on implicitly defined meshes"};
    Join join_(ctx);
    const Level& L = ctx->levels[0];
    const int d = ctx->g.d;
    if (!xstar || !origins || !feat || !targ || ncycles < 1 || ncrops < 1) throw Fail{LDGS_E_ARG, "bad argument"};
    if (!pow2(crop) || crop < 4 || crop > L.n) throw Fail{LDGS_E_ARG, "crop must be a power of two in [4, n]"};
    const int64_t norig = (int64_t)ncycles * ncrops * d;
    for (int64_t i = 0; i < norig; ++i) {
      const int k = (int)(i % d);
      const int o = origins[i];
      const bool per = ctx->P.bc[k] == LDGS_PERIODIC;
      if (o < 0 || o >= L.n || (!per && o + crop > L.n)) throw Fail{LDGS_E_ARG, "crop origin out of range"};
    }
    learned_buffers(ctx);
    const NetShape ns = net_shape(d, ctx->P.degree);
    const int64_t N = ctx->ndof();
    const int nb = ctx->g.nb, nvel = d * ctx->g.nq;
    if (!ctx->w_cb) {
      ctx->w_cb = dalloc<double>(ctx, N);
      ctx->w_cx = dalloc<double>(ctx, N);
      ctx->w_ce = dalloc<double>(ctx, N);
    }
    if (ctx->d_orig_cap < norig) {
      ctx->d_orig = dalloc<int>(ctx, norig);
      ctx->d_orig_cap = norig;
    }
    HIPCHK(hipMemcpy(ctx->d_orig, origins, norig * sizeof(int), hipMemcpyHostToDevice));
    int64_t Md = 1, Cd = 1;
    for (int k = 0; k < d; ++k) {
      Md *= crop + 2;
      Cd *= crop;
    }
    LaunchCfg cfg{d, ctx->g.p, ctx->stream, ctx->small_grid};
    LCHK(launch_residual<double>(cfg, ctx->s64.lv[0].unscaled, ctx->tab, nullptr, xstar, ctx->w_cb, 1));
    LCHK(launch_fill<double>(ctx->stream, N, 0.0, ctx->w_cx));
    const double cu = (double)L.NE * nvel, cp = (double)L.NE * (nb - nvel);
    for (int k = 0; k < ncycles; ++k) {
      vcycle_user(ctx, ctx->vprec, ctx->w_cb, ctx->w_cx, false);
      residual_fine(ctx, ctx->w_cb, ctx->w_cx, ctx->w_r);
      LCHK(launch_scale_copy(ctx->stream, N, 1.0, xstar, ctx->w_ce));
      LCHK(launch_axpy(ctx->stream, N, -1.0, ctx->w_cx, ctx->w_ce));
      project_kernel(ctx, ctx->w_ce);
      LCHK(launch_field_sumsq<double>(ctx->stream, L.NE, nb, nvel, ctx->w_r, nullptr, ctx->w_part, SUMSQ_BLK,
                                      ctx->d_sums));
      LCHK(launch_collect_crops(ctx->stream, d, ctx->g.p, L.n, log2i(L.n), periodic_mask(ctx->P), crop, log2i(crop),
                                ncrops, ctx->d_orig + (int64_t)k * ncrops * d, ctx->w_r, ctx->w_ce, ctx->d_logmu,
                                ctx->d_sums, cu, cp, feat + (int64_t)k * ncrops * Md * ns.chp,
                                targ + (int64_t)k * ncrops * Cd * nb));
      if (stats) {
        double sr[2], se[2];
        HIPCHK(hipMemcpyAsync(sr, ctx->d_sums, 2 * sizeof(double), hipMemcpyDeviceToHost, ctx->stream));
        HIPCHK(hipStreamSynchronize(ctx->stream));
        LCHK(launch_field_sumsq<double>(ctx->stream, L.NE, nb, nvel, ctx->w_ce, nullptr, ctx->w_part, SUMSQ_BLK,
                                        ctx->d_sums));
        HIPCHK(hipMemcpyAsync(se, ctx->d_sums, 2 * sizeof(double), hipMemcpyDeviceToHost, ctx->stream));
        HIPCHK(hipStreamSynchronize(ctx->stream));
        const double su = sr[0] > 0 ? std::sqrt(sr[0] / cu) : 1.0, sp = sr[1] > 0 ? std::sqrt(sr[1] / cp) : 1.0;
        stats[4 * k + 0] = su;
        stats[4 * k + 1] = sp;
        stats[4 * k + 2] = std::sqrt(se[0] / cu) / su;
        stats[4 * k + 3] = std::sqrt(se[1] / cp) / sp;
      }
    }
    HIPCHK(hipStreamSynchronize(ctx->stream));
    return LDGS_OK;
  } catch (const Fail& f) {
    return handle(ctx, f);
  }
}

ldgs_status ldgs_learned_train(const ldgs_train_args* a, float* params, double* loss_out, float* grad0_out) {
  try {
    const NetShape ns = check_train_args(a, params);
    const int nsteps = a->steps > 0 ? a->steps : 1;
    DevBufs B;
    TrainBufs T{};
    T.w = B.get<float>(ns.total);
    T.wbf = B.get<uint16_t>(ns.total);
    T.g = B.get<float>(ns.total);
    T.m = B.get<float>(ns.total);
    T.v = B.get<float>(ns.total);
    T.dl = B.get<double>(nsteps);
    T.ord = B.get<int>((size_t)nsteps * a->batch);
    train_run(a, ns, T, params, loss_out, grad0_out);
    return LDGS_OK;
  } catch (const Fail& f) {
    g_setup_error = f.msg;
    return f.st;
  }
}

ldgs_status ldgs_learned_train_noalloc(const ldgs_train_args* a, float* params, double* loss_out, float* grad0_out) {
  try {
    const NetShape ns = check_train_args(a, params);
    const int64_t nsteps = a->steps > 0 ? a->steps : 1;
    // the run's buffers, each at a 256-byte boundary of the workspace
    size_t off = 0;
    auto take = [&](size_t bytes) {
      const size_t o = off;
      off += (bytes + 255) & ~(size_t)255;
      return o;
    };
    const size_t ow = take(ns.total * sizeof(float)), obf = take(ns.total * sizeof(uint16_t));
    const size_t og = take(ns.total * sizeof(float)), om = take(ns.total * sizeof(float));
    const size_t ov = take(ns.total * sizeof(float)), odl = take(nsteps * sizeof(double));
    const size_t oord = take((size_t)nsteps * a->batch * sizeof(int));
    if (off > LDGS_TRAIN_WORKSPACE_BYTES)
      throw Fail{LDGS_E_ARG, "the run needs " + std::to_string(off) + " bytes of workspace, more than the " +
                                 std::to_string(LDGS_TRAIN_WORKSPACE_BYTES) + " available (fewer steps x batch)"};
    void* base = nullptr;
    if (train_workspace(&base) != 0) throw Fail{LDGS_E_HIP, "address of the training workspace not available"};
    char* b = (char*)base;
    const TrainBufs T{(float*)(b + ow), (uint16_t*)(b + obf), (float*)(b + og), (float*)(b + om),
                      (float*)(b + ov), (double*)(b + odl), (int*)(b + oord)};
    train_run(a, ns, T, params, loss_out, grad0_out);
    return LDGS_OK;
  } catch (const Fail& f) {
    g_setup_error = f.msg;
    return f.st;
  }
}

ldgs_status ldgs_project_kernel(ldgs_ctx* ctx, double* v) {
  try {
    check_ctx(ctx, true);
    Join join_(ctx);
    if (!v) throw Fail{LDGS_E_ARG, "null argument"};
    project_kernel(ctx, v);
    return LDGS_OK;
  } catch (const Fail& f) {
    return handle(ctx, f);
  }
}

ldgs_status ldgs_solve(ldgs_ctx* ctx, double* b, double* x, double tol, int maxit, int outer, int fgmres_m,
                       int use_learned, ldgs_info* info) {
  try {
    check_ctx(ctx, true);
    Join join_(ctx);
    if (!b || !x || maxit < 0 || !(tol >= 0)) throw Fail{LDGS_E_ARG, "bad argument"};
    if (use_learned) {
      if (outer != LDGS_IR && outer != LDGS_FGMRES)
        throw Fail{LDGS_E_UNSUPPORTED, "the learned correction is used with outer = IR or FGMRES"};
      if (!ctx->net_loaded) throw Fail{LDGS_E_ARG, "no network loaded"};
    }
    auto t0 = std::chrono::steady_clock::now();
    const int64_t N = ctx->ndof();
    project_kernel(ctx, b);
    const double bn = std::sqrt(dot(ctx, b, b));
    int it = 0;
    double rel = 0.0;
    std::vector<double> hist;
    ldgs_status st = LDGS_OK;
    int events = 0;
    auto relres = [&]() {
      residual_fine(ctx, b, x, ctx->w_r);
      double v = std::sqrt(dot(ctx, ctx->w_r, ctx->w_r));
      return bn > 0 ? v / bn : v;
    };
    if (bn == 0.0) {
      LCHK(launch_fill<double>(ctx->stream, N, 0.0, x));
      rel = 0.0;
      hist.push_back(0.0);
    } else if (outer == LDGS_STATIONARY || outer == LDGS_IR) {
      rel = relres();
      hist.push_back(rel);
      bool learn_on = use_learned != 0;
      double rho_plain = 0.0;
      int strikes = 0;
      while (rel > tol && it < maxit) {
        double rn;
        if (outer == LDGS_STATIONARY) {
          vcycle_user(ctx, ctx->vprec, b, x, false);
          rn = relres();
        } else if (!(learn_on && it >= 2)) {
          // r = b - A x is in w_r from relres()
          precond_add(ctx, ctx->vprec, ctx->w_r, x);
          rn = relres();
        } else {
          // z = V(r); x_old + (z + dx), dx from r - A z; guarded below
          vcycle_user(ctx, ctx->vprec, ctx->w_r, ctx->w_z, true);
          learned_minres(ctx, ctx->vprec, ctx->w_z, ctx->w_zl);
          HIPCHK(hipMemcpyAsync(ctx->w_xold, x, N * sizeof(double), hipMemcpyDeviceToDevice, ctx->stream));
          LCHK(launch_axpy(ctx->stream, N, 1.0, ctx->w_zl, x));
          rn = relres();
          const double ck = rn / hist.back();
          strikes = (ck > 1.1 * rho_plain) ? strikes + 1 : 0;
          if (ck > 1.0 || strikes >= 2) {
            learn_on = false;
            ++events;
            HIPCHK(hipMemcpyAsync(x, ctx->w_xold, N * sizeof(double), hipMemcpyDeviceToDevice, ctx->stream));
            LCHK(launch_axpy(ctx->stream, N, 1.0, ctx->w_z, x));
            rn = relres();
          }
        }
        ++it;
        rel = rn;
        hist.push_back(rel);
        if (use_learned && it == 2) rho_plain = std::sqrt(hist[2] / hist[0]);
        if (!std::isfinite(rel)) { st = LDGS_E_NONFINITE; break; }
        if (rel > 1e10 * hist[0]) { st = LDGS_E_NOT_CONVERGED; break; }   // blow-up (a first cycle may raise the residual transiently)
      }
    } else if (outer == LDGS_FGMRES || outer == LDGS_GMRES) {
      const bool flex = outer == LDGS_FGMRES;
      const int m = fgmres_m > 0 ? fgmres_m : 30;
      const int nvec = flex ? 2 * m + 1 : m + 2;
      while ((int)ctx->kry.size() < nvec) ctx->kry.push_back(dalloc<double>(ctx, N));
      double* const* V = ctx->kry.data();
      // flexible: Z[j] = M v_j kept; fixed M: one temporary, M applied to V y at the end
      double* const* Z = ctx->kry.data() + (m + 1);
      double* T = ctx->kry[m + 1];
      rel = relres();
      hist.push_back(rel);
      while (rel > tol && it < maxit) {
        double beta = rel * bn;
        LCHK(launch_scale_copy(ctx->stream, N, 1.0 / beta, ctx->w_r, V[0]));
        std::vector<double> H((m + 1) * m, 0.0), cs(m), sn(m), gvec(m + 1, 0.0);
        gvec[0] = beta;
        int jdone = 0;
        for (int j = 0; j < m && it < maxit; ++j) {
          double* zj = flex ? Z[j] : T;
          vcycle_user(ctx, ctx->vprec, V[j], zj, true);
          if (use_learned) learned_minres(ctx, ctx->vprec, zj, zj);   // a variable preconditioner: FGMRES only
          apply_fine(ctx, zj, V[j + 1]);
          std::vector<double> hcol(j + 1);
          double hn = mgs(ctx, V, j, V[j + 1], hcol.data());
          for (int i = 0; i <= j; ++i) H[i * m + j] = hcol[i];
          H[(j + 1) * m + j] = hn;
          if (hn > 0) LCHK(launch_scale_copy(ctx->stream, N, 1.0 / hn, V[j + 1], V[j + 1]));
          for (int i = 0; i < j; ++i) {
            double t = cs[i] * H[i * m + j] + sn[i] * H[(i + 1) * m + j];
            H[(i + 1) * m + j] = -sn[i] * H[i * m + j] + cs[i] * H[(i + 1) * m + j];
            H[i * m + j] = t;
          }
          double den = std::hypot(H[j * m + j], H[(j + 1) * m + j]);
          cs[j] = H[j * m + j] / den;
          sn[j] = H[(j + 1) * m + j] / den;
          H[j * m + j] = den;
          H[(j + 1) * m + j] = 0.0;
          gvec[j + 1] = -sn[j] * gvec[j];
          gvec[j] = cs[j] * gvec[j];
          ++it;
          jdone = j + 1;
          double est = std::fabs(gvec[j + 1]) / bn;
          hist.push_back(est);
          if (!std::isfinite(est)) { st = LDGS_E_NONFINITE; break; }
          if (est <= tol) break;
        }
        if (st != LDGS_OK) break;
        std::vector<double> y(jdone);
        for (int i = jdone - 1; i >= 0; --i) {
          double s = gvec[i];
          for (int q = i + 1; q < jdone; ++q) s -= H[i * m + q] * y[q];
          y[i] = s / H[i * m + i];
        }
        if (flex) {
          for (int i = 0; i < jdone; ++i) LCHK(launch_axpy(ctx->stream, N, y[i], Z[i], x));
        } else {
          // x += M (V y): the combination into V[0] (no longer needed), then one cycle
          LCHK(launch_scale_copy(ctx->stream, N, y[0], V[0], V[0]));
          for (int i = 1; i < jdone; ++i) LCHK(launch_axpy(ctx->stream, N, y[i], V[i], V[0]));
          precond_add(ctx, ctx->vprec, V[0], x);
        }
        rel = relres();
        if (!hist.empty()) hist.back() = rel;
        if (!std::isfinite(rel)) { st = LDGS_E_NONFINITE; break; }
      }
    } else {
      throw Fail{LDGS_E_ARG, "outer"};
    }
    HIPCHK(hipStreamSynchronize(ctx->stream));
    double secs = std::chrono::duration<double>(std::chrono::steady_clock::now() - t0).count();
    if (st == LDGS_OK && rel > tol) st = LDGS_E_NOT_CONVERGED;
    if (info) {
      info->iters = it;
      info->fallback_events = events;
      info->relres = rel;
      info->rho_measured = (it > 0 && rel > 0 && hist[0] > 0) ? std::pow(rel / hist[0], 1.0 / it) : 0.0;
      info->t_solve_s = secs;
      info->history_len = 0;
      if (info->history)
        for (size_t i = 0; i < hist.size() && (int)i < info->history_cap; ++i) {
          info->history[i] = hist[i];
          info->history_len = (int)i + 1;
        }
    }
    if (st != LDGS_OK) ctx->err = std::string("solve ended with relres ") + std::to_string(rel);
    return st;
  } catch (const Fail& f) {
    return handle(ctx, f);
  }
}

// Convergence rate of eq. (rho): GMRES, left-preconditioned by one V-cycle
// from zero (the linear operator V), on V A x = V b with b = 0 from x0,
// without restarts: modified Gram-Schmidt Arnoldi on w = V A v in FP64,
// Givens rotations for the residual norms ||V A x_k|| (section 4).
ldgs_status ldgs_gmres_rho(ldgs_ctx* ctx, const double* x0, double reduction, int maxit, double* rho, int* iters,
                           double* history, int history_cap) {
  try {
    check_ctx(ctx, true);
    Join join_(ctx);
    if (!x0 || !rho || maxit < 1 || maxit > 1000 || !(reduction > 0.0 && reduction < 1.0))
      throw Fail{LDGS_E_ARG, "bad argument"};
    const int64_t N = ctx->ndof();
    while ((int)ctx->kry.size() < maxit + 2) ctx->kry.push_back(dalloc<double>(ctx, N));
    double* const* V = ctx->kry.data();
    double* Av = ctx->kry[maxit + 1];            // A v, the V-cycle's input
    auto VA = [&](const double* v, double* out) {
      apply_fine(ctx, v, Av);
      vcycle_user(ctx, ctx->vprec, Av, out, true);
    };
    // r0 = V (b - A x0) = -V A x0
    VA(x0, V[0]);
    const double beta = std::sqrt(dot(ctx, V[0], V[0]));
    if (!(beta > 0.0) || !std::isfinite(beta)) throw Fail{LDGS_E_NONFINITE, "initial preconditioned residual"};
    LCHK(launch_scale_copy(ctx->stream, N, -1.0 / beta, V[0], V[0]));
    const int m = maxit;
    std::vector<double> H((size_t)(m + 1) * m, 0.0), cs(m), sn(m), g(m + 1, 0.0), res(1, 1.0);
    g[0] = beta;
    int n = 0;
    for (int j = 0; j < m; ++j) {
      VA(V[j], V[j + 1]);
      std::vector<double> hcol(j + 1);
      const double hn = mgs(ctx, V, j, V[j + 1], hcol.data());
      for (int i = 0; i <= j; ++i) H[(size_t)i * m + j] = hcol[i];
      H[(size_t)(j + 1) * m + j] = hn;
      if (hn > 0.0) LCHK(launch_scale_copy(ctx->stream, N, 1.0 / hn, V[j + 1], V[j + 1]));
      for (int i = 0; i < j; ++i) {
        const double t = cs[i] * H[(size_t)i * m + j] + sn[i] * H[(size_t)(i + 1) * m + j];
        H[(size_t)(i + 1) * m + j] = -sn[i] * H[(size_t)i * m + j] + cs[i] * H[(size_t)(i + 1) * m + j];
        H[(size_t)i * m + j] = t;
      }
      const double den = std::hypot(H[(size_t)j * m + j], H[(size_t)(j + 1) * m + j]);
      cs[j] = H[(size_t)j * m + j] / den;
      sn[j] = H[(size_t)(j + 1) * m + j] / den;
      g[j + 1] = -sn[j] * g[j];
      g[j] = cs[j] * g[j];
      n = j + 1;
      const double rel = std::fabs(g[j + 1]) / beta;
      res.push_back(rel);
      if (!std::isfinite(rel)) throw Fail{LDGS_E_NONFINITE, "GMRES residual"};
      if (rel <= reduction || hn == 0.0) break;
    }
    *rho = std::exp(std::log(res.back()) / n);
    if (iters) *iters = n;
    if (history)
      for (int k = 0; k < (int)res.size() && k < history_cap; ++k) history[k] = res[k];
    return res.back() <= reduction ? LDGS_OK : LDGS_E_NOT_CONVERGED;
  } catch (const Fail& f) {
    return handle(ctx, f);
  }
}

// ---- profiling -------------------------------------------------------------
ldgs_status ldgs_profile(ldgs_ctx* ctx, int enable) {
  if (!ctx) return LDGS_E_ARG;
  ctx->prof = enable > 0 ? enable : 0;
  ctx->prof_count = 0;
  ctx->prof_ev.clear();
  ctx->ev_used = 0;
  return LDGS_OK;
}

ldgs_status ldgs_profile_read(ldgs_ctx* ctx, double* total_ms, int64_t* launches) {
  try {
    check_ctx(ctx, true);
    Join join_(ctx);
    HIPCHK(hipStreamSynchronize(ctx->stream));
    double tot = 0.0;
    int64_t n = 0;
    for (auto& pr : ctx->prof_ev) {
      float ms = 0.f;
      HIPCHK(hipEventElapsedTime(&ms, pr.e0, pr.e1));
      tot += ms;
      n += pr.passes;
    }
    if (total_ms) *total_ms = tot;
    if (launches) *launches = n;
    ctx->prof_ev.clear();
    ctx->ev_used = 0;
    return LDGS_OK;
  } catch (const Fail& f) {
    return handle(ctx, f);
  }
}

// ---- stage entry points --------------------------------------------------
namespace {
// level and colour checks of the level-stage entry points on implicit meshes
void imp_level_check(ldgs_ctx* ctx, int level, bool smoothed) {
  const int nl = (int)ctx->imp->lv.size();
  if (level < 0 || level >= nl || (smoothed && level + 1 >= nl)) throw Fail{LDGS_E_ARG, "level"};
}
}  // namespace

ldgs_status ldgs_level_elements(const ldgs_ctx* ctx, int level, int64_t* ne) {
  if (!ctx || !ne) return LDGS_E_ARG;
  if (ctx->imp) {
    if (level < 0 || level >= (int)ctx->imp->lv.size()) return LDGS_E_ARG;
    *ne = ctx->imp->lv[level].NE;
  } else {
    if (level < 0 || level >= (int)ctx->levels.size()) return LDGS_E_ARG;
    *ne = ctx->levels[level].NE;
  }
  return LDGS_OK;
}

ldgs_status ldgs_level_blocks(const ldgs_ctx* ctx, int level, int64_t* nblocks) {
  if (!ctx || !nblocks) return LDGS_E_ARG;
  if (!ctx->imp) return LDGS_E_UNSUPPORTED;   // Cartesian levels hold no explicit blocks
  if (level < 0 || level >= (int)ctx->imp->lv.size()) return LDGS_E_ARG;
  *nblocks = ctx->imp->lv[level].rowptr.empty() ? 0 : ctx->imp->lv[level].rowptr.back();
  return LDGS_OK;
}

ldgs_status ldgs_level_smooth_colour(ldgs_ctx* ctx, int level, int colour, const double* b, double* x) {
  try {
    check_ctx(ctx, true);
    Join join_(ctx);
    if (ctx->imp) {
      if (!ctx->imp64) throw Fail{LDGS_E_UNSUPPORTED, "FP64 V-cycle not built"};
      imp_level_check(ctx, level, true);
      if (colour < 0 || colour >= ctx->imp->lv[level].ncol || !b || !x) throw Fail{LDGS_E_ARG, "colour"};
      imp_colour<double>(ctx, level, colour, b, x);
      return LDGS_OK;
    }
    if (!ctx->s64.built) throw Fail{LDGS_E_UNSUPPORTED, "FP64 V-cycle not built"};
    if (level < 0 || level + 1 >= (int)ctx->levels.size()) throw Fail{LDGS_E_ARG, "level"};
    if (colour < 0 || colour >= ctx->levels[level].ncol || !b || !x) throw Fail{LDGS_E_ARG, "colour"};
    smooth_colour<double>(ctx, ctx->s64, level, colour, b, x);
    return LDGS_OK;
  } catch (const Fail& f) {
    return handle(ctx, f);
  }
}

ldgs_status ldgs_level_smooth_colour_f32(ldgs_ctx* ctx, int level, int colour, int vprec, const float* b, float* x) {
  try {
    check_ctx(ctx, true);
    Join join_(ctx);
    if (ctx->imp) {
      if (vprec != LDGS_V_FP32 || !ctx->imp32) throw Fail{LDGS_E_UNSUPPORTED, "requested float V-cycle not built"};
      imp_level_check(ctx, level, true);
      if (colour < 0 || colour >= ctx->imp->lv[level].ncol || !b || !x) throw Fail{LDGS_E_ARG, "colour"};
      imp_colour<float>(ctx, level, colour, b, x);
      return LDGS_OK;
    }
    PrecStore<float>* S = vprec == LDGS_V_FP32 ? &ctx->s32 : (vprec == LDGS_V_FP32_BF16BLK ? &ctx->s16 : nullptr);
    if (!S || !S->built) throw Fail{LDGS_E_UNSUPPORTED, "requested float V-cycle not built"};
    if (level < 0 || level + 1 >= (int)ctx->levels.size()) throw Fail{LDGS_E_ARG, "level"};
    if (colour < 0 || colour >= ctx->levels[level].ncol || !b || !x) throw Fail{LDGS_E_ARG, "colour"};
    smooth_colour<float>(ctx, *S, level, colour, b, x);
    return LDGS_OK;
  } catch (const Fail& f) {
    return handle(ctx, f);
  }
}

ldgs_status ldgs_level_residual_restrict(ldgs_ctx* ctx, int level, const double* b, const double* x, double* rc) {
  try {
    check_ctx(ctx, true);
    Join join_(ctx);
    if (ctx->imp) {
      if (!ctx->imp64) throw Fail{LDGS_E_UNSUPPORTED, "FP64 V-cycle not built"};
      imp_level_check(ctx, level, true);
      if (!b || !x || !rc) throw Fail{LDGS_E_ARG, "null argument"};
      ldgs_ctx::ImpDev& D = ctx->idev[level];
      ldgs_ctx::ImpDev& C = ctx->idev[level + 1];
      const int nb = ctx->imp->nb;
      LCHK(launch_bsr_residual<double>(ctx->stream, nb, D.NE, D.rowptr, D.cols, D.blk64, b, x, D.r64, nullptr));
      LCHK(launch_bsr_restrict<double>(ctx->stream, nb, C.NE, C.kid_ptr, C.kids, D.I64, D.r64, rc));
      return LDGS_OK;
    }
    if (!ctx->s64.built) throw Fail{LDGS_E_UNSUPPORTED, "FP64 V-cycle not built"};
    if (level < 0 || level + 1 >= (int)ctx->levels.size() || !b || !x || !rc) throw Fail{LDGS_E_ARG, "level"};
    LaunchCfg cfg{ctx->g.d, ctx->g.p, ctx->stream, ctx->small_grid};
    LCHK(launch_residual_restrict<double>(cfg, ctx->s64.lv[level].view, ctx->tab, b, x, rc, ctx->w_rf64));
    return LDGS_OK;
  } catch (const Fail& f) {
    return handle(ctx, f);
  }
}

ldgs_status ldgs_level_prolong_add(ldgs_ctx* ctx, int level, const double* xc, double* x) {
  try {
    check_ctx(ctx, true);
    Join join_(ctx);
    if (ctx->imp) {
      if (!ctx->imp64) throw Fail{LDGS_E_UNSUPPORTED, "FP64 V-cycle not built"};
      imp_level_check(ctx, level, true);
      if (!xc || !x) throw Fail{LDGS_E_ARG, "null argument"};
      ldgs_ctx::ImpDev& D = ctx->idev[level];
      LCHK(launch_bsr_prolong<double>(ctx->stream, ctx->imp->nb, D.NE, D.parent, D.I64, xc, x));
      return LDGS_OK;
    }
    if (level < 0 || level + 1 >= (int)ctx->levels.size() || !xc || !x) throw Fail{LDGS_E_ARG, "level"};
    LaunchCfg cfg{ctx->g.d, ctx->g.p, ctx->stream, ctx->small_grid};
    LCHK(launch_prolong_add<double>(cfg, ctx->levels[level].n, ctx->tab, xc, x));
    return LDGS_OK;
  } catch (const Fail& f) {
    return handle(ctx, f);
  }
}

ldgs_status ldgs_bottom_solve(ldgs_ctx* ctx, const double* b, double* x) {
  try {
    check_ctx(ctx, true);
    Join join_(ctx);
    if (!b || !x || b == x) throw Fail{LDGS_E_ARG, "b, x must be distinct non-null"};
    bottom_solve<double>(ctx, b, x);
    return LDGS_OK;
  } catch (const Fail& f) {
    return handle(ctx, f);
  }
}

ldgs_status ldgs_level_apply(ldgs_ctx* ctx, int level, const double* x, double* y) {
  try {
    check_ctx(ctx, true);
    Join join_(ctx);
    if (ctx->imp) {
      imp_level_check(ctx, level, false);
      ldgs_ctx::ImpDev& D = ctx->idev[level];
      if (!D.blk64) throw Fail{LDGS_E_UNSUPPORTED, "FP64 operator of the level not built"};
      if (!x || !y) throw Fail{LDGS_E_ARG, "null argument"};
      LCHK(launch_bsr_residual<double>(ctx->stream, ctx->imp->nb, D.NE, D.rowptr, D.cols, D.blk64, nullptr, x, y,
                                       nullptr));
      return LDGS_OK;
    }
    if (!ctx->s64.built && level != 0) throw Fail{LDGS_E_UNSUPPORTED, "FP64 V-cycle not built"};
    if (level < 0 || level >= (int)ctx->levels.size() || !x || !y) throw Fail{LDGS_E_ARG, "level"};
    if (level == (int)ctx->levels.size() - 1 && ctx->levels[level].n < 4)
      throw Fail{LDGS_E_UNSUPPORTED, "device apply needs n >= 4 on the level"};
    LaunchCfg cfg{ctx->g.d, ctx->g.p, ctx->stream, ctx->small_grid};
    LCHK(launch_residual<double>(cfg, ctx->s64.lv[level].view, ctx->tab, nullptr, x, y, 1));
    return LDGS_OK;
  } catch (const Fail& f) {
    return handle(ctx, f);
  }
}

ldgs_status ldgs_level_block_inverse(ldgs_ctx* ctx, int level, int64_t element, double* inv_host) {
  try {
    check_ctx(ctx, false);
    if (ctx->imp) {
      imp_level_check(ctx, level, true);
      const ImpLevel& L = ctx->imp->lv[level];
      if (element < 0 || element >= L.NE || !inv_host) throw Fail{LDGS_E_ARG, "element"};
      const int nb = ctx->imp->nb;
      const double* I = L.inv.data() + (size_t)element * nb * nb;   // column-major
      for (int r = 0; r < nb; ++r)
        for (int c = 0; c < nb; ++c) inv_host[r * nb + c] = I[(size_t)c * nb + r];
      return LDGS_OK;
    }
    if (level < 0 || level + 1 >= (int)ctx->levels.size() || !inv_host) throw Fail{LDGS_E_ARG, "level"};
    const Level& L = ctx->levels[level];
    if (element < 0 || element >= L.NE) throw Fail{LDGS_E_ARG, "element"};
    const int nb = ctx->g.nb;
    std::vector<double> A((size_t)nb * nb);
    host_diag_block(L, ctx->g, ctx->B, ctx->P.form, element, A.data());
    if (!block_inverse(nb, A.data(), inv_host, 1e-14)) throw Fail{LDGS_E_SINGULAR_BLOCK, "singular block"};
    return LDGS_OK;
  } catch (const Fail& f) {
    return handle(ctx, f);
  }
}

ldgs_status ldgs_host_level_apply(ldgs_ctx* ctx, int level, const double* x, double* y) {
  try {
    check_ctx(ctx, false);
    if (ctx->imp) {
      // y = A_l x from the level's host element blocks
      imp_level_check(ctx, level, false);
      if (!x || !y) throw Fail{LDGS_E_ARG, "null argument"};
      const ImpLevel& L = ctx->imp->lv[level];
      const int nb = ctx->imp->nb;
      for (int64_t e = 0; e < L.NE; ++e)
        for (int r = 0; r < nb; ++r) {
          double s = 0.0;
          for (int k = L.rowptr[e]; k < L.rowptr[e + 1]; ++k) {
            const double* B = L.blk.data() + (size_t)k * nb * nb;
            const double* xf = x + (size_t)L.cols[k] * nb;
            for (int c = 0; c < nb; ++c) s += B[(size_t)c * nb + r] * xf[c];
          }
          y[e * nb + r] = s;
        }
      return LDGS_OK;
    }
    if (level < 0 || level >= (int)ctx->levels.size() || !x || !y) throw Fail{LDGS_E_ARG, "level"};
    host_apply(ctx->levels[level], ctx->g, ctx->B, ctx->P.form, x, y);
    return LDGS_OK;
  } catch (const Fail& f) {
    return handle(ctx, f);
  }
}

ldgs_status ldgs_bottom_info(ldgs_ctx* ctx, int64_t* nc, double* pinv, double* eig) {
  if (!ctx) return LDGS_E_ARG;
  if (nc) *nc = ctx->Nc;
  if (pinv) std::memcpy(pinv, ctx->h_pinv.data(), ctx->h_pinv.size() * sizeof(double));
  if (eig) std::memcpy(eig, ctx->h_eig.data(), ctx->h_eig.size() * sizeof(double));
  return LDGS_OK;
}

}  // extern "C"
