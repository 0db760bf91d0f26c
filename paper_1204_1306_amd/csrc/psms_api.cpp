// C-ABI of libpsms: context, staging of caller buffers, the operators of the
// domain-decomposed Wilson-Dirac hot path, the batched flexible GCR solver with
// Schwarz (SAP) preconditioning and FP64 defect correction, the Schur complement
// and its inverse, and the stochastic determinant-ratio estimator.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <chrono>
#include <cmath>
#include <cstdio>
#include <cstring>
#include <map>
#include <mutex>
#include <random>
#include <string>
#include <vector>

#include "../../include/psms.h"
#include "kernels.h"

using namespace psms;

namespace {

struct Err {
  psms_status st;
  std::string msg;
};

#define HIPCHK(x)                                                                                     \
  do {                                                                                                \
    hipError_t e_ = (x);                                                                              \
    if (e_ != hipSuccess) throw Err{PSMS_EHIP, std::string(#x) + ": " + hipGetErrorString(e_)};        \
  } while (0)

#define REQUIRE(cond, msg) \
  do {                     \
    if (!(cond)) throw Err{PSMS_EINVAL, msg}; \
  } while (0)

struct DevBuf {
  void* p = nullptr;
  size_t n = 0;
};

struct Slot {
  bool loaded = false;
  bool su3 = false;
  void* f64 = nullptr;
  void* c12 = nullptr;
  void* f64_s = nullptr;  // the same links in the solver layout (when the layouts differ)
  void* c12_s = nullptr;
  void* f18 = nullptr;    // FP32 18-real copies, made on first use by a mixed-precision
  void* f18_s = nullptr;  // launch that includes a field that is not SU(3)
};

struct ProfRec {
  int fam;
  hipEvent_t a, b;
  double bytes;
};

enum Fam { FAM_DSLASH = 0, FAM_DSLASH_PART, FAM_BLOCK, FAM_BLOCK_SOLVE, FAM_BLAS, FAM_NET, NFAM };
// block_mr: Schwarz sweeps (fixed iterations); block_solve: block inverses to a tolerance
const char* fam_names[NFAM] = {"dslash", "dslash_part", "block_mr", "block_solve", "blas", "net"};

}  // namespace

// Scratch of psms_apply_dw_noalloc: the two internal-layout fields of one call. Each
// device holds its own copy at its own address (hipGetSymbolAddress, taken once per
// device when a context is created there); host code uses only that address.
constexpr size_t kNoAllocScratchBytes = size_t(64) << 20;
static __device__ __align__(256) unsigned char scratch[kNoAllocScratchBytes];

struct psms_ctx {
  psms_geom geom;
  Geo g;
  int device = 0;
  hipStream_t st = nullptr;
  int V = 0, Vh = 0;
  std::vector<void*> geo_mem;  // device tables of the layouts
  bool split = false;          // the solver works in a second layout with Schwarz blocks sap_b
  Geo gs;                      // that layout
  bool solver_view = false;    // links_of hands out the solver-layout links
  int op_colour = -1;          // >= 0: the solver's operator is D_cc of that colour
  int block_solver = 0;        // block inverses to tolerance: 0 minimal residual, 1 flexible GCR
  int block_lanes = 0;         // LDS-resident block solver: lanes per site (1, 2; 0 = by grid size)
  int block_eo = 2;            // LDS-resident block solver: 1 even-odd, 0 plain, 2 by launch shape
  int block_eo_lanes = 0;      // even-odd form on 256-site FP32 blocks: lanes per site (2, 4; 0 = by grid)
  int block_tol_prec = 0;      // mixed block inverses to tolerance: 1 FP32 passes, 2 FP64, 0 = by block size
  int sap_bf16 = 1;            // BF16 Krylov basis: Schwarz fields in BF16 (1) or FP32 (0)
  int sap_link16 = 2;          // Schwarz sweeps: staged links FP32 (0), FP16 12-real (1), FP16 links and fields (2)
  int block_xcd = 2;           // block launches: right-hand sides of a block back to back on one XCD
                               // (1), launch order (0), 1 when the links exceed the Infinity Cache (2)
  // pinned host slots for the lagged convergence check of the GCR iteration
  double* pinned[2] = {nullptr, nullptr};
  size_t pinned_n = 0;
  hipEvent_t rn_ev[2] = {nullptr, nullptr};
  Slot slots[64];
  std::map<std::string, DevBuf> bufs;
  std::string err;
  size_t held = 0;
  // profiling
  bool prof = false;
  std::vector<ProfRec> recs;
  std::vector<hipEvent_t> pool;
  double prof_ms[NFAM] = {0};
  long long prof_n[NFAM] = {0};
  double prof_bytes[NFAM] = {0};
  // launch tuning (right-hand sides per stencil thread, by precision)
  int nr_f64 = 1, nr_low = 2;
  int variant[3] = {0, 0, 0};  // full-lattice stencil form per spinor storage (F64, F32, BF16)
  int xcd_map = 1;             // per-XCD contiguous tile ranges for stencil launches
  std::string tuned_from;      // "", "autotune" or "cache"
  // learned preconditioner: FP32 master weights, Adam moments, FP64 gradient
  struct Net {
    int nlayers = 0;
    std::vector<int> ch;        // channels, nlayers + 1 entries
    std::vector<size_t> woff;   // complex offset of each layer's weights
    size_t nw = 0;              // complex weights in total
    float* w = nullptr;         // [nw] complex as float pairs
    float* m = nullptr;
    float* v = nullptr;
    double* grad = nullptr;     // [nw] complex as double pairs
    int adam_step = 0;
    std::vector<uint2*> pack_f, pack_a;  // bf16 MFMA fragments of each layer (forward, adjoint)
    bool packed = false;                 // fragments match the FP32 weights
  } net;
  int net_mfma = 1;  // channel mixing on the matrix cores (bf16) or on the vector units (FP32)
  void* noalloc_scratch = nullptr;  // this device's address of `scratch`
};

namespace {

// ------------------------------------------------------------------ memory
void* dev_alloc(psms_ctx* c, size_t bytes) {
  void* p = nullptr;
  if (hipMalloc(&p, std::max<size_t>(bytes, 256)) != hipSuccess) {
    (void)hipGetLastError();
    throw Err{PSMS_ENOMEM, "hipMalloc of " + std::to_string(bytes) + " bytes failed"};
  }
  c->held += bytes;
  return p;
}

void* buf(psms_ctx* c, const std::string& name, size_t bytes) {
  DevBuf& b = c->bufs[name];
  if (b.n < bytes) {
    if (b.p) {
      HIPCHK(hipStreamSynchronize(c->st));
      HIPCHK(hipFree(b.p));
      c->held -= b.n;
    }
    b.p = nullptr;
    b.n = 0;
    b.p = dev_alloc(c, bytes);
    b.n = bytes;
  }
  return b.p;
}

FieldBatch field(psms_ctx* c, const std::string& name, Prec prec, int nprop, int nrhs, int copies = 1) {
  size_t bytes = bytes_per_field(prec, c->Vh) * size_t(nprop) * nrhs * copies;
  return FieldBatch{buf(c, name, bytes), prec, nprop, nrhs};
}

template <class T> T* dscratch(psms_ctx* c, const std::string& name, size_t n) {
  return reinterpret_cast<T*>(buf(c, name, n * sizeof(T)));
}

bool is_device_ptr(const void* p) {
  hipPointerAttribute_t attr;
  if (hipPointerGetAttributes(&attr, p) != hipSuccess) {
    (void)hipGetLastError();
    return false;
  }
  return attr.type == hipMemoryTypeDevice || attr.type == hipMemoryTypeManaged;
}

const double* stage_in(psms_ctx* c, const double* user, size_t ndoubles, const char* name) {
  if (is_device_ptr(user)) return user;
  double* d = dscratch<double>(c, name, ndoubles);
  HIPCHK(hipMemcpyAsync(d, user, ndoubles * sizeof(double), hipMemcpyHostToDevice, c->st));
  return d;
}

double* stage_out(psms_ctx* c, double* user, size_t ndoubles, const char* name) {
  if (is_device_ptr(user)) return user;
  return dscratch<double>(c, name, ndoubles);
}

void finish_out(psms_ctx* c, double* user, double* dev, size_t ndoubles) {
  if (user != dev) HIPCHK(hipMemcpyAsync(user, dev, ndoubles * sizeof(double), hipMemcpyDeviceToHost, c->st));
  HIPCHK(hipStreamSynchronize(c->st));
}

// ------------------------------------------------------------------ profiling
hipEvent_t get_event(psms_ctx* c) {
  if (!c->pool.empty()) {
    hipEvent_t e = c->pool.back();
    c->pool.pop_back();
    return e;
  }
  hipEvent_t e;
  HIPCHK(hipEventCreate(&e));
  return e;
}

}  // namespace
thread_local psms::KernelTimer* psms::t_kernel_timer = nullptr;
namespace {

// Times one family's work on the library's stream. The stencil and block-solver
// families launch through launch_timed, so their span runs from the first kernel's
// start to the last kernel's end (what a kernel trace reports); the other families
// are bracketed by event records.
struct ProfScope {
  psms_ctx* c;
  int fam;
  double bytes;
  hipEvent_t a{}, b{};
  KernelTimer kt{};
  bool kernel_timed = false;
  ProfScope(psms_ctx* c_, int fam_, double bytes_) : c(c_), fam(fam_), bytes(bytes_) {
    if (c->prof) {
      a = get_event(c);
      b = get_event(c);
      kernel_timed = fam == FAM_DSLASH || fam == FAM_DSLASH_PART || fam == FAM_BLOCK || fam == FAM_BLOCK_SOLVE;
      if (kernel_timed) {
        kt = KernelTimer{a, b, false};
        t_kernel_timer = &kt;
      } else {
        HIPCHK(hipEventRecord(a, c->st));
      }
    }
  }
  ~ProfScope() {
    if (c->prof) {
      if (kernel_timed) {
        t_kernel_timer = nullptr;
        if (!kt.used) {  // nothing was launched: an empty span
          (void)hipEventRecord(a, c->st);
          (void)hipEventRecord(b, c->st);
        }
      } else {
        (void)hipEventRecord(b, c->st);
      }
      c->recs.push_back(ProfRec{fam, a, b, bytes});
    }
  }
};

void prof_collect(psms_ctx* c) {
  if (c->recs.empty()) return;
  HIPCHK(hipStreamSynchronize(c->st));
  for (auto& r : c->recs) {
    float ms = 0;
    HIPCHK(hipEventElapsedTime(&ms, r.a, r.b));
    c->prof_ms[r.fam] += ms;
    c->prof_n[r.fam] += 1;
    c->prof_bytes[r.fam] += r.bytes;
    c->pool.push_back(r.a);
    c->pool.push_back(r.b);
  }
  c->recs.clear();
}

// ------------------------------------------------------------------ geometry
// Builds the block-major layout of a lattice L with blocks b (device tables owned by c).
void build_geo(psms_ctx* c, const int* L, const int* b, int apbc, const int* ob, Geo& g) {
  int V = 1, nblk = 1, Vb = 1;
  for (int m = 0; m < 4; ++m) g.ob[m] = ob ? ob[m] : 0;
  for (int m = 0; m < 4; ++m) {
    REQUIRE(L[m] > 0 && L[m] <= 255, "L[mu] must be in [1, 255]");
    REQUIRE(b[m] > 0 && L[m] % b[m] == 0, "L[mu] must be a multiple of b[mu]");
    REQUIRE(b[m] % 2 == 0, "b[mu] must be even (even-odd order inside blocks)");
    REQUIRE((L[m] / b[m]) % 2 == 0, "L[mu]/b[mu] must be even (consistent block colouring)");
    g.L[m] = L[m];
    g.b[m] = b[m];
    g.NB[m] = L[m] / b[m];
    V *= g.L[m];
    nblk *= g.NB[m];
    Vb *= g.b[m];
  }
  g.sB[3] = 1; g.sB[2] = g.NB[3]; g.sB[1] = g.NB[3] * g.NB[2]; g.sB[0] = g.sB[1] * g.NB[1];
  g.sl[3] = 1; g.sl[2] = g.b[3]; g.sl[1] = g.b[3] * g.b[2]; g.sl[0] = g.sl[1] * g.b[1];
  g.Vh = V / 2;
  g.Vbh = Vb / 2;
  g.nblk = nblk;
  g.nblk_c = nblk / 2;
  g.apbc = apbc;
  // local coordinates of (parity, i) and block coordinates of blk
  std::vector<uint32_t> lc(2 * g.Vbh), bc(nblk);
  for (int l0 = 0; l0 < g.b[0]; ++l0)
    for (int l1 = 0; l1 < g.b[1]; ++l1)
      for (int l2 = 0; l2 < g.b[2]; ++l2)
        for (int l3 = 0; l3 < g.b[3]; ++l3) {
          int ll = ((l0 * g.b[1] + l1) * g.b[2] + l2) * g.b[3] + l3;
          int p = (l0 + l1 + l2 + l3) & 1;
          lc[p * g.Vbh + (ll >> 1)] = uint32_t(l0) | (uint32_t(l1) << 8) | (uint32_t(l2) << 16) | (uint32_t(l3) << 24);
        }
  for (int B0 = 0; B0 < g.NB[0]; ++B0)
    for (int B1 = 0; B1 < g.NB[1]; ++B1)
      for (int B2 = 0; B2 < g.NB[2]; ++B2)
        for (int B3 = 0; B3 < g.NB[3]; ++B3) {
          int lexB = ((B0 * g.NB[1] + B1) * g.NB[2] + B2) * g.NB[3] + B3;
          int col = (B0 + B1 + B2 + B3) & 1;
          bc[col * g.nblk_c + (lexB >> 1)] = uint32_t(B0) | (uint32_t(B1) << 8) | (uint32_t(B2) << 16) | (uint32_t(B3) << 24);
        }
  // schedule of blocks for full-lattice launches: black block bi then white block
  // bi (neighbours along direction 3), in lexicographic order of bi. (A Morton order
  // of the block coordinates was measured slower, also for the one-workgroup-per-block
  // forms at 32^4: FP64 283 -> 340 us per launch.)
  std::vector<int> order(nblk);
  for (int k = 0; k < nblk; ++k) order[k] = (k & 1) * g.nblk_c + (k >> 1);
  uint32_t* dl = (uint32_t*)dev_alloc(c, lc.size() * 4);
  uint32_t* db = (uint32_t*)dev_alloc(c, bc.size() * 4);
  int* dord = (int*)dev_alloc(c, order.size() * 4);
  c->geo_mem.insert(c->geo_mem.end(), {(void*)dl, (void*)db, (void*)dord});
  HIPCHK(hipMemcpy(dl, lc.data(), lc.size() * 4, hipMemcpyHostToDevice));
  HIPCHK(hipMemcpy(db, bc.data(), bc.size() * 4, hipMemcpyHostToDevice));
  HIPCHK(hipMemcpy(dord, order.data(), order.size() * 4, hipMemcpyHostToDevice));
  g.lcoord = dl;
  g.bcoord = db;
  g.border = dord;
}

// Host-only checks of a geometry, before any device work: a bad geometry is
// PSMS_EINVAL with a message, whether or not a GPU is present.
void check_geometry(const psms_geom* gm) {
  REQUIRE(gm->kappa > 0 && std::isfinite(gm->kappa), "kappa must be positive");
  const bool any = gm->sap_b[0] || gm->sap_b[1] || gm->sap_b[2] || gm->sap_b[3];
  for (int m = 0; m < 4; ++m) {
    REQUIRE(gm->L[m] > 0 && gm->L[m] <= 255, "L[mu] must be in [1, 255]");
    REQUIRE(gm->b[m] > 0 && gm->L[m] % gm->b[m] == 0, "L[mu] must be a multiple of b[mu]");
    REQUIRE(gm->b[m] % 2 == 0, "b[mu] must be even (even-odd order inside blocks)");
    REQUIRE((gm->L[m] / gm->b[m]) % 2 == 0, "L[mu]/b[mu] must be even (consistent block colouring)");
    if (any) {
      REQUIRE(gm->sap_b[m] > 0 && gm->b[m] % gm->sap_b[m] == 0, "sap_b[mu] must divide b[mu]");
      REQUIRE(gm->sap_b[m] % 2 == 0, "sap_b[mu] must be even");
      REQUIRE((gm->L[m] / gm->sap_b[m]) % 2 == 0, "L[mu]/sap_b[mu] must be even");
    }
  }
  const bool outer = gm->outer_b[0] || gm->outer_b[1] || gm->outer_b[2] || gm->outer_b[3];
  if (outer)
    for (int m = 0; m < 4; ++m) {
      REQUIRE(gm->outer_b[m] > 0 && gm->outer_b[m] % gm->b[m] == 0, "outer_b[mu] must be a multiple of b[mu]");
      REQUIRE((gm->outer_b[m] / gm->b[m]) % 2 == 0, "outer_b[mu]/b[mu] must be even (sub-block colours)");
      REQUIRE(gm->L[m] % gm->outer_b[m] == 0, "outer_b[mu] must divide L[mu]");
    }
}

void setup_geometry(psms_ctx* c, const psms_geom* gm) {
  REQUIRE(gm->kappa > 0 && std::isfinite(gm->kappa), "kappa must be positive");
  const bool outer = gm->outer_b[0] || gm->outer_b[1] || gm->outer_b[2] || gm->outer_b[3];
  build_geo(c, gm->L, gm->b, gm->antiperiodic_t ? 1 : 0, outer ? gm->outer_b : nullptr, c->g);
  c->V = 2 * c->g.Vh;
  c->Vh = c->g.Vh;
  const bool any = gm->sap_b[0] || gm->sap_b[1] || gm->sap_b[2] || gm->sap_b[3];
  c->split = false;
  if (any) {
    for (int m = 0; m < 4; ++m) {
      REQUIRE(gm->sap_b[m] > 0 && gm->b[m] % gm->sap_b[m] == 0, "sap_b[mu] must divide b[mu]");
      c->split |= gm->sap_b[m] != gm->b[m];
    }
    if (c->split) build_geo(c, gm->L, gm->sap_b, gm->antiperiodic_t ? 1 : 0, outer ? gm->outer_b : nullptr, c->gs);
  }
}

// ------------------------------------------------------------------ constants
double2* const_cx(psms_ctx* c, const char* name, int n, double re, double im) {
  std::string key = std::string("const_") + name;
  DevBuf& b = c->bufs[key];
  size_t need = size_t(n) * sizeof(double2);
  if (b.n < need) {
    buf(c, key, need);
    std::vector<double2> h(n, make_double2(re, im));
    HIPCHK(hipMemcpy(c->bufs[key].p, h.data(), need, hipMemcpyHostToDevice));
  }
  return (double2*)c->bufs[key].p;
}

Reducer reducer(psms_ctx* c, int nrhs_total, int kmax) {
  Reducer R;
  R.nwg = 64;
  R.partial = dscratch<double>(c, "reduce_partial", size_t(nrhs_total) * R.nwg * 2 * std::max(kmax, 1));
  return R;
}

// ------------------------------------------------------------------ operators
struct Links {
  const void* p[MAXPROP];
  int fmt;
};

// FP32 18-real copies of a slot's links in both layouts (from its FP64 links, so outer-face
// cuts carry over), made once per load.
static void build_f18(psms_ctx* c, Slot& sl) {
  // the internal layouts: g and, when the solver has its own, gs (swapped in solver view)
  const Geo& gmain = c->solver_view ? c->gs : c->g;
  launch_links_f64_to_f18(c->st, gmain, sl.f64, sl.f18);
  if (c->split) {
    const Geo& gsolv = c->solver_view ? c->g : c->gs;
    launch_links_f64_to_f18(c->st, gsolv, sl.f64_s, sl.f18_s);
  }
}
static void ensure_f18(psms_ctx* c, Slot& sl) {
  if (sl.f18) return;
  sl.f18 = dev_alloc(c, size_t(c->V) * 4 * LkF32F18::NC * 16);
  if (c->split) sl.f18_s = dev_alloc(c, size_t(c->V) * 4 * LkF32F18::NC * 16);
  build_f18(c, sl);
}

// Links of `nprop` gauge slots in the format fmt. A request for FP32 links (LK_F32C12)
// gets the 12-real form when every slot is SU(3); with allow_f18 and a slot that is not,
// every slot of the launch gets the 18-real form (LK_F32F18) instead; without allow_f18
// (the network, which needs SU(3)) such a slot is PSMS_ENOTSU3.
Links links_of(psms_ctx* c, const int* slots, int nprop, int fmt, bool allow_f18) {
  Links L{};
  L.fmt = fmt;
  bool all_su3 = true;
  for (int i = 0; i < nprop; ++i) {
    REQUIRE(slots[i] >= 0 && slots[i] < 64 && c->slots[slots[i]].loaded, "gauge slot not loaded");
    all_su3 &= c->slots[slots[i]].su3;
  }
  if (fmt == LK_F32C12 && !all_su3) {
    if (!allow_f18) throw Err{PSMS_ENOTSU3, "this operation needs SU(3) links (12-real compression)"};
    L.fmt = LK_F32F18;
  }
  for (int i = 0; i < nprop; ++i) {
    Slot& sl = c->slots[slots[i]];
    if (L.fmt == LK_F32C12) {
      L.p[i] = c->solver_view ? sl.c12_s : sl.c12;
    } else if (L.fmt == LK_F32F18) {
      ensure_f18(c, sl);
      L.p[i] = c->solver_view ? sl.f18_s : sl.f18;
    } else {
      L.p[i] = c->solver_view ? sl.f64_s : sl.f64;
    }
  }
  return L;
}
Links links_of(psms_ctx* c, const int* slots, int nprop, int fmt) { return links_of(c, slots, nprop, fmt, false); }

// Workgroup order of a block-solver launch over `nprop` gauge fields (tuning key
// block_xcd). Running the right-hand sides of a block back to back on one XCD pays when
// the links the launch reads do not stay in the 256 MB Infinity Cache between them.
static int block_xcd_of(psms_ctx* c, int fmt, int nprop) {
  if (c->block_xcd != 2) return c->block_xcd;
  const double link_bytes = double(c->V) * 4 * (fmt == LK_F64 ? 144 : 48) * nprop;
  return link_bytes > 256.0 * (1 << 20) ? 1 : 0;
}

double spinor_bytes(Prec p) { return p == P_F64 ? 192.0 : p == P_F32 ? 96.0 : 48.0; }
double link_bytes(int fmt) { return fmt == LK_F64 ? 144.0 : 48.0; }

DslashParams dslash_params(psms_ctx* c, const FieldBatch& in, int sel, int out_colour, double cdiag, double chop,
                           int accumulate) {
  DslashParams dp;
  dp.sel = sel;
  dp.p0 = 0;
  dp.np = 2;
  dp.blk0 = out_colour < 0 ? 0 : out_colour * c->g.nblk_c;
  dp.nb = out_colour < 0 ? c->g.nblk : c->g.nblk_c;
  dp.cdiag = cdiag;
  dp.chop = chop;
  dp.accumulate = accumulate;
  dp.variant = c->variant[in.prec];
  dp.xcd_map = c->xcd_map;
  return dp;
}

// out = cdiag in + chop H_sel in (+ out), on blocks of out_colour (-1: all)
void dslash(psms_ctx* c, const Links& L, const FieldBatch& in, const FieldBatch& out, int sel, int out_colour, double cdiag,
            double chop, int accumulate) {
  DslashParams dp = dslash_params(c, in, sel, out_colour, cdiag, chop, accumulate);
  bool full = sel == HOP_ALL && out_colour < 0 && !accumulate;
  // algorithmic bytes of a full application: every link once, input and output once per rhs
  double bytes = double(c->V) * in.nprop * (4 * link_bytes(L.fmt) + in.nrhs * (spinor_bytes(in.prec) + spinor_bytes(out.prec)));
  ProfScope ps(c, full ? FAM_DSLASH : FAM_DSLASH_PART, full ? bytes : 0.0);
  launch_dslash(c->st, c->g, L.p, L.fmt, in, out, dp, in.prec == P_F64 ? c->nr_f64 : c->nr_low);
}

// The solver's operator: D on the full lattice, or D_cc (blocks of one colour, the
// other colour kept at zero) while a block-diagonal system is being solved.
void apply_D(psms_ctx* c, const Links& L, const FieldBatch& in, const FieldBatch& out) {
  if (c->op_colour >= 0) {
    dslash(c, L, in, out, HOP_INTRA, c->op_colour, 1.0, -c->geom.kappa, 0);
    ProfScope ps(c, FAM_BLAS, 0);
    launch_keep_colour(c->st, c->g, out, c->op_colour);
    return;
  }
  dslash(c, L, in, out, HOP_ALL, -1, 1.0, -c->geom.kappa, 0);
}

void norm2(psms_ctx* c, const FieldBatch& x, double* d_out) {
  ProfScope ps(c, FAM_BLAS, 0);
  reduce_norm2(c->st, c->g, x, reducer(c, x.nprop * x.nrhs, 1), d_out);
}

// Pinned host slot (page-locked, allocated by hipHostMalloc) for n doubles.
double* pinned_slot(psms_ctx* c, int slot, int n) {
  if (c->pinned_n < size_t(n)) {
    HIPCHK(hipStreamSynchronize(c->st));
    for (auto& p : c->pinned) {
      if (p) HIPCHK(hipHostFree(p));
      p = nullptr;
    }
    for (auto& p : c->pinned) HIPCHK(hipHostMalloc((void**)&p, size_t(n) * sizeof(double), hipHostMallocDefault));
    c->pinned_n = n;
  }
  if (!c->rn_ev[0])
    for (auto& e : c->rn_ev) HIPCHK(hipEventCreateWithFlags(&e, hipEventDisableTiming));
  return c->pinned[slot];
}

std::vector<double> to_host(psms_ctx* c, const double* d, int n) {
  std::vector<double> h(n);
  HIPCHK(hipMemcpyAsync(h.data(), d, n * sizeof(double), hipMemcpyDeviceToHost, c->st));
  HIPCHK(hipStreamSynchronize(c->st));
  return h;
}

// Two device arrays (n1 and n2 doubles) to the host behind one synchronisation.
void to_host2(psms_ctx* c, const double* d1, int n1, std::vector<double>& h1, const double* d2, int n2,
              std::vector<double>& h2) {
  h1.resize(n1);
  h2.resize(n2);
  HIPCHK(hipMemcpyAsync(h1.data(), d1, n1 * sizeof(double), hipMemcpyDeviceToHost, c->st));
  HIPCHK(hipMemcpyAsync(h2.data(), d2, n2 * sizeof(double), hipMemcpyDeviceToHost, c->st));
  HIPCHK(hipStreamSynchronize(c->st));
}

// ------------------------------------------------------------------ Schwarz preconditioner
struct SapCfg {
  int cycles, iters;
  Prec prec;
};

// Algorithmic bytes of one block-solver launch over the blocks of one colour: the
// block's links once, rho and x read and written once, delta written once; with the
// face update, also the link and the neighbour's delta of every hop leaving a block.
double block_bytes(psms_ctx* c, const Links& L, const FieldBatch& rho, int face = 0) {
  double sites = double(c->Vh);  // one colour = half the lattice
  double b = sites * rho.nprop * (4 * link_bytes(L.fmt) + rho.nrhs * 5 * spinor_bytes(rho.prec));
  if (face) {
    double hops = 0;  // hops leaving a block, over the sites of one colour
    for (int m = 0; m < 4; ++m) hops += 2.0 * sites / c->g.b[m];
    b += hops * rho.nprop * (link_bytes(L.fmt) + rho.nrhs * spinor_bytes(rho.prec));
  }
  return b;
}

// z = SAP(r): multiplicative Schwarz over black then white blocks, MR block solves.
void sap_apply(psms_ctx* c, const Links& L, const SapCfg& sc, const FieldBatch& r, const FieldBatch& z) {
  const int np = r.nprop, nr = r.nrhs;
  FieldBatch rho = field(c, "sap_rho", sc.prec, np, nr);
  FieldBatch dl = field(c, "sap_delta", sc.prec, np, nr);
  FieldBatch pb = field(c, "sap_p", sc.prec, np, nr);
  // The sweeps of the first cycle assign the iterate (x = delta), so it needs no zeroing,
  // and read their residual straight from r when r has the solver's storage or is the FP32
  // residual of BF16 sweeps (else from a converted copy); the iterate is z itself when z
  // has the solver's storage.
  const bool dz = z.prec == sc.prec, dr = r.prec == sc.prec;
  const bool dr32 = !dr && r.prec == P_F32 && sc.prec == P_BF16;  // the sweeps read an FP32 residual too
  FieldBatch xs = dz ? z : field(c, "sap_x", sc.prec, np, nr);
  if (sc.cycles <= 0) {
    ProfScope ps(c, FAM_BLAS, 0);
    launch_zero(c->st, xs, c->Vh);
  } else if (!dr && !dr32) {
    ProfScope ps(c, FAM_BLAS, 0);
    launch_copy(c->st, c->g, r, rho, nullptr);
  }
  // Block solver form: plain minimal residual (block_eo 0) or even-odd with the 12-real
  // links staged in LDS (1, 2) or read from L2 (3). With 2 (the default) and 3 the Schwarz
  // sweeps run half the iterations, one even-odd iteration reducing the residual about as
  // much as two plain ones. The staged form takes 73 KB of LDS, so two workgroups share a
  // CU, and a hop reads its kappa-scaled link from LDS: at 32^4 a sweep takes 4.55 ms
  // against 5.14 ms with the links read from L2, at 16^4 1.15 against 1.26 ms. With the
  // staged 12-real links in FP16 (sap_link16 1) it takes 49 KB and three workgroups
  // share a CU: 3.66 ms at 32^4, 0.94 ms at 16^4, the same iteration counts. With whole
  // FP16 links, the fields exchanged in FP16 and the face update spread over all lanes
  // (sap_link16 2, the default; 4^4 blocks), 3.19 ms at 32^4, again the same iterations.
  // (Block inverses to a tolerance keep FP32 links.)
  const int eo_form = c->block_eo == 0 ? 0 : c->block_eo == 3 ? 2 : 1;
  const int iters = c->block_eo >= 2 ? (sc.iters + 1) / 2 : sc.iters;
  // Each sweep first applies rho_col -= D_{col,other} delta_other across its block
  // faces (fused into the block kernel), except the very first, where no delta exists.
  for (int cy = 0; cy < sc.cycles; ++cy) {
    for (int col = 0; col < 2; ++col) {
      BlockMRParams bp{col, iters, 0.0, c->geom.kappa};
      bp.face = (cy > 0 || col > 0) ? 1 : 0;
      bp.lanes = c->block_lanes;
      bp.eo_lanes = c->block_eo_lanes;
      bp.xcd_map = block_xcd_of(c, L.fmt, np);
      bp.link16 = c->sap_link16;
      bp.eo = eo_form;
      if (cy == 0) {
        if (dr || dr32) bp.rho_in = r.p;
        bp.rho_in_f32 = dr32 ? 1 : 0;
        bp.x_assign = 1;
      }
      ProfScope ps(c, FAM_BLOCK, block_bytes(c, L, rho, bp.face));
      launch_block_mr(c->st, c->g, L.p, L.fmt, rho, xs, dl, pb, bp, nullptr);
    }
  }
  if (!dz) {
    ProfScope ps(c, FAM_BLAS, 0);
    launch_copy(c->st, c->g, xs, z, nullptr);
  }
}

// ------------------------------------------------------------------ flexible GCR
struct GcrCfg {
  Prec wprec;   // Krylov basis storage
  Prec rprec;   // residual / solution storage
  double tol;
  int maxit, m;
  int pc;
  SapCfg sap;
  const Links* net_links = nullptr;  // 12-real links for the network preconditioner
};

// z = N(r): the learned preconditioner (defined with the network code below)
void net_precondition(psms_ctx* c, const Links& L12, const FieldBatch& r, const FieldBatch& z);

struct GcrResult {
  int iters = 0;
  bool converged = false;
  bool nan = false;
  std::vector<double> rel;  // final recursive relative residual per rhs
};

// Solves D x = b for every rhs of the batch; x is overwritten (start from 0).
GcrResult fgcr(psms_ctx* c, const Links& L, const GcrCfg& cf, const FieldBatch& b, const FieldBatch& x,
               const std::vector<int>* active_in = nullptr) {
  const int np = b.nprop, nrb = b.nrhs, nr = np * nrb, m = cf.m;
  const hipStream_t st = c->st;
  const Geo& g = c->g;
  GcrResult res;
  FieldBatch r = field(c, "gcr_r", cf.rprec, np, nrb);
  FieldBatch Z = field(c, "gcr_Z", cf.wprec, np, nrb, m);
  FieldBatch W = field(c, "gcr_W", cf.wprec, np, nrb, m);
  const size_t vstride = units_per_field(cf.wprec, c->Vh) * size_t(nr);
  const size_t vbytes = bytes_per_field(cf.wprec, c->Vh) * size_t(nr);
  double* bn2 = dscratch<double>(c, "gcr_bn2", nr);
  double* rn2 = dscratch<double>(c, "gcr_rn2", nr);
  double* nw1 = dscratch<double>(c, "gcr_nw1", nr);
  double* NW = dscratch<double>(c, "gcr_NW", size_t(nr) * m);
  double2* A = dscratch<double2>(c, "gcr_A", size_t(nr) * m);
  double2* T = dscratch<double2>(c, "gcr_T", size_t(nr) * m * m);
  double2* ALPHA = dscratch<double2>(c, "gcr_alpha", size_t(nr) * m);
  double2* NEGA = dscratch<double2>(c, "gcr_nega", nr);
  double2* BETA = dscratch<double2>(c, "gcr_beta", size_t(nr) * m);
  double2* D1 = dscratch<double2>(c, "gcr_d", nr);
  int* active = dscratch<int>(c, "gcr_active", nr);
  double* ND = dscratch<double>(c, "gcr_nd", size_t(nr) * 3);
  const double2* ONE = const_cx(c, "one", nr, 1.0, 0.0);
  const double2* MONE = const_cx(c, "mone", nr, -1.0, 0.0);
  const bool same = cf.wprec == cf.rprec;
  Reducer R = reducer(c, nr, std::max(m, 2));  // the fused |w|^2, (w, r) pass needs 3 doubles per partial

  {
    ProfScope ps(c, FAM_BLAS, 0);
    launch_copy(st, g, b, r, nullptr);
    launch_zero(st, x, c->Vh);
  }
  norm2(c, b, bn2);
  std::vector<double> hb = to_host(c, bn2, nr);
  std::vector<int> act(nr);
  for (int i = 0; i < nr; ++i) act[i] = (hb[i] > 0 && (!active_in || (*active_in)[i])) ? 1 : 0;
  HIPCHK(hipMemcpyAsync(active, act.data(), nr * sizeof(int), hipMemcpyHostToDevice, st));
  res.rel.assign(nr, 0.0);
  bool any = false;
  for (int i = 0; i < nr; ++i) any |= act[i] != 0;
  if (!any) {
    res.converged = true;
    return res;
  }

  const double tol2 = cf.tol * cf.tol;
  while (true) {
    int used = 0;
    bool conv = false;
    for (int k = 0; k < m; ++k) {
      FieldBatch Zk{(char*)Z.p + k * vbytes, cf.wprec, np, nrb};
      FieldBatch Wk{(char*)W.p + k * vbytes, cf.wprec, np, nrb};
      if (cf.pc == PSMS_PC_SAP) {
        sap_apply(c, L, cf.sap, r, Zk);
      } else if (cf.pc == PSMS_PC_NET) {
        net_precondition(c, *cf.net_links, r, Zk);
      } else {
        ProfScope ps(c, FAM_BLAS, 0);
        launch_copy(st, g, r, Zk, nullptr);
      }
      apply_D(c, L, Zk, Wk);
      {
        ProfScope ps(c, FAM_BLAS, 0);
        // the scalar steps (projection coefficients, step length) run in the last
        // pass of the reductions that feed them
        const GcrStep gs{k, m, nr, active, NW, A, T, ALPHA, NEGA};
        if (k > 0) reduce_multidot(st, g, W, vstride, k, Wk, R, nullptr, &gs);  // A, T from (W_j, w_k)
        if (same) {
          // fused passes: the orthogonalisation of w_k with |w_k|^2 and (w_k, r), then
          // r -= alpha w_k with |r|^2
          if (k > 0) lincomb_norm_dot(st, g, W, vstride, k, A, m, Wk, r, R, gs);
          else reduce_norm_dot(st, g, Wk, r, R, ND, &gs);
          axpy_norm2(st, g, NEGA, Wk, r, R, rn2);
        } else {
          if (k > 0) launch_lincomb(st, g, W, vstride, k, A, m, Wk, -1);
          if (fused_mixed_ok(Wk, r)) {
            reduce_norm_dot_mixed(st, g, Wk, r, R, ND, &gs);
            axpy_norm2_mixed(st, g, NEGA, Wk, r, R, rn2);
          } else {
            reduce_norm2(st, g, Wk, R, nw1);
            scatter_col(st, nw1, k, m, nr, NW);
            reduce_dot_mixed(st, g, Wk, r, R, D1);
            gcr_alpha(st, D1, NW, k, m, nr, active, ALPHA, NEGA);
            launch_axpy_mixed(st, g, NEGA, Wk, r, +1);
            reduce_norm2(st, g, r, R, rn2);
          }
        }
      }
      // Residual norms go to pinned host memory behind an event; the check of
      // iteration k - 1 happens after iteration k is enqueued, so the host never idles
      // the GPU. Convergence seen one iteration late costs one extra (harmless) step.
      double* hslot = pinned_slot(c, k & 1, nr);
      HIPCHK(hipMemcpyAsync(hslot, rn2, nr * sizeof(double), hipMemcpyDeviceToHost, st));
      HIPCHK(hipEventRecord(c->rn_ev[k & 1], st));
      ++res.iters;
      used = k + 1;
      const bool last = k == m - 1 || res.iters >= cf.maxit;
      auto check = [&](int slot) {
        HIPCHK(hipEventSynchronize(c->rn_ev[slot]));
        const double* hr = pinned_slot(c, slot, nr);
        bool cv = true;
        for (int i = 0; i < nr; ++i) {
          if (!std::isfinite(hr[i])) res.nan = true;
          res.rel[i] = hb[i] > 0 ? std::sqrt(hr[i] / hb[i]) : 0.0;
          if (act[i] && hr[i] > tol2 * hb[i]) cv = false;
        }
        return cv;
      };
      if (k > 0) conv = check((k - 1) & 1);
      if (!conv && !res.nan && last) conv = check(k & 1);
      if (res.nan || conv || res.iters >= cf.maxit) break;
    }
    {
      ProfScope ps(c, FAM_BLAS, 0);
      gcr_backsub(st, T, ALPHA, used, m, nr, BETA);
      if (x.prec == cf.wprec) {
        launch_lincomb(st, g, Z, vstride, used, BETA, m, x, +1);
      } else if (!launch_lincomb_mixed(st, g, Z, vstride, used, BETA, m, x, +1)) {
        // x += beta_j Z_j with Z in a different storage: one mixed axpy per basis vector
        double2* bj = dscratch<double2>(c, "gcr_bj", nr);
        for (int j = 0; j < used; ++j) {
          HIPCHK(hipMemcpy2DAsync(bj, sizeof(double2), BETA + j, m * sizeof(double2), sizeof(double2), nr,
                                  hipMemcpyDeviceToDevice, st));
          FieldBatch Zj{(char*)Z.p + j * vbytes, cf.wprec, np, nrb};
          launch_axpy_mixed(st, g, bj, Zj, x, +1);
        }
      }
    }
    if (res.nan || conv || res.iters >= cf.maxit) {
      res.converged = conv && !res.nan;
      break;
    }
    // restart from the true residual r = b - D x
    apply_D(c, L, x, r);
    ProfScope ps(c, FAM_BLAS, 0);
    launch_axpby(st, g, ONE, b, MONE, r, +1);
  }
  return res;
}

// ------------------------------------------------------------------ full solve (FP64 in and out)
struct FullSolveOut {
  int outer = 0, inner = 0;
  bool converged = false, nan = false, used_fallback = false;
  double max_rel = 0;
};

FullSolveOut solve_full_impl(psms_ctx* c, const int* slots, const psms_solve_params* pp, const FieldBatch& b64,
                             const FieldBatch& x64, const FieldBatch* x0 = nullptr);

// Full-lattice solve D x = b. With a separate Schwarz block size the right-hand sides
// are permuted into the solver layout, solved there and the solutions permuted back.
FullSolveOut solve_full(psms_ctx* c, const int* slots, const psms_solve_params* pp, const FieldBatch& b64,
                        const FieldBatch& x64, const FieldBatch* x0 = nullptr) {
  if (!c->split || c->solver_view) return solve_full_impl(c, slots, pp, b64, x64, x0);
  FieldBatch bs = field(c, "sv_b", P_F64, b64.nprop, b64.nrhs), xs = field(c, "sv_x", P_F64, b64.nprop, b64.nrhs);
  launch_permute(c->st, c->g, c->gs, b64, bs);
  FieldBatch x0s{};
  if (x0) {
    x0s = field(c, "sv_x0", P_F64, x0->nprop, x0->nrhs);
    launch_permute(c->st, c->g, c->gs, *x0, x0s);
  }
  std::swap(c->g, c->gs);
  c->solver_view = true;
  FullSolveOut o;
  try {
    o = solve_full_impl(c, slots, pp, bs, xs, x0 ? &x0s : nullptr);
  } catch (...) {
    std::swap(c->g, c->gs);
    c->solver_view = false;
    throw;
  }
  std::swap(c->g, c->gs);
  c->solver_view = false;
  launch_permute(c->st, c->gs, c->g, xs, x64);
  return o;
}

// x0 (optional): an initial guess of the same shape; convergence is still judged
// against |b|.
FullSolveOut solve_full_impl(psms_ctx* c, const int* slots, const psms_solve_params* pp, const FieldBatch& b64,
                             const FieldBatch& x64, const FieldBatch* x0) {
  FullSolveOut o;
  const int np = b64.nprop, nrb = b64.nrhs, nr = np * nrb;
  const hipStream_t st = c->st;
  Links L64 = links_of(c, slots, np, LK_F64);
  std::vector<double> fin_r2, fin_b2;  // |b - D x|^2 and |b|^2 when already on the host
  int restart = std::max(2, std::min(pp->restart, 64));
  const bool use_net = pp->pc == PSMS_PC_NET;
  if (use_net) REQUIRE(c->net.nlayers > 0, "PC_NET needs a network (psms_net_init or psms_net_load)");
  Links L32{};
  if (pp->prec != PSMS_F64 || use_net) L32 = links_of(c, slots, np, LK_F32C12, !use_net);
  if (pp->prec == PSMS_F64) {
    GcrCfg cf{P_F64, P_F64, pp->tol, pp->max_iter, restart, pp->pc == PSMS_PC_NONE ? PSMS_PC_NONE : PSMS_PC_SAP,
              SapCfg{pp->sap_cycles, pp->block_iters, P_F64}};
    if (use_net) {
      cf.pc = PSMS_PC_NET;
      cf.net_links = &L32;
      if (pp->net_fallback) cf.maxit = std::min(pp->max_iter, 8 * restart);
    }
    // with a guess: D e = b - D x0 to the same absolute residual, x = x0 + e
    FieldBatch rb = b64;
    if (x0) {
      rb = field(c, "fs_r0", P_F64, np, nrb);
      apply_D(c, L64, *x0, rb);
      {
        ProfScope ps(c, FAM_BLAS, 0);
        launch_axpby(st, c->g, const_cx(c, "one", nr, 1, 0), b64, const_cx(c, "mone", nr, -1, 0), rb, +1);
      }
      double* n1 = dscratch<double>(c, "fs_g1", nr);
      double* n2 = dscratch<double>(c, "fs_g2", nr);
      norm2(c, rb, n1);
      norm2(c, b64, n2);
      std::vector<double> h1, h2;
      to_host2(c, n1, nr, h1, n2, nr, h2);
      double ratio = 1e300;
      for (int i = 0; i < nr; ++i)
        if (h1[i] > 0) ratio = std::min(ratio, std::sqrt(h2[i] / h1[i]));
      cf.tol = ratio < 1e300 ? pp->tol * ratio : pp->tol;
    }
    GcrResult gr = fgcr(c, L64, cf, rb, x64);
    if (x0) {
      ProfScope ps(c, FAM_BLAS, 0);
      launch_axpby(st, c->g, const_cx(c, "one", nr, 1, 0), *x0, nullptr, x64, +1);
    }
    o.inner = gr.iters;
    o.outer = 1;
    o.nan = gr.nan;
    if (use_net && pp->net_fallback && !gr.converged && !gr.nan) {
      // the network stalled: finish with Schwarz-preconditioned GCR on the residual
      o.used_fallback = true;
      FieldBatch r64 = field(c, "fb_r64", P_F64, np, nrb);
      FieldBatch e64 = field(c, "fb_e64", P_F64, np, nrb);
      apply_D(c, L64, x64, r64);
      {
        ProfScope ps(c, FAM_BLAS, 0);
        launch_axpby(st, c->g, const_cx(c, "one", nr, 1, 0), b64, const_cx(c, "mone", nr, -1, 0), r64, +1);
      }
      // relative tolerance of the correction solve: tol |b| / |r|
      double* n1 = dscratch<double>(c, "fb_n1", nr);
      double* n2 = dscratch<double>(c, "fb_n2", nr);
      norm2(c, r64, n1);
      norm2(c, b64, n2);
      std::vector<double> h1, h2;
      to_host2(c, n1, nr, h1, n2, nr, h2);
      double ratio = 1.0;
      for (int i = 0; i < nr; ++i)
        if (h1[i] > 0) ratio = std::min(ratio, std::sqrt(h2[i] / h1[i]));
      GcrCfg cs = cf;
      cs.pc = PSMS_PC_SAP;
      cs.maxit = std::max(1, pp->max_iter - gr.iters);
      cs.tol = pp->tol * ratio;
      GcrResult g2 = fgcr(c, L64, cs, r64, e64);
      o.inner += g2.iters;
      o.nan |= g2.nan;
      ProfScope ps(c, FAM_BLAS, 0);
      launch_axpby(st, c->g, const_cx(c, "one", nr, 1, 0), e64, nullptr, x64, +1);
    }
  } else {
    Prec wp = pp->inner_storage == PSMS_SPINOR_BF16 ? P_BF16 : P_F32;
    double itol = pp->inner_tol;
    if (wp == P_BF16) itol = std::max(itol, 5e-3);
    GcrCfg cf{wp, P_F32, itol, restart, restart, pp->pc == PSMS_PC_NONE ? PSMS_PC_NONE : PSMS_PC_SAP,
              SapCfg{pp->sap_cycles, pp->block_iters, (wp == P_BF16 && c->sap_bf16) ? P_BF16 : P_F32}};
    if (use_net) {
      cf.pc = PSMS_PC_NET;
      cf.net_links = &L32;
    }
    FieldBatch r64 = field(c, "dc_r64", P_F64, np, nrb);
    FieldBatch rin = field(c, "dc_rin", P_F32, np, nrb);
    FieldBatch e = field(c, "dc_e", P_F32, np, nrb);
    double* bn2 = dscratch<double>(c, "dc_bn2", nr);
    double* rn2 = dscratch<double>(c, "dc_rn2", nr);
    double* inv = dscratch<double>(c, "dc_inv", nr);
    double2* sq2 = dscratch<double2>(c, "dc_sq2", nr);
    int* dact = dscratch<int>(c, "dc_active", nr);
    const double2* ONE = const_cx(c, "one", nr, 1.0, 0.0);
    const double2* MONE = const_cx(c, "mone", nr, -1.0, 0.0);
    if (x0) {  // start from the guess: x = x0, r = b - D x0
      {
        ProfScope ps(c, FAM_BLAS, 0);
        launch_copy(st, c->g, *x0, x64, nullptr);
      }
      apply_D(c, L64, x64, r64);
      ProfScope ps(c, FAM_BLAS, 0);
      launch_axpby(st, c->g, ONE, b64, MONE, r64, +1);
    } else {
      ProfScope ps(c, FAM_BLAS, 0);
      launch_copy(st, c->g, b64, r64, nullptr);
      launch_zero(st, x64, c->Vh);
    }
    norm2(c, b64, bn2);
    std::vector<double> hb, hr;
    const double tol2 = pp->tol * pp->tol;
    while (true) {
      norm2(c, r64, rn2);
      if (hb.empty()) {
        to_host2(c, bn2, nr, hb, rn2, nr, hr);
      } else {
        hr = to_host(c, rn2, nr);
      }
      std::vector<int> act(nr);
      bool all = true;
      for (int i = 0; i < nr; ++i) {
        if (!std::isfinite(hr[i])) o.nan = true;
        act[i] = (hb[i] > 0 && hr[i] > tol2 * hb[i]) ? 1 : 0;
        if (act[i]) all = false;
      }
      if (all || o.nan || o.inner >= pp->max_iter) {
        o.converged = all && !o.nan;
        // r64 = b - D x64 was just formed in FP64: it is the true residual
        fin_r2 = hr;
        fin_b2 = hb;
        break;
      }
      HIPCHK(hipMemcpyAsync(dact, act.data(), nr * sizeof(int), hipMemcpyHostToDevice, st));
      defect_scales(st, rn2, dact, nr, inv, sq2);
      {
        ProfScope ps(c, FAM_BLAS, 0);
        launch_copy(st, c->g, r64, rin, inv);
      }
      // A pass only has to bring every residual down to tol |b|: once the residual is
      // small, the inner tolerance loosens to half the reduction still needed (never
      // tighter than inner_tol), so the last pass does not over-solve.
      double need = 1.0;
      for (int i = 0; i < nr; ++i)
        if (act[i]) need = std::min(need, pp->tol * std::sqrt(hb[i] / hr[i]));
      GcrCfg ci = cf;
      ci.tol = std::max(cf.tol, 0.5 * need);
      GcrResult gr = fgcr(c, L32, ci, rin, e, &act);
      o.inner += gr.iters;
      if (cf.pc == PSMS_PC_NET && pp->net_fallback) {
        // a network-preconditioned inner solve that does not halve the residual
        // hands the remaining inner solves to the Schwarz preconditioner
        double worst = 0;
        for (int i = 0; i < nr; ++i)
          if (act[i]) worst = std::max(worst, gr.rel[i]);
        if (!(worst <= 0.5)) {
          cf.pc = PSMS_PC_SAP;
          o.used_fallback = true;
        }
      }
      ++o.outer;
      if (gr.nan) {
        o.nan = true;
        break;
      }
      {
        ProfScope ps(c, FAM_BLAS, 0);
        launch_axpy_mixed(st, c->g, sq2, e, x64, +1);
      }
      apply_D(c, L64, x64, r64);
      ProfScope ps(c, FAM_BLAS, 0);
      launch_axpby(st, c->g, ONE, b64, MONE, r64, +1);
    }
  }
  // true FP64 residual (the defect-correction loop ends with it in hand)
  std::vector<double> h1, h2;
  if (!fin_r2.empty()) {
    h1.swap(fin_r2);
    h2.swap(fin_b2);
  } else {
    FieldBatch r64 = field(c, "fs_r", P_F64, np, nrb);
    apply_D(c, L64, x64, r64);
    {
      ProfScope ps(c, FAM_BLAS, 0);
      launch_axpby(st, c->g, const_cx(c, "one", nr, 1, 0), b64, const_cx(c, "mone", nr, -1, 0), r64, +1);
    }
    double* t1 = dscratch<double>(c, "fs_n1", nr);
    double* t2 = dscratch<double>(c, "fs_n2", nr);
    norm2(c, r64, t1);
    norm2(c, b64, t2);
    to_host2(c, t1, nr, h1, t2, nr, h2);
  }
  o.max_rel = 0;
  for (int i = 0; i < nr; ++i) {
    double rel = h2[i] > 0 ? std::sqrt(h1[i] / h2[i]) : std::sqrt(h1[i]);
    if (!std::isfinite(rel)) o.nan = true;
    o.max_rel = std::max(o.max_rel, rel);
  }
  o.converged = !o.nan && o.max_rel <= pp->tol;
  return o;
}

// ------------------------------------------------------------------ block solves to tolerance
// While alive, the solver's operator is D_cc (the blocks of one colour, Dirichlet).
struct ColourOperator {
  psms_ctx* c;
  ColourOperator(psms_ctx* c_, int col) : c(c_) { c->op_colour = col; }
  ~ColourOperator() { c->op_colour = -1; }
};

// Mixed-precision block inverse x = D_cc^-1 b (SU(3) links): FP64 defect correction
// around the FP32 block solver (12-real links, FP32 fields). Each pass solves
// D_cc e = r to 1e-5 relative per block in FP32, adds e to x in FP64 and recomputes
// the FP64 residual r = b_c - D_cc x, until |r| <= tol |b_c| for every right-hand side
// or maxit block iterations are spent. Returns the max relative FP64 residual.
double solve_colour_mixed(psms_ctx* c, const int* slots, int col, const FieldBatch& b, const FieldBatch& x, double tol,
                          int maxit, int* iters_host) {
  const int np = b.nprop, nrb = b.nrhs, nr = np * nrb;
  Links L64 = links_of(c, slots, np, LK_F64);
  Links L32 = links_of(c, slots, np, LK_F32C12, true);
  FieldBatch bc = field(c, "bs_bc", P_F64, np, nrb);
  FieldBatch rt = field(c, "bs_rt", P_F64, np, nrb);
  FieldBatch rho = field(c, "bs_rho32", P_F32, np, nrb);
  FieldBatch e = field(c, "bs_e32", P_F32, np, nrb);
  FieldBatch dl = field(c, "bs_delta32", P_F32, np, nrb);
  FieldBatch pb = field(c, "bs_p32", P_F32, np, nrb);
  int* it = dscratch<int>(c, "bs_iters", 1);
  double* n1 = dscratch<double>(c, "bs_n1", nr);
  double* n2 = dscratch<double>(c, "bs_n2", nr);
  const double2* ONE = const_cx(c, "one", nr, 1, 0);
  const double2* MONE = const_cx(c, "mone", nr, -1, 0);
  {
    ProfScope ps(c, FAM_BLAS, 0);
    launch_copy(c->st, c->g, b, bc, nullptr);
    launch_keep_colour(c->st, c->g, bc, col);
    launch_copy(c->st, c->g, bc, rt, nullptr);  // r = b_c for x = 0
    launch_zero(c->st, x, c->Vh);
  }
  norm2(c, bc, n2);
  const std::vector<double> h2 = to_host(c, n2, nr);
  int total = 0;
  double mx = 1.0;
  for (int pass = 0; pass < 8 && total < maxit; ++pass) {
    HIPCHK(hipMemsetAsync(it, 0, sizeof(int), c->st));
    {
      ProfScope ps(c, FAM_BLAS, 0);
      launch_copy(c->st, c->g, rt, rho, nullptr);  // FP64 -> FP32
      launch_zero(c->st, e, c->Vh);
    }
    {
      ProfScope ps(c, FAM_BLOCK_SOLVE, block_bytes(c, L32, rho));
      BlockMRParams bp{col, maxit - total, 1e-5, c->geom.kappa};
      bp.lanes = c->block_lanes;
      bp.eo_lanes = c->block_eo_lanes;
      bp.xcd_map = block_xcd_of(c, L32.fmt, rho.nprop);
      bp.eo = c->block_eo != 0 ? 1 : 0;
      launch_block_mr(c->st, c->g, L32.p, L32.fmt, rho, e, dl, pb, bp, it);
    }
    int hit = 0;
    HIPCHK(hipMemcpyAsync(&hit, it, sizeof(int), hipMemcpyDeviceToHost, c->st));
    {
      ProfScope ps(c, FAM_BLAS, 0);
      launch_axpy_mixed(c->st, c->g, ONE, e, x, +1);  // x += e in FP64
    }
    dslash(c, L64, x, rt, HOP_INTRA, col, 1.0, -c->geom.kappa, 0);
    {
      ProfScope ps(c, FAM_BLAS, 0);
      launch_keep_colour(c->st, c->g, rt, col);
      launch_axpby(c->st, c->g, ONE, bc, MONE, rt, +1);  // r = b_c - D_cc x
    }
    norm2(c, rt, n1);
    const std::vector<double> h1 = to_host(c, n1, nr);  // synchronises: `hit` is valid
    total += hit;
    mx = 0;
    for (int i = 0; i < nr; ++i) mx = std::max(mx, h2[i] > 0 ? std::sqrt(h1[i] / h2[i]) : std::sqrt(h1[i]));
    if (mx <= tol || hit == 0) break;
  }
  if (iters_host) *iters_host = total;
  return mx;
}

// x = D_cc^-1 b on the blocks of colour col; b is left unchanged. Returns max relative residual.
// By default every block is solved by the minimal-residual kernel, one workgroup per
// block (LDS-resident for blocks of 256 sites). With `mixed` (SU(3) links) and blocks
// that are not LDS-resident, whose solver is bound by memory traffic, the FP64 defect
// correction of solve_colour_mixed runs the block solver in FP32. block_solver = 1
// instead runs flexible GCR on the block-diagonal operator (mixed precision with FP64
// defect correction); measured slower for 8^4 blocks at 32^4 (its Krylov basis costs
// more than it saves).
double solve_colour(psms_ctx* c, const int* slots, int col, const FieldBatch& b, const FieldBatch& x, double tol, int maxit,
                    int* iters_host, bool mixed = false) {
  const int np = b.nprop, nrb = b.nrhs, nr = np * nrb;
  Links L = links_of(c, slots, np, LK_F64);
  const bool passes32 = c->block_tol_prec == 1 || (c->block_tol_prec == 0 && 2 * c->g.Vbh != 256);
  if (mixed && c->block_solver == 0 && passes32) return solve_colour_mixed(c, slots, col, b, x, tol, maxit, iters_host);
  if (c->block_solver == 1) {
    FieldBatch bc = field(c, "bs_bc", P_F64, np, nrb);
    {
      ProfScope ps(c, FAM_BLAS, 0);
      launch_copy(c->st, c->g, b, bc, nullptr);
      launch_keep_colour(c->st, c->g, bc, col);
    }
    psms_solve_params p;
    psms_default_params(&p);
    p.tol = tol;
    p.max_iter = maxit;
    p.restart = 32;
    p.pc = PSMS_PC_NONE;
    p.prec = PSMS_MIXED;
    p.inner_tol = 1e-4;
    ColourOperator guard(c, col);
    FullSolveOut o = solve_full_impl(c, slots, &p, bc, x);
    if (iters_host) *iters_host = o.inner;
    return o.nan ? std::nan("") : o.max_rel;
  }
  FieldBatch rho = field(c, "bs_rho", P_F64, np, nrb);
  FieldBatch dl = field(c, "bs_delta", P_F64, np, nrb);
  FieldBatch pb = field(c, "bs_p", P_F64, np, nrb);
  FieldBatch bc = field(c, "bs_bc", P_F64, np, nrb);
  int* it = dscratch<int>(c, "bs_iters", 1);
  double* n1 = dscratch<double>(c, "bs_n1", nr);
  double* n2 = dscratch<double>(c, "bs_n2", nr);
  {
    ProfScope ps(c, FAM_BLAS, 0);
    launch_copy(c->st, c->g, b, bc, nullptr);
    launch_keep_colour(c->st, c->g, bc, col);
    launch_copy(c->st, c->g, bc, rho, nullptr);
    launch_zero(c->st, x, c->Vh);
  }
  norm2(c, bc, n2);
  HIPCHK(hipMemsetAsync(it, 0, sizeof(int), c->st));
  {
    ProfScope ps(c, FAM_BLOCK_SOLVE, block_bytes(c, L, rho));
    BlockMRParams bp{col, maxit, tol, c->geom.kappa};
    bp.lanes = c->block_lanes;
    bp.eo_lanes = c->block_eo_lanes;
    bp.xcd_map = block_xcd_of(c, L.fmt, rho.nprop);
    bp.eo = c->block_eo != 0 ? 1 : 0;  // to a tolerance the even-odd form always pays
    launch_block_mr(c->st, c->g, L.p, L.fmt, rho, x, dl, pb, bp, it);
  }
  if (iters_host) HIPCHK(hipMemcpyAsync(iters_host, it, sizeof(int), hipMemcpyDeviceToHost, c->st));
  // true relative residual |b_c - D_cc x| / |b_c|
  FieldBatch rt = field(c, "bs_rt", P_F64, np, nrb);
  dslash(c, L, x, rt, HOP_INTRA, col, 1.0, -c->geom.kappa, 0);
  {
    ProfScope ps(c, FAM_BLAS, 0);
    launch_keep_colour(c->st, c->g, rt, col);
    launch_axpby(c->st, c->g, const_cx(c, "one", nr, 1, 0), bc, const_cx(c, "mone", nr, -1, 0), rt, +1);
  }
  norm2(c, rt, n1);
  std::vector<double> h1, h2;
  to_host2(c, n1, nr, h1, n2, nr, h2);
  double mx = 0;
  for (int i = 0; i < nr; ++i) mx = std::max(mx, h2[i] > 0 ? std::sqrt(h1[i] / h2[i]) : std::sqrt(h1[i]));
  return mx;
}

// out = (1 - P Q) xi, Q = D_bb^-1 D_bw D_ww^-1 D_wb. Returns worst block-solve residual.
// With zg: also zg = [-Q xi]_black + [D_ww^-1 D_wb xi]_white, which solves
// D z = 0 (+) D_wb (1 - PQ) xi exactly (D_wb P = D_wb): the solution that the inverse
// of eq. inverseschur needs for these links, and a close guess for nearby links.
double schur_apply(psms_ctx* c, const int* slots, const FieldBatch& xi, const FieldBatch& out, double tol, int maxit,
                   bool mixed = false, const FieldBatch* zg = nullptr) {
  const int np = xi.nprop, nrb = xi.nrhs;
  Links L = links_of(c, slots, np, LK_F64);
  FieldBatch t1 = field(c, "sc_t1", P_F64, np, nrb);
  FieldBatch t2 = field(c, "sc_t2", P_F64, np, nrb);
  {
    ProfScope ps(c, FAM_BLAS, 0);
    launch_zero(c->st, t1, c->Vh);
  }
  dslash(c, L, xi, t1, HOP_CROSS, 1, 0.0, -c->geom.kappa, 0);  // D_wb xi (white sites)
  double r1 = solve_colour(c, slots, 1, t1, t2, tol, maxit, nullptr, mixed);  // D_ww^-1
  {
    ProfScope ps(c, FAM_BLAS, 0);
    if (zg) launch_copy(c->st, c->g, t2, *zg, nullptr);  // white part (black sites are zero)
    launch_zero(c->st, t1, c->Vh);
  }
  dslash(c, L, t2, t1, HOP_CROSS, 0, 0.0, -c->geom.kappa, 0);  // D_bw (black sites)
  double r2 = solve_colour(c, slots, 0, t1, t2, tol, maxit, nullptr, mixed);  // D_bb^-1
  {
    ProfScope ps(c, FAM_BLAS, 0);
    const int nr = np * nrb;
    if (zg) launch_axpby(c->st, c->g, const_cx(c, "mone", nr, -1, 0), t2, nullptr, *zg, +1);  // black part -Q xi
    launch_project(c->st, c->g, t2, t1);
    launch_copy(c->st, c->g, xi, out, nullptr);
    launch_axpby(c->st, c->g, const_cx(c, "mone", nr, -1, 0), t1, nullptr, out, +1);
  }
  return std::max(r1, r2);
}

// out = phi - P [D^-1 (0 + D_wb phi)]  (eq. inverseschur)
FullSolveOut schur_inverse(psms_ctx* c, const int* slots, const psms_solve_params* pp, const FieldBatch& phi,
                           const FieldBatch& out, const FieldBatch* x0 = nullptr) {
  const int np = phi.nprop, nrb = phi.nrhs, nr = np * nrb;
  Links L64 = links_of(c, slots, np, LK_F64);
  FieldBatch v = field(c, "si_v", P_F64, np, nrb);
  FieldBatch x = field(c, "si_x", P_F64, np, nrb);
  {
    ProfScope ps(c, FAM_BLAS, 0);
    launch_zero(c->st, v, c->Vh);
  }
  dslash(c, L64, phi, v, HOP_CROSS, 1, 0.0, -c->geom.kappa, 0);
  FullSolveOut o = solve_full(c, slots, pp, v, x, x0);
  ProfScope ps(c, FAM_BLAS, 0);
  launch_project(c->st, c->g, x, v);
  launch_copy(c->st, c->g, phi, out, nullptr);
  launch_axpby(c->st, c->g, const_cx(c, "mone", nr, -1, 0), v, nullptr, out, +1);
  return o;
}

psms_status fail(psms_ctx* c, const Err& e) {
  if (c) c->err = e.msg;
  return e.st;
}

#define API_BEGIN(ctx)                         \
  if (!(ctx)) return PSMS_EINVAL;              \
  try {                                        \
    HIPCHK(hipSetDevice((ctx)->device));
#define API_END(ctx)                           \
  }                                            \
  catch (const Err& e) {                       \
    return fail(ctx, e);                       \
  }                                            \
  catch (const std::exception& e) {            \
    return fail(ctx, Err{PSMS_EINVAL, e.what()}); \
  }

void check_rhs(int nrhs) { REQUIRE(nrhs >= 1, "nrhs must be >= 1"); }

}  // namespace

// ====================================================================== network host code
namespace {

size_t net_layer_size(int cin, int cout) { return size_t(9) * cout * cin * 16; }  // complex entries

void net_free(psms_ctx* c) {
  auto& n = c->net;
  for (void* p : {(void*)n.w, (void*)n.m, (void*)n.v, (void*)n.grad})
    if (p) (void)hipFree(p);
  for (auto* p : n.pack_f) (void)hipFree(p);
  for (auto* p : n.pack_a) (void)hipFree(p);
  n = psms_ctx::Net{};
}

void net_alloc(psms_ctx* c, const std::vector<int>& ch) {
  REQUIRE(ch.size() >= 2, "a network needs at least one layer");
  for (int v : ch) REQUIRE(v >= 1 && v <= 8, "channel counts must be in [1, 8]");
  REQUIRE(ch.front() == 1 && ch.back() == 1, "the preconditioner maps one spinor field to one");
  HIPCHK(hipStreamSynchronize(c->st));
  net_free(c);
  auto& n = c->net;
  n.nlayers = int(ch.size()) - 1;
  n.ch = ch;
  n.nw = 0;
  for (int l = 0; l < n.nlayers; ++l) {
    n.woff.push_back(n.nw);
    n.nw += net_layer_size(ch[l], ch[l + 1]);
  }
  n.w = (float*)dev_alloc(c, n.nw * 2 * sizeof(float));
  n.m = (float*)dev_alloc(c, n.nw * 2 * sizeof(float));
  n.v = (float*)dev_alloc(c, n.nw * 2 * sizeof(float));
  n.grad = (double*)dev_alloc(c, n.nw * 2 * sizeof(double));
  std::vector<float> z(n.nw * 2, 0.f);
  HIPCHK(hipMemcpy(n.m, z.data(), z.size() * sizeof(float), hipMemcpyHostToDevice));
  HIPCHK(hipMemcpy(n.v, z.data(), z.size() * sizeof(float), hipMemcpyHostToDevice));
  n.adam_step = 0;
  for (int l = 0; l < n.nlayers; ++l) {
    n.pack_f.push_back((uint2*)dev_alloc(c, net_pack_units(ch[l], ch[l + 1], 0) * sizeof(uint2)));
    n.pack_a.push_back((uint2*)dev_alloc(c, net_pack_units(ch[l], ch[l + 1], 1) * sizeof(uint2)));
  }
  n.packed = false;
}

const float2* net_W(psms_ctx* c, int l) { return reinterpret_cast<const float2*>(c->net.w) + c->net.woff[l]; }

// (re)pack the bf16 MFMA fragments after the FP32 weights changed
void net_ensure_packed(psms_ctx* c) {
  auto& n = c->net;
  if (n.packed || !c->net_mfma) return;
  for (int l = 0; l < n.nlayers; ++l) {
    launch_net_pack(c->st, net_W(c, l), n.ch[l], n.ch[l + 1], 0, n.pack_f[l]);
    launch_net_pack(c->st, net_W(c, l), n.ch[l], n.ch[l + 1], 1, n.pack_a[l]);
  }
  n.packed = true;
}

void net_layer(psms_ctx* c, const void* links12, const void* in, void* out, int l, int adj, int nb) {
  auto& n = c->net;
  ProfScope ps(c, FAM_NET, 0);
  if (c->net_mfma) {
    net_ensure_packed(c);
    launch_net_layer_mfma(c->st, c->g, links12, in, out, adj ? n.pack_a[l] : n.pack_f[l], n.ch[l], n.ch[l + 1], adj, nb);
  } else {
    launch_net_layer(c->st, c->g, links12, in, out, net_W(c, l), n.ch[l], n.ch[l + 1], adj, nb);
  }
}

// Forward pass of a batch of nb F32 fields (one gauge field). acts[l] receive the
// activations when given (training); otherwise two ping-pong buffers are used.
void net_forward(psms_ctx* c, const void* links12, const void* in, int nb, void* out, std::vector<void*>* acts) {
  auto& n = c->net;
  const size_t fb = bytes_per_field(P_F32, c->Vh);
  int maxc = 1;
  for (int v : n.ch) maxc = std::max(maxc, v);
  const void* cur = in;
  for (int l = 0; l < n.nlayers; ++l) {
    void* dst;
    if (l == n.nlayers - 1) dst = out;
    else if (acts) dst = (*acts)[l + 1];
    else dst = buf(c, (l & 1) ? "net_pong" : "net_ping", fb * nb * maxc);
    net_layer(c, links12, cur, dst, l, 0, nb);
    cur = dst;
  }
}

void net_precondition(psms_ctx* c, const Links& L12, const FieldBatch& r, const FieldBatch& z) {
  const int nrb = r.nrhs;
  FieldBatch in = field(c, "net_in", P_F32, 1, nrb), out = field(c, "net_out", P_F32, 1, nrb);
  for (int p = 0; p < r.nprop; ++p) {
    FieldBatch rp{(char*)r.p + size_t(p) * nrb * bytes_per_field(r.prec, c->Vh), r.prec, 1, nrb};
    FieldBatch zp{(char*)z.p + size_t(p) * nrb * bytes_per_field(z.prec, c->Vh), z.prec, 1, nrb};
    {
      ProfScope ps(c, FAM_BLAS, 0);
      launch_copy(c->st, c->g, rp, in, nullptr);
    }
    net_forward(c, L12.p[p], in.p, nrb, out.p, nullptr);
    ProfScope ps(c, FAM_BLAS, 0);
    launch_copy(c->st, c->g, out, zp, nullptr);
  }
}

// One optimisation step (or, with step == false, only loss and gradient) on nb pairs
// (r, e) held as F32 fields. Loss sum_b |N(r_b) - e_b|^2 / |e_b|^2, divided by nb when
// mean is set; the gradient dL/dconj(W) lands in c->net.grad.
double net_loss_grad(psms_ctx* c, const void* links12, const FieldBatch& r, const FieldBatch& e, const double* en2_host,
                     int nb, bool mean) {
  auto& n = c->net;
  const hipStream_t st = c->st;
  const size_t fb = bytes_per_field(P_F32, c->Vh);
  std::vector<void*> acts(n.nlayers + 1), grads(n.nlayers + 1);
  acts[0] = r.p;
  for (int l = 1; l <= n.nlayers; ++l) {
    acts[l] = buf(c, "net_act" + std::to_string(l), fb * nb * n.ch[l]);
    grads[l] = buf(c, "net_grad" + std::to_string(l), fb * nb * n.ch[l]);
  }
  net_forward(c, links12, r.p, nb, acts[n.nlayers], &acts);
  // G_L = (out - e) / (|e|^2 [nb])
  FieldBatch out{acts[n.nlayers], P_F32, 1, nb};
  FieldBatch G{grads[n.nlayers], P_F32, 1, nb};
  double2* s = dscratch<double2>(c, "net_scale", nb);
  std::vector<double> hs(nb);
  std::vector<double2> hs2(nb);
  for (int b = 0; b < nb; ++b) {
    hs[b] = 1.0 / (en2_host[b] * (mean ? nb : 1));
    hs2[b] = make_double2(hs[b], 0.0);
  }
  HIPCHK(hipMemcpyAsync(s, hs2.data(), nb * sizeof(double2), hipMemcpyHostToDevice, st));
  double* d2 = dscratch<double>(c, "net_d2", nb);
  {
    ProfScope ps(c, FAM_BLAS, 0);
    launch_copy(st, c->g, out, G, nullptr);
    launch_axpby(st, c->g, const_cx(c, "mone", nb, -1, 0), e, nullptr, G, +1);
    reduce_norm2(st, c->g, G, reducer(c, nb, 1), d2);
    launch_axpby(st, c->g, nullptr, G, s, G, +1);  // G *= s per pair
  }
  HIPCHK(hipStreamSynchronize(st));  // hs2 lives on the host stack
  std::vector<double> hd = to_host(c, d2, nb);
  double loss = 0;
  for (int b = 0; b < nb; ++b) loss += hd[b] * hs[b];
  // backward
  const int nparts = net_wgrad_partials(c->g, nb);
  size_t maxent = 0;
  for (int l = 0; l < n.nlayers; ++l) maxent = std::max(maxent, net_layer_size(n.ch[l], n.ch[l + 1]));
  float2* partial = dscratch<float2>(c, "net_partial", size_t(nparts) * maxent);
  for (int l = n.nlayers - 1; l >= 0; --l) {
    ProfScope ps(c, FAM_NET, 0);
    launch_net_wgrad(st, c->g, links12, acts[l], grads[l + 1], n.ch[l], n.ch[l + 1], nb, partial,
                     reinterpret_cast<double2*>(n.grad) + n.woff[l]);
    if (l > 0) net_layer(c, links12, grads[l + 1], grads[l], l, 1, nb);
  }
  return loss;
}

}  // namespace

// ====================================================================== C-ABI
extern "C" {

void psms_default_params(psms_solve_params* p) {
  if (!p) return;
  p->tol = 1e-10;
  p->max_iter = 2000;
  p->restart = 16;
  p->prec = PSMS_F64;
  p->pc = PSMS_PC_SAP;
  p->sap_cycles = 4;
  p->block_iters = 6;
  p->inner_tol = 1e-2;
  p->inner_storage = PSMS_SPINOR_F32;
  p->net_fallback = 1;
  p->rhs_chunk = 0;
}

const char* psms_status_string(psms_status s) {
  switch (s) {
    case PSMS_OK: return "ok";
    case PSMS_EINVAL: return "invalid argument";
    case PSMS_ENOMEM: return "out of device memory";
    case PSMS_EHIP: return "HIP runtime error";
    case PSMS_ENOTCONV: return "solver did not converge";
    case PSMS_ENOTSU3: return "link not in SU(3)";
    case PSMS_ENAN: return "NaN in residual";
  }
  return "unknown status";
}

// Device address of `scratch` on `device` (current), looked up once per device.
static void* noalloc_scratch_address(int device) {
  static std::mutex mu;
  static std::map<int, void*> addr;
  std::lock_guard<std::mutex> lock(mu);
  auto it = addr.find(device);
  if (it != addr.end()) return it->second;
  void* p = nullptr;
  HIPCHK(hipGetSymbolAddress(&p, HIP_SYMBOL(scratch)));
  addr[device] = p;
  return p;
}

psms_status psms_create(const psms_geom* geom, int device, void* hip_stream, psms_ctx** out) {
  if (!geom || !out) return PSMS_EINVAL;
  *out = nullptr;
  try {
    check_geometry(geom);
  } catch (const Err& e) {
    fprintf(stderr, "psms_create: %s\n", e.msg.c_str());
    return e.st;
  }
  psms_ctx* c = new psms_ctx();
  try {
    c->geom = *geom;
    c->device = device;
    HIPCHK(hipSetDevice(device));
    c->st = reinterpret_cast<hipStream_t>(hip_stream);
    c->noalloc_scratch = noalloc_scratch_address(device);
    setup_geometry(c, geom);
  } catch (const Err& e) {
    psms_status s = e.st;
    fprintf(stderr, "psms_create: %s\n", e.msg.c_str());
    psms_destroy(c);
    return s;
  }
  *out = c;
  return PSMS_OK;
}

void psms_destroy(psms_ctx* c) {
  if (!c) return;
  (void)hipSetDevice(c->device);
  (void)hipStreamSynchronize(c->st);
  for (auto& kv : c->bufs)
    if (kv.second.p) (void)hipFree(kv.second.p);
  for (auto& s : c->slots)
    for (void* p : {s.f64, s.c12, s.f64_s, s.c12_s, s.f18, s.f18_s})
      if (p) (void)hipFree(p);
  for (void* p : c->geo_mem) (void)hipFree(p);
  for (auto& r : c->recs) {
    (void)hipEventDestroy(r.a);
    (void)hipEventDestroy(r.b);
  }
  for (auto e : c->pool) (void)hipEventDestroy(e);
  for (auto p : c->pinned)
    if (p) (void)hipHostFree(p);
  for (auto e : c->rn_ev)
    if (e) (void)hipEventDestroy(e);
  net_free(c);
  delete c;
}

const char* psms_last_error(const psms_ctx* c) { return c ? c->err.c_str() : "null context"; }

unsigned long long psms_device_bytes(const psms_ctx* c) { return c ? (unsigned long long)c->held : 0ull; }

// Loads the device field dU (boundary layout) into slot: internal FP64 and 12-real copies
// in every layout, outer-face links removed, unitarity checked. Returns PSMS_ENOTSU3 (the
// FP64 copy still loaded) for links that are not SU(3).
static psms_status load_links(psms_ctx* c, int slot, const double* dU) {
  Slot& s = c->slots[slot];
  if (!s.f64) s.f64 = dev_alloc(c, size_t(c->V) * 4 * 9 * 16);
  if (!s.c12) s.c12 = dev_alloc(c, size_t(c->V) * 4 * 3 * 16);
  launch_pack_links(c->st, c->g, dU, s.f64, LK_F64);
  launch_pack_links(c->st, c->g, dU, s.c12, LK_F32C12);
  if (c->split) {
    if (!s.f64_s) s.f64_s = dev_alloc(c, size_t(c->V) * 4 * 9 * 16);
    if (!s.c12_s) s.c12_s = dev_alloc(c, size_t(c->V) * 4 * 3 * 16);
    launch_pack_links(c->st, c->gs, dU, s.f64_s, LK_F64);
    launch_pack_links(c->st, c->gs, dU, s.c12_s, LK_F32C12);
  }
  if (c->g.ob[0]) {
    // recursive decomposition: the operator is the direct sum of the outer blocks'
    // Dirichlet operators, i.e. D of the field without its links across outer faces
    // (a zero link is exact in the 12-real form as well: its rebuilt row is zero too)
    launch_cut_links(c->st, c->g, s.f64, LK_F64);
    launch_cut_links(c->st, c->g, s.c12, LK_F32C12);
    if (c->split) {
      launch_cut_links(c->st, c->gs, s.f64_s, LK_F64);
      launch_cut_links(c->st, c->gs, s.c12_s, LK_F32C12);
    }
  }
  if (s.f18) build_f18(c, s);  // 18-real copies made for the previous field follow the new one
  const int nwg = 256;
  double* part = dscratch<double>(c, "unit_partial", nwg);
  launch_unitarity(c->st, c->g, dU, part, nwg);
  std::vector<double> h = to_host(c, part, nwg);
  double dev = 0;
  for (double v : h) dev = (v > dev || v != v) ? v : dev;
  if (!std::isfinite(dev)) {
    s.loaded = false;
    throw Err{PSMS_EINVAL, "gauge field holds a NaN or Inf entry; slot left unloaded"};
  }
  s.loaded = true;
  s.su3 = dev <= 1e-6;
  if (!s.su3) {
    c->err = "gauge field deviates from SU(3) by " + std::to_string(dev) + "; mixed precision disabled for this slot";
    return PSMS_ENOTSU3;
  }
  return PSMS_OK;
}

psms_status psms_gauge_load(psms_ctx* c, int slot, const double* U) {
  API_BEGIN(c)
  REQUIRE(slot >= 0 && slot < 64, "slot out of range");
  REQUIRE(U != nullptr, "null gauge field");
  const double* dU = stage_in(c, U, size_t(c->V) * 4 * 18, "stage_gauge");
  return load_links(c, slot, dU);
  API_END(c)
  return PSMS_OK;
}

void psms_default_gf_params(psms_gf_params* p) {
  if (!p) return;
  p->alpha = 0.15;
  p->alpha_min = 0.10;
  p->theta_tol = 1e-3;
  p->max_iter = 1000;
}

psms_status psms_relative_gauge_fix(psms_ctx* c, int slot_U, int slot_Up, const psms_gf_params* gp, int slot_gU,
                                    int slot_gUp, double* g_out, psms_gf_stats* stats) {
  API_BEGIN(c)
  psms_gf_params def;
  psms_default_gf_params(&def);
  const psms_gf_params& P = gp ? *gp : def;
  REQUIRE(P.alpha > 0 && P.alpha_min > 0 && P.alpha_min <= P.alpha && P.max_iter >= 0 && P.theta_tol >= 0,
          "bad gauge-fixing parameters");
  for (int sl : {slot_U, slot_Up, slot_gU, slot_gUp}) REQUIRE(sl >= 0 && sl < 64, "slot out of range");
  REQUIRE(c->slots[slot_U].loaded && c->slots[slot_Up].loaded, "gauge slot not loaded");
  REQUIRE(slot_gU != slot_gUp, "the two output slots must differ");
  REQUIRE(!c->g.ob[0], "relative gauge fixing takes a context without outer blocks");
  const Geo& g = c->g;
  const size_t nl = size_t(c->V) * 4 * 18, ns = size_t(c->V) * 18;
  double* U = dscratch<double>(c, "gf_U", nl);
  double* Up = dscratch<double>(c, "gf_Up", nl);
  double* Upc = dscratch<double>(c, "gf_Upc", nl);
  double* Upt = dscratch<double>(c, "gf_Upt", nl);
  double* K = dscratch<double>(c, "gf_K", ns);
  double* G = dscratch<double>(c, "gf_G", ns);
  double* gf = dscratch<double>(c, "gf_g", ns);
  const int np = gf_partials(g);
  double* part = dscratch<double>(c, "gf_part", np);
  launch_gf_unpack(c->st, g, c->slots[slot_U].f64, U);
  launch_gf_unpack(c->st, g, c->slots[slot_Up].f64, Up);
  HIPCHK(hipMemcpyAsync(Upc, Up, nl * sizeof(double), hipMemcpyDeviceToDevice, c->st));
  launch_gf_eye(c->st, g, G);
  long long ndom = 1;
  for (int m = 0; m < 4; ++m) ndom *= std::max(0, g.b[m] - 2);
  ndom *= g.nblk;
  auto total = [&](void) {
    std::vector<double> h = to_host(c, part, np);
    double t = 0.0;
    for (double v : h) t += v;
    return t;
  };
  const double norm = 12.0 * c->V;
  launch_gf_overlap(c->st, g, U, Upc, part);
  double f = (norm - total()) / norm;
  psms_gf_stats st{0, f, f, 0.0, P.alpha};
  double alpha = P.alpha;
  int it = 0;
  while (ndom > 0 && it < P.max_iter) {
    launch_gf_step(c->st, g, U, Upc, K, 0.5 * alpha, part);
    const double th = total() / double(ndom);
    st.theta_end = th;
    if (th < P.theta_tol) break;
    launch_gf_trial(c->st, g, U, Upc, K, Upt, part);
    const double fn = (norm - total()) / norm;
    ++it;
    if (fn > f) {
      // the step raised eq. relgf: rejected, alpha lowered by 0.01 down to alpha_min
      if (alpha - 0.01 < P.alpha_min - 1e-12) break;
      alpha -= 0.01;
      continue;
    }
    std::swap(Upc, Upt);
    f = fn;
    launch_gf_accept(c->st, g, G, K);
  }
  // Upc/Upt were swapped on the host only: keep the buffer names pointing where they were
  c->bufs["gf_Upc"].p = Upc;
  c->bufs["gf_Upt"].p = Upt;
  st.iterations = it;
  st.functional_end = f;
  st.alpha_end = alpha;
  // g = G^(1/2), then the fixed pair into the output slots (U and Upt hold them in turn)
  double* Ug = Upt;
  double* Upg = dscratch<double>(c, "gf_Upg", nl);
  launch_gf_finish(c->st, g, G, gf, U, Up, Ug, Upg);
  HIPCHK(hipGetLastError());
  psms_status s1 = load_links(c, slot_gU, Ug);
  psms_status s2 = load_links(c, slot_gUp, Upg);
  if (g_out) {
    if (is_device_ptr(g_out)) {
      HIPCHK(hipMemcpyAsync(g_out, gf, ns * sizeof(double), hipMemcpyDeviceToDevice, c->st));
    } else {
      HIPCHK(hipMemcpyAsync(g_out, gf, ns * sizeof(double), hipMemcpyDeviceToHost, c->st));
    }
  }
  HIPCHK(hipStreamSynchronize(c->st));
  if (stats) *stats = st;
  if (s1 != PSMS_OK) return s1;
  if (s2 != PSMS_OK) return s2;
  API_END(c)
  return PSMS_OK;
}

psms_status psms_apply_dw(psms_ctx* c, int slot, const double* in, double* out, int nrhs, psms_prec prec) {
  API_BEGIN(c)
  check_rhs(nrhs);
  size_t nd = size_t(nrhs) * c->V * 24;
  const double* din = stage_in(c, in, nd, "stage_in");
  double* dout = stage_out(c, out, nd, "stage_out");
  Prec p = prec == PSMS_F64 ? P_F64 : P_F32;
  Links L = links_of(c, &slot, 1, prec == PSMS_F64 ? LK_F64 : LK_F32C12, true);
  FieldBatch a = field(c, "api_a", p, 1, nrhs), b = field(c, "api_b", p, 1, nrhs);
  launch_pack(c->st, c->g, din, a);
  apply_D(c, L, a, b);
  launch_unpack(c->st, c->g, b, dout);
  finish_out(c, out, dout, nd);
  API_END(c)
  return PSMS_OK;
}

psms_status psms_apply_dw_lowp(psms_ctx* c, int slot, const double* in, double* out, int nrhs,
                               psms_inner_storage in_storage, psms_inner_storage out_storage) {
  API_BEGIN(c)
  check_rhs(nrhs);
  REQUIRE((in_storage == PSMS_SPINOR_F32 || in_storage == PSMS_SPINOR_BF16) &&
              (out_storage == PSMS_SPINOR_F32 || out_storage == PSMS_SPINOR_BF16),
          "storage must be PSMS_SPINOR_F32 or PSMS_SPINOR_BF16");
  REQUIRE(!(in_storage == PSMS_SPINOR_F32 && out_storage == PSMS_SPINOR_BF16),
          "an FP32 input takes an FP32 output (the solvers never round an FP32 stencil result to BF16)");
  size_t nd = size_t(nrhs) * c->V * 24;
  const double* din = stage_in(c, in, nd, "stage_in");
  double* dout = stage_out(c, out, nd, "stage_out");
  Prec pi = in_storage == PSMS_SPINOR_BF16 ? P_BF16 : P_F32;
  Prec po = out_storage == PSMS_SPINOR_BF16 ? P_BF16 : P_F32;
  Links L = links_of(c, &slot, 1, LK_F32C12, true);
  FieldBatch a = field(c, "api_lp_a", pi, 1, nrhs), b = field(c, "api_lp_b", po, 1, nrhs);
  launch_pack(c->st, c->g, din, a);
  dslash(c, L, a, b, HOP_ALL, -1, 1.0, -c->geom.kappa, 0);
  launch_unpack(c->st, c->g, b, dout);
  finish_out(c, out, dout, nd);
  API_END(c)
  return PSMS_OK;
}

psms_status psms_apply_dw_noalloc(psms_ctx* c, int slot, const double* in, double* out, int nrhs, psms_prec prec) {
  API_BEGIN(c)
  check_rhs(nrhs);
  REQUIRE(in && out, "null field pointer");
  REQUIRE(prec == PSMS_F64 || prec == PSMS_MIXED, "prec must be PSMS_F64 or PSMS_MIXED");
  for (const void* p : {(const void*)in, (const void*)out}) {
    hipPointerAttribute_t attr;
    bool dev = hipPointerGetAttributes(&attr, p) == hipSuccess &&
               (attr.type == hipMemoryTypeDevice || attr.type == hipMemoryTypeManaged) && attr.device == c->device;
    if (!dev) (void)hipGetLastError();
    REQUIRE(dev, "psms_apply_dw_noalloc takes device memory of the context's device only (host buffers would need "
                 "staging buffers)");
  }
  Prec p = prec == PSMS_F64 ? P_F64 : P_F32;
  const size_t one = bytes_per_field(p, c->Vh) * size_t(nrhs);  // one batch of fields
  const size_t off = (one + 255) & ~size_t(255);                  // the output batch starts 256-aligned
  const size_t need = off + one;
  if (need > kNoAllocScratchBytes)
    throw Err{PSMS_EINVAL, "psms_apply_dw_noalloc: " + std::to_string(nrhs) + " fields need " + std::to_string(need) +
                               " bytes of scratch, more than its " + std::to_string(kNoAllocScratchBytes) +
                               "; pass fewer right-hand sides per call"};
  REQUIRE(c->noalloc_scratch != nullptr, "no scratch address for this device");
  Links L = links_of(c, &slot, 1, prec == PSMS_F64 ? LK_F64 : LK_F32C12);
  unsigned char* base = static_cast<unsigned char*>(c->noalloc_scratch);
  FieldBatch a{base, p, 1, nrhs}, b{base + off, p, 1, nrhs};
  // pack writes every unit of a and the full-lattice stencil every unit of b, so
  // nothing left by an earlier call is read
  launch_pack(c->st, c->g, in, a);
  DslashParams dp = dslash_params(c, a, HOP_ALL, -1, 1.0, -c->geom.kappa, 0);
  launch_dslash(c->st, c->g, L.p, L.fmt, a, b, dp, p == P_F64 ? c->nr_f64 : c->nr_low);
  launch_unpack(c->st, c->g, b, out);
  HIPCHK(hipGetLastError());
  API_END(c)
  return PSMS_OK;
}

psms_status psms_apply_dhat_ee(psms_ctx* c, int slot, const double* in, double* out, int nrhs) {
  API_BEGIN(c)
  check_rhs(nrhs);
  size_t nd = size_t(nrhs) * c->V * 24;
  const double* din = stage_in(c, in, nd, "stage_in");
  double* dout = stage_out(c, out, nd, "stage_out");
  Links L = links_of(c, &slot, 1, LK_F64);
  FieldBatch a = field(c, "api_a", P_F64, 1, nrhs), b = field(c, "api_b", P_F64, 1, nrhs);
  launch_pack(c->st, c->g, din, a);
  // b_o = H_oe a_e (odd outputs read only even inputs), then
  // out_e = a_e - kappa^2 H_eo b_o, out_o = 0.
  FieldBatch o = field(c, "api_c", P_F64, 1, nrhs);
  launch_zero_parity(c->st, a, c->Vh, 1);
  DslashParams dp{HOP_ALL, 1, 1, 0, c->g.nblk, 0.0, 1.0, 0};
  launch_dslash(c->st, c->g, L.p, L.fmt, a, b, dp, 4);
  launch_zero(c->st, o, c->Vh);
  DslashParams de{HOP_ALL, 0, 1, 0, c->g.nblk, 0.0, -c->geom.kappa * c->geom.kappa, 0};
  launch_dslash(c->st, c->g, L.p, L.fmt, b, o, de, 4);
  launch_axpby(c->st, c->g, const_cx(c, "one", nrhs, 1, 0), a, nullptr, o, +1);
  b = o;
  launch_unpack(c->st, c->g, b, dout);
  finish_out(c, out, dout, nd);
  API_END(c)
  return PSMS_OK;
}

psms_status psms_apply_block(psms_ctx* c, int slot, int colour, const double* in, double* out, int nrhs) {
  API_BEGIN(c)
  check_rhs(nrhs);
  REQUIRE(colour == 0 || colour == 1, "colour must be 0 (black) or 1 (white)");
  size_t nd = size_t(nrhs) * c->V * 24;
  const double* din = stage_in(c, in, nd, "stage_in");
  double* dout = stage_out(c, out, nd, "stage_out");
  Links L = links_of(c, &slot, 1, LK_F64);
  FieldBatch a = field(c, "api_a", P_F64, 1, nrhs), b = field(c, "api_b", P_F64, 1, nrhs);
  launch_pack(c->st, c->g, din, a);
  launch_keep_colour(c->st, c->g, a, colour);
  launch_zero(c->st, b, c->Vh);
  dslash(c, L, a, b, HOP_INTRA, colour, 1.0, -c->geom.kappa, 0);
  launch_unpack(c->st, c->g, b, dout);
  finish_out(c, out, dout, nd);
  API_END(c)
  return PSMS_OK;
}

psms_status psms_apply_hop_bw(psms_ctx* c, int slot, int from_colour, const double* in, double* out, int nrhs) {
  API_BEGIN(c)
  check_rhs(nrhs);
  REQUIRE(from_colour == 0 || from_colour == 1, "colour must be 0 (black) or 1 (white)");
  size_t nd = size_t(nrhs) * c->V * 24;
  const double* din = stage_in(c, in, nd, "stage_in");
  double* dout = stage_out(c, out, nd, "stage_out");
  Links L = links_of(c, &slot, 1, LK_F64);
  FieldBatch a = field(c, "api_a", P_F64, 1, nrhs), b = field(c, "api_b", P_F64, 1, nrhs);
  launch_pack(c->st, c->g, din, a);
  launch_keep_colour(c->st, c->g, a, from_colour);
  launch_zero(c->st, b, c->Vh);
  dslash(c, L, a, b, HOP_CROSS, 1 - from_colour, 0.0, -c->geom.kappa, 0);
  launch_unpack(c->st, c->g, b, dout);
  finish_out(c, out, dout, nd);
  API_END(c)
  return PSMS_OK;
}

psms_status psms_apply_proj(psms_ctx* c, const double* in, double* out, int nrhs) {
  API_BEGIN(c)
  check_rhs(nrhs);
  size_t nd = size_t(nrhs) * c->V * 24;
  const double* din = stage_in(c, in, nd, "stage_in");
  double* dout = stage_out(c, out, nd, "stage_out");
  FieldBatch a = field(c, "api_a", P_F64, 1, nrhs), b = field(c, "api_b", P_F64, 1, nrhs);
  launch_pack(c->st, c->g, din, a);
  launch_project(c->st, c->g, a, b);
  launch_unpack(c->st, c->g, b, dout);
  finish_out(c, out, dout, nd);
  API_END(c)
  return PSMS_OK;
}

static void fill_stats(psms_solve_stats* s, const FullSolveOut& o, double secs) {
  if (!s) return;
  s->converged = o.converged ? 1 : 0;
  s->outer_iters = o.outer;
  s->inner_iters = o.inner;
  s->used_fallback = o.used_fallback ? 1 : 0;
  s->true_rel_residual = o.max_rel;
  s->seconds = secs;
}

static void check_params(const psms_solve_params* p) {
  REQUIRE(p != nullptr, "null params");
  REQUIRE(p->tol > 0 && p->max_iter > 0 && p->restart >= 2, "tol > 0, max_iter > 0 and restart >= 2 required");
  REQUIRE(p->pc == PSMS_PC_NONE || p->pc == PSMS_PC_SAP || p->pc == PSMS_PC_NET, "unknown preconditioner");
  REQUIRE(p->pc == PSMS_PC_NONE || (p->sap_cycles >= 1 && p->block_iters >= 1), "SAP needs cycles >= 1 and block_iters >= 1");
}

psms_status psms_solve(psms_ctx* c, int slot, const double* b, double* x, int nrhs, const psms_solve_params* pp,
                       psms_solve_stats* stats) {
  API_BEGIN(c)
  check_rhs(nrhs);
  check_params(pp);
  auto t0 = std::chrono::steady_clock::now();
  size_t nd = size_t(nrhs) * c->V * 24;
  const double* db = stage_in(c, b, nd, "stage_in");
  double* dx = stage_out(c, x, nd, "stage_out");
  FieldBatch b64 = field(c, "api_b64", P_F64, 1, nrhs), x64 = field(c, "api_x64", P_F64, 1, nrhs);
  launch_pack(c->st, c->g, db, b64);
  FullSolveOut o = solve_full(c, &slot, pp, b64, x64);
  launch_unpack(c->st, c->g, x64, dx);
  finish_out(c, x, dx, nd);
  fill_stats(stats, o, std::chrono::duration<double>(std::chrono::steady_clock::now() - t0).count());
  if (o.nan) {
    c->err = "NaN/Inf in residual";
    return PSMS_ENAN;
  }
  if (!o.converged) {
    c->err = "solver did not reach tol (true relative residual " + std::to_string(o.max_rel) + ")";
    return PSMS_ENOTCONV;
  }
  API_END(c)
  return PSMS_OK;
}

psms_status psms_solve_block(psms_ctx* c, int slot, int colour, const double* b, double* x, int nrhs,
                             const psms_solve_params* pp, psms_solve_stats* stats) {
  API_BEGIN(c)
  check_rhs(nrhs);
  REQUIRE(pp != nullptr && pp->tol > 0 && pp->max_iter > 0, "bad params");
  REQUIRE(colour == 0 || colour == 1, "colour must be 0 or 1");
  auto t0 = std::chrono::steady_clock::now();
  size_t nd = size_t(nrhs) * c->V * 24;
  const double* db = stage_in(c, b, nd, "stage_in");
  double* dx = stage_out(c, x, nd, "stage_out");
  Links L = links_of(c, &slot, 1, LK_F64);
  FieldBatch b64 = field(c, "api_b64", P_F64, 1, nrhs), x64 = field(c, "api_x64", P_F64, 1, nrhs);
  launch_pack(c->st, c->g, db, b64);
  int iters = 0;
  double rel = solve_colour(c, &slot, colour, b64, x64, pp->tol, pp->max_iter, &iters, pp->prec == PSMS_MIXED);
  launch_unpack(c->st, c->g, x64, dx);
  finish_out(c, x, dx, nd);
  FullSolveOut o;
  o.inner = iters;
  o.outer = 1;
  o.max_rel = rel;
  o.converged = std::isfinite(rel) && rel <= pp->tol * 1.0001;
  fill_stats(stats, o, std::chrono::duration<double>(std::chrono::steady_clock::now() - t0).count());
  if (!std::isfinite(rel)) return PSMS_ENAN;
  if (!o.converged) {
    c->err = "block solve did not reach tol (relative residual " + std::to_string(rel) + ")";
    return PSMS_ENOTCONV;
  }
  API_END(c)
  return PSMS_OK;
}

psms_status psms_apply_schur(psms_ctx* c, int slot, const double* in, double* out, int nrhs, const psms_solve_params* pp,
                             psms_solve_stats* stats) {
  API_BEGIN(c)
  check_rhs(nrhs);
  REQUIRE(pp != nullptr && pp->tol > 0 && pp->max_iter > 0, "bad params");
  auto t0 = std::chrono::steady_clock::now();
  size_t nd = size_t(nrhs) * c->V * 24;
  const double* din = stage_in(c, in, nd, "stage_in");
  double* dout = stage_out(c, out, nd, "stage_out");
  Links L = links_of(c, &slot, 1, LK_F64);
  FieldBatch a = field(c, "api_a", P_F64, 1, nrhs), b = field(c, "api_b", P_F64, 1, nrhs);
  launch_pack(c->st, c->g, din, a);
  double rel = schur_apply(c, &slot, a, b, pp->tol, pp->max_iter, pp->prec == PSMS_MIXED);
  launch_unpack(c->st, c->g, b, dout);
  finish_out(c, out, dout, nd);
  FullSolveOut o;
  o.max_rel = rel;
  o.converged = rel <= pp->tol * 1.0001;
  fill_stats(stats, o, std::chrono::duration<double>(std::chrono::steady_clock::now() - t0).count());
  if (!o.converged) {
    c->err = "block solves inside the Schur complement did not reach tol";
    return PSMS_ENOTCONV;
  }
  API_END(c)
  return PSMS_OK;
}

psms_status psms_apply_schur_inv(psms_ctx* c, int slot, const double* in, double* out, int nrhs,
                                 const psms_solve_params* pp, psms_solve_stats* stats) {
  API_BEGIN(c)
  check_rhs(nrhs);
  check_params(pp);
  auto t0 = std::chrono::steady_clock::now();
  size_t nd = size_t(nrhs) * c->V * 24;
  const double* din = stage_in(c, in, nd, "stage_in");
  double* dout = stage_out(c, out, nd, "stage_out");
  FieldBatch a = field(c, "api_a", P_F64, 1, nrhs), b = field(c, "api_b", P_F64, 1, nrhs);
  launch_pack(c->st, c->g, din, a);
  FullSolveOut o = schur_inverse(c, &slot, pp, a, b);
  launch_unpack(c->st, c->g, b, dout);
  finish_out(c, out, dout, nd);
  fill_stats(stats, o, std::chrono::duration<double>(std::chrono::steady_clock::now() - t0).count());
  if (!o.converged) {
    c->err = "full solve inside the Schur inverse did not reach tol";
    return o.nan ? PSMS_ENAN : PSMS_ENOTCONV;
  }
  API_END(c)
  return PSMS_OK;
}

// One estimator step: hdelta[p*nnoise + j] = |M xi_j|^2 - |xi_j|^2 for the fields in
// slot_U and slot_Up[p] (eq. stacc, eq. Deltaistoch); solver outcomes go into agg.
// Outer (Dirichlet) block of each internal sub-block index, and the number of outer blocks.
static std::vector<int> outer_of_blocks(const psms_ctx* c, int* nouter) {
  const Geo& g = c->g;
  int NO[4];
  for (int m = 0; m < 4; ++m) NO[m] = g.L[m] / g.ob[m];
  *nouter = NO[0] * NO[1] * NO[2] * NO[3];
  std::vector<int> o(g.nblk);
  for (int lex = 0; lex < g.nblk; ++lex) {
    int B[4], r = lex;
    for (int m = 3; m >= 0; --m) {
      B[m] = r % g.NB[m];
      r /= g.NB[m];
    }
    const int col = (B[0] + B[1] + B[2] + B[3]) & 1;
    int O[4];
    for (int m = 0; m < 4; ++m) O[m] = B[m] * g.b[m] / g.ob[m];
    o[col * g.nblk_c + (lex >> 1)] = ((O[0] * NO[1] + O[1]) * NO[2] + O[2]) * NO[3] + O[3];
  }
  return o;
}

// With hblocks (a context with outer blocks): also hblocks[(p*nnoise + j)*nouter + B] =
// |(M xi_j)_B|^2 - |(xi_j)_B|^2 per outer block B, the sums over each outer block's
// sub-blocks taken in a fixed order.
static void logdet_core(psms_ctx* c, psms_op op, int slot_U, const int* slot_Up, int nprop, const double* noise, int nnoise,
                        const psms_solve_params* pp, std::vector<double>& hdelta, FullSolveOut& agg,
                        std::vector<double>* hblocks = nullptr) {
  const size_t fd = size_t(c->V) * 24;
  const double* dn = stage_in(c, noise, fd * nnoise, "stage_noise");
  hdelta.assign(size_t(nprop) * nnoise, 0.0);
  int nouter = 0;
  std::vector<int> outer_of;
  if (hblocks) {
    outer_of = outer_of_blocks(c, &nouter);
    hblocks->assign(size_t(nprop) * nnoise * nouter, 0.0);
  }
  const int nblk = c->g.nblk;
  Links LU = links_of(c, &slot_U, 1, LK_F64);
  // chunking: noise vectors per batch and proposals per batch
  int pchunk = std::min(nprop, MAXPROP);
  int jchunk = pp->rhs_chunk > 0 ? std::max(1, pp->rhs_chunk / pchunk) : nnoise;
  jchunk = std::min(jchunk, nnoise);
  for (int j0 = 0; j0 < nnoise; j0 += jchunk) {
    const int nj = std::min(jchunk, nnoise - j0);
    // xi_j (and phi_j for SCHUR), computed once with U and shared by all proposals
    FieldBatch eta = field(c, "ld_eta", P_F64, 1, nj);
    FieldBatch xi = field(c, "ld_xi", P_F64, 1, nj);
    FieldBatch phi = field(c, "ld_phi", P_F64, 1, nj);
    launch_pack(c->st, c->g, dn + size_t(j0) * fd, eta);
    double* xin2 = dscratch<double>(c, "ld_xin2", nj);
    // SCHUR: the full solve inside (1 - PQ(U'))^-1 starts from the solution of the same
    // system with U, which (1 - PQ(U)) xi yields as a by-product
    FieldBatch z0 = field(c, "ld_z0", P_F64, 1, nj);
    if (op == PSMS_OP_SCHUR) {
      launch_project(c->st, c->g, eta, xi);
      double rel = schur_apply(c, &slot_U, xi, phi, pp->tol, pp->max_iter, pp->prec == PSMS_MIXED, &z0);
      if (!(rel <= pp->tol * 1.0001)) agg.converged = false;
    } else {
      launch_copy(c->st, c->g, eta, xi, nullptr);
      apply_D(c, LU, xi, phi);
    }
    norm2(c, xi, xin2);
    std::vector<double> hx;  // fetched with the first chunk's |y|^2
    for (int p0 = 0; p0 < nprop; p0 += pchunk) {
      const int npp = std::min(pchunk, nprop - p0);
      FieldBatch rhs = field(c, "ld_rhs", P_F64, npp, nj);
      FieldBatch y = field(c, "ld_y", P_F64, npp, nj);
      const size_t fb = bytes_per_field(P_F64, c->Vh) * nj;
      for (int p = 0; p < npp; ++p)
        HIPCHK(hipMemcpyAsync((char*)rhs.p + p * fb, phi.p, fb, hipMemcpyDeviceToDevice, c->st));
      FullSolveOut o;
      if (op == PSMS_OP_SCHUR) {
        FieldBatch z0p = field(c, "ld_z0p", P_F64, npp, nj);
        for (int p = 0; p < npp; ++p)
          HIPCHK(hipMemcpyAsync((char*)z0p.p + p * fb, z0.p, fb, hipMemcpyDeviceToDevice, c->st));
        o = schur_inverse(c, slot_Up + p0, pp, rhs, y, &z0p);
      } else {
        o = solve_full(c, slot_Up + p0, pp, rhs, y);
      }
      agg.outer += o.outer;
      agg.inner += o.inner;
      agg.max_rel = std::max(agg.max_rel, o.max_rel);
      agg.nan |= o.nan;
      agg.converged &= o.converged;
      agg.used_fallback |= o.used_fallback;
      double* yn2 = dscratch<double>(c, "ld_yn2", size_t(npp) * nj);
      norm2(c, y, yn2);
      std::vector<double> hy;
      if (hx.empty()) {
        to_host2(c, xin2, nj, hx, yn2, npp * nj, hy);
      } else {
        hy = to_host(c, yn2, npp * nj);
      }
      for (int p = 0; p < npp; ++p)
        for (int j = 0; j < nj; ++j) hdelta[size_t(p0 + p) * nnoise + j0 + j] = hy[size_t(p) * nj + j] - hx[j];
      if (hblocks) {
        double* by = dscratch<double>(c, "ld_by", size_t(npp) * nj * nblk);
        double* bx = dscratch<double>(c, "ld_bx", size_t(nj) * nblk);
        launch_block_norm2(c->st, c->g, y, by);
        launch_block_norm2(c->st, c->g, xi, bx);
        std::vector<double> hby, hbx;
        to_host2(c, by, npp * nj * nblk, hby, bx, nj * nblk, hbx);
        for (int p = 0; p < npp; ++p)
          for (int j = 0; j < nj; ++j) {
            double* o = &(*hblocks)[(size_t(p0 + p) * nnoise + j0 + j) * nouter];
            for (int k = 0; k < nblk; ++k)
              o[outer_of[k]] += hby[(size_t(p) * nj + j) * nblk + k] - hbx[size_t(j) * nblk + k];
          }
      }
    }
  }
}

// The field U_i of eq. gfparam (g = 1) for the fields in slots s0 and s1, into slot dst:
// FP64 links only (not SU(3) in general), in every layout the context holds.
static void interp_slot(psms_ctx* c, int dst, int s0, int s1, int N, int i) {
  Slot& d = c->slots[dst];
  const Slot& a = c->slots[s0];
  const Slot& b = c->slots[s1];
  const size_t n = size_t(c->V) * 4 * 18;  // doubles of one FP64 link field
  const double wa = double(N - i) / N, wb = double(i) / N;
  if (!d.f64) d.f64 = dev_alloc(c, n * sizeof(double));
  launch_lerp(c->st, (const double*)a.f64, (const double*)b.f64, wa, wb, (double*)d.f64, n);
  if (c->split) {
    if (!d.f64_s) d.f64_s = dev_alloc(c, n * sizeof(double));
    launch_lerp(c->st, (const double*)a.f64_s, (const double*)b.f64_s, wa, wb, (double*)d.f64_s, n);
  }
  d.loaded = true;
  d.su3 = false;
  if (d.f18) build_f18(c, d);  // FP32 copies made for an earlier field of this slot
}

psms_status psms_logdet_ratio(psms_ctx* c, psms_op op, int slot_U, const int* slot_Up, int nprop, const double* noise,
                              int nnoise, int n_interp, const psms_solve_params* pp, double* delta, psms_solve_stats* stats) {
  API_BEGIN(c)
  check_params(pp);
  REQUIRE(op == PSMS_OP_FULL || op == PSMS_OP_SCHUR, "unknown operator");
  REQUIRE(n_interp >= 1 && n_interp <= 1024, "n_interp must be in [1, 1024]");
  REQUIRE(nprop >= 1 && nnoise >= 1 && slot_Up && noise && delta, "bad sizes or null pointers");
  REQUIRE(slot_U >= 0 && slot_U < 64 && c->slots[slot_U].loaded, "gauge slot not loaded");
  for (int p = 0; p < nprop; ++p)
    REQUIRE(slot_Up[p] >= 0 && slot_Up[p] < 64 && c->slots[slot_Up[p]].loaded, "gauge slot not loaded");
  auto t0 = std::chrono::steady_clock::now();
  std::vector<double> hdelta;
  FullSolveOut agg;
  agg.converged = true;
  if (n_interp == 1) {
    logdet_core(c, op, slot_U, slot_Up, nprop, noise, nnoise, pp, hdelta, agg);
  } else {
    // eq. staccN: per proposal, the sum over the N factors M_i = D(U_{i+1})^-1 D(U_i) of
    // eq. Mparam, factor i with noise fields i*nnoise .. (i+1)*nnoise - 1; the
    // intermediate fields go into two free slots, released afterwards
    int fr[2] = {-1, -1};
    for (int k = 63, n = 0; k >= 0 && n < 2; --k)
      if (!c->slots[k].loaded) fr[n++] = k;
    REQUIRE(fr[1] >= 0, "n_interp > 1 needs two free gauge slots");
    struct Release {
      psms_ctx* c;
      int a, b;
      ~Release() { c->slots[a].loaded = c->slots[b].loaded = false; }
    } release{c, fr[0], fr[1]};
    const size_t fd = size_t(c->V) * 24;
    hdelta.assign(size_t(nprop) * nnoise, 0.0);
    std::vector<double> step;
    for (int p = 0; p < nprop; ++p)
      for (int i = 0; i < n_interp; ++i) {
        const int a = i == 0 ? slot_U : fr[0];
        const int b = i + 1 == n_interp ? slot_Up[p] : fr[1];
        if (i > 0) interp_slot(c, fr[0], slot_U, slot_Up[p], n_interp, i);
        if (i + 1 < n_interp) interp_slot(c, fr[1], slot_U, slot_Up[p], n_interp, i + 1);
        logdet_core(c, op, a, &b, 1, noise + size_t(i) * nnoise * fd, nnoise, pp, step, agg);
        for (int j = 0; j < nnoise; ++j) hdelta[size_t(p) * nnoise + j] += step[j];
      }
  }
  if (is_device_ptr(delta)) {
    HIPCHK(hipMemcpyAsync(delta, hdelta.data(), hdelta.size() * sizeof(double), hipMemcpyHostToDevice, c->st));
    HIPCHK(hipStreamSynchronize(c->st));
  } else {
    std::memcpy(delta, hdelta.data(), hdelta.size() * sizeof(double));
  }
  fill_stats(stats, agg, std::chrono::duration<double>(std::chrono::steady_clock::now() - t0).count());
  if (agg.nan) return PSMS_ENAN;
  if (!agg.converged) {
    c->err = "a solve inside the estimator did not reach tol";
    return PSMS_ENOTCONV;
  }
  API_END(c)
  return PSMS_OK;
}

psms_status psms_block_logdet(psms_ctx* c, const int* slots, int nslot, double* out) {
  API_BEGIN(c)
  REQUIRE(slots && out && nslot >= 1, "null argument or no gauge slot");
  const Geo& g = c->g;
  const int n = 12 * g.Vbh;  // even sites of a block x 12
  const int npad = (n + 63) / 64 * 64;
  REQUIRE(n <= 6144, "exact block determinants take blocks of at most 1024 sites (the dense even-odd reduced "
                     "operator has 6 V_b rows); factorise larger blocks by their Schur complement");
  const size_t mat_doubles = size_t(2) * npad * npad;
  const int per_batch = int(std::max<size_t>(1, std::min<size_t>(g.nblk, (size_t(16) << 30) / (8 * mat_doubles))));
  double* M = dscratch<double>(c, "lu_M", mat_doubles * per_batch);
  double2* dld = dscratch<double2>(c, "lu_logdet", per_batch);
  double* dmp = dscratch<double>(c, "lu_minpiv", per_batch);
  double* inv = dscratch<double>(c, "lu_inv", size_t(4) * 64 * 64 * per_batch);
  const int nc = std::min(n, 96);  // columns assembled per pass
  FieldBatch e = field(c, "lu_e", P_F64, 1, nc), tb = field(c, "lu_t", P_F64, 1, nc), y = field(c, "lu_y", P_F64, 1, nc);
  // internal block index of each lexicographic block (black blocks first, eq. domdec)
  std::vector<int> lex_of(g.nblk);
  for (int lex = 0; lex < g.nblk; ++lex) {
    int B[4], r = lex;
    for (int m = 3; m >= 0; --m) {
      B[m] = r % g.NB[m];
      r /= g.NB[m];
    }
    const int col = (B[0] + B[1] + B[2] + B[3]) & 1;
    lex_of[col * g.nblk_c + (lex >> 1)] = lex;
  }
  const double k2 = c->geom.kappa * c->geom.kappa;
  std::vector<double2> zero_ld(per_batch, make_double2(0.0, 0.0));
  std::vector<double> big_mp(per_batch, 1e300);
  std::vector<double> res(size_t(nslot) * g.nblk * 2);
  for (int si = 0; si < nslot; ++si) {
    Links L = links_of(c, &slots[si], 1, LK_F64);
    for (int b0 = 0; b0 < g.nblk; b0 += per_batch) {
      const int nb = std::min(per_batch, g.nblk - b0);
      launch_lu_init(c->st, M, n, npad, nb);
      for (int k0 = 0; k0 < n; k0 += nc) {
        const int nr = std::min(nc, n - k0);
        FieldBatch ee{e.p, P_F64, 1, nr}, tt{tb.p, P_F64, 1, nr}, yy{y.p, P_F64, 1, nr};
        launch_zero(c->st, ee, c->Vh);
        launch_zero(c->st, tt, c->Vh);  // its even half is read (times zero) by the second hop
        launch_lu_units(c->st, g, (double2*)ee.p, k0, nr, n);
        // t_odd = H_oe e, then y_even = -kappa^2 H_eo t: hops inside the blocks only
        DslashParams d1{HOP_INTRA, 1, 1, 0, g.nblk, 0.0, 1.0, 0};
        launch_dslash(c->st, g, L.p, L.fmt, ee, tt, d1, 1);
        DslashParams d2{HOP_INTRA, 0, 1, 0, g.nblk, 0.0, -k2, 0};
        launch_dslash(c->st, g, L.p, L.fmt, tt, yy, d2, 1);
        launch_lu_scatter(c->st, g, (const double2*)yy.p, M, k0, nr, n, npad, b0, nb);
      }
      HIPCHK(hipMemcpyAsync(dld, zero_ld.data(), sizeof(double2) * nb, hipMemcpyHostToDevice, c->st));
      HIPCHK(hipMemcpyAsync(dmp, big_mp.data(), sizeof(double) * nb, hipMemcpyHostToDevice, c->st));
      launch_lu_factor(c->st, M, npad, nb, dld, dmp, inv);
      HIPCHK(hipGetLastError());
      std::vector<double2> hld(nb);
      std::vector<double> hmp(nb);
      HIPCHK(hipMemcpyAsync(hld.data(), dld, sizeof(double2) * nb, hipMemcpyDeviceToHost, c->st));
      HIPCHK(hipMemcpyAsync(hmp.data(), dmp, sizeof(double) * nb, hipMemcpyDeviceToHost, c->st));
      HIPCHK(hipStreamSynchronize(c->st));
      for (int k = 0; k < nb; ++k) {
        if (!(hmp[k] >= 1e-8) || !std::isfinite(hld[k].x))
          throw Err{PSMS_ENOTCONV, "block LU met a pivot of modulus " + std::to_string(hmp[k]) + " in block " +
                                       std::to_string(lex_of[b0 + k]) + " (no exchanges are made; result refused)"};
        double* o = &res[(size_t(si) * g.nblk + lex_of[b0 + k]) * 2];
        o[0] = hld[k].x;
        o[1] = std::remainder(hld[k].y, 2.0 * M_PI);
      }
    }
  }
  if (is_device_ptr(out)) {
    HIPCHK(hipMemcpyAsync(out, res.data(), res.size() * sizeof(double), hipMemcpyHostToDevice, c->st));
    HIPCHK(hipStreamSynchronize(c->st));
  } else {
    std::memcpy(out, res.data(), res.size() * sizeof(double));
  }
  API_END(c)
  return PSMS_OK;
}

psms_status psms_logdet_ratio_blocks(psms_ctx* c, int slot_U, const int* slot_Up, int nprop, const double* noise,
                                     int nnoise, const psms_solve_params* pp, double* delta, psms_solve_stats* stats) {
  API_BEGIN(c)
  check_params(pp);
  REQUIRE(c->g.ob[0] > 0, "psms_logdet_ratio_blocks needs a context with outer blocks (geom.outer_b)");
  REQUIRE(nprop >= 1 && nnoise >= 1 && slot_Up && noise && delta, "bad sizes or null pointers");
  REQUIRE(slot_U >= 0 && slot_U < 64 && c->slots[slot_U].loaded, "gauge slot not loaded");
  for (int p = 0; p < nprop; ++p)
    REQUIRE(slot_Up[p] >= 0 && slot_Up[p] < 64 && c->slots[slot_Up[p]].loaded, "gauge slot not loaded");
  auto t0 = std::chrono::steady_clock::now();
  std::vector<double> hdelta, hblocks;
  FullSolveOut agg;
  agg.converged = true;
  logdet_core(c, PSMS_OP_SCHUR, slot_U, slot_Up, nprop, noise, nnoise, pp, hdelta, agg, &hblocks);
  if (is_device_ptr(delta)) {
    HIPCHK(hipMemcpyAsync(delta, hblocks.data(), hblocks.size() * sizeof(double), hipMemcpyHostToDevice, c->st));
    HIPCHK(hipStreamSynchronize(c->st));
  } else {
    std::memcpy(delta, hblocks.data(), hblocks.size() * sizeof(double));
  }
  fill_stats(stats, agg, std::chrono::duration<double>(std::chrono::steady_clock::now() - t0).count());
  if (agg.nan) return PSMS_ENAN;
  if (!agg.converged) {
    c->err = "a solve inside the estimator did not reach tol";
    return PSMS_ENOTCONV;
  }
  API_END(c)
  return PSMS_OK;
}

void psms_default_filter_params(psms_filter_params* p) {
  if (!p) return;
  p->beta[0] = 1.0;
  p->beta[1] = 0.0;
  p->beta[2] = 0.0;
  psms_default_params(&p->solve);
  p->work_slot[0] = 62;
  p->work_slot[1] = 63;
  p->slot_out = -1;
}

psms_status psms_filter_step(psms_ctx* in, psms_ctx* out, int slot_U, int slot_Up, const psms_filter_params* fp,
                             const double* uniforms, const double* noise, psms_filter_result* res) {
  if (!in || !out) return PSMS_EINVAL;
  API_BEGIN(out)
  REQUIRE(fp && uniforms && noise && res, "null argument");
  const Geo& gi = in->g;
  const Geo& go = out->g;
  REQUIRE(gi.ob[0] > 0 && !go.ob[0], "the first context needs outer blocks, the second none");
  for (int m = 0; m < 4; ++m) {
    REQUIRE(gi.L[m] == go.L[m], "the two contexts must share the lattice");
    REQUIRE(gi.ob[m] == go.b[m], "the outer blocks of the first context must be the blocks of the second");
  }
  REQUIRE(in->geom.kappa == out->geom.kappa && in->geom.antiperiodic_t == out->geom.antiperiodic_t &&
              in->device == out->device && in->st == out->st,
          "the two contexts must share kappa, boundary conditions, device and stream");
  REQUIRE(std::fabs(fp->beta[0] + fp->beta[1] + fp->beta[2] - 1.0) < 1e-12,
          "the beta coefficients of the block-determinant action must sum to 1 (App. C)");
  const int w1 = fp->work_slot[0], w2 = fp->work_slot[1];
  for (int sl : {slot_U, slot_Up, w1, w2}) REQUIRE(sl >= 0 && sl < 64, "slot out of range");
  REQUIRE(w1 != w2 && w1 != slot_U && w1 != slot_Up && w2 != slot_U && w2 != slot_Up, "work slots must be free");
  for (psms_ctx* c : {in, out})
    REQUIRE(c->slots[slot_U].loaded && c->slots[slot_Up].loaded, "U and U' must be loaded in both contexts");
  const int nsmall = gi.nblk, nouter = go.nblk;
  // lexicographic outer block of each lexicographic small block
  std::vector<int> small_outer(nsmall);
  for (int lex = 0; lex < nsmall; ++lex) {
    int B[4], r = lex, O[4];
    for (int m = 3; m >= 0; --m) {
      B[m] = r % gi.NB[m];
      r /= gi.NB[m];
    }
    for (int m = 0; m < 4; ++m) O[m] = B[m] * gi.b[m] / gi.ob[m];
    small_outer[lex] = ((O[0] * go.NB[1] + O[1]) * go.NB[2] + O[2]) * go.NB[3] + O[3];
  }
  const double* u1 = uniforms;
  const double* u2 = uniforms + nsmall;
  const double u3 = uniforms[nsmall + nouter];
  // step 1: exact block filter on the smallest blocks
  std::vector<double> ld(size_t(2) * nsmall * 2);
  const int pair[2] = {slot_U, slot_Up};
  psms_status s = psms_block_logdet(in, pair, 2, ld.data());
  if (s != PSMS_OK) {
    out->err = std::string("block filter: ") + in->err;
    return s;
  }
  std::vector<double> dS1(nsmall);
  std::vector<int> a1(nsmall);
  for (int k = 0; k < nsmall; ++k) {
    dS1[k] = -2.0 * (ld[(size_t(nsmall) + k) * 2] - ld[size_t(k) * 2]);
    const double d = fp->beta[0] * dS1[k];
    a1[k] = u1[k] < std::exp(-d) ? 1 : 0;
    if (res->delta1) res->delta1[k] = d;
    if (res->accept1) res->accept1[k] = a1[k];
  }
  // the fields in the boundary layout (from the context without outer blocks: uncut links)
  const size_t nl = size_t(out->V) * 4 * 18;
  double* U = dscratch<double>(out, "flt_U", nl);
  double* Up = dscratch<double>(out, "flt_Up", nl);
  double* U1 = dscratch<double>(out, "flt_U1", nl);
  double* U2 = dscratch<double>(out, "flt_U2", nl);
  int* acc = dscratch<int>(out, "flt_acc", std::max(nsmall, nouter));
  const int np = gf_partials(go);
  double* part = dscratch<double>(out, "flt_part", np);
  launch_gf_unpack(out->st, go, out->slots[slot_U].f64, U);
  launch_gf_unpack(out->st, go, out->slots[slot_Up].f64, Up);
  launch_change_across(out->st, go, gi.b, U, Up, part);
  {
    std::vector<double> h = to_host(out, part, np);
    double m = 0.0;
    for (double v : h) m = (v > m || v != v) ? v : m;
    REQUIRE(m == 0.0, "the proposal changes links between the smallest blocks (the block filters would not decouple)");
  }
  HIPCHK(hipMemcpyAsync(acc, a1.data(), sizeof(int) * nsmall, hipMemcpyHostToDevice, out->st));
  launch_merge_links(out->st, go, gi.b, acc, U, Up, U1);
  HIPCHK(hipStreamSynchronize(out->st));  // a1 is read by the merge before it goes out of use
  s = load_links(in, w1, U1);
  if (s != PSMS_OK && s != PSMS_ENOTSU3) return s;
  s = load_links(out, w1, U1);
  if (s != PSMS_OK && s != PSMS_ENOTSU3) return s;
  // step 2: block-Schur filter per outer block, one noise field
  std::vector<double> dS2(nouter);
  psms_solve_stats st2{}, st3{};
  s = psms_logdet_ratio_blocks(in, slot_U, &w1, 1, noise, 1, &fp->solve, dS2.data(), &st2);
  if (s != PSMS_OK) {
    out->err = std::string("block-Schur filter: ") + in->err;
    return s;
  }
  std::vector<double> blk_sum(nouter, 0.0);
  for (int k = 0; k < nsmall; ++k)
    if (a1[k]) blk_sum[small_outer[k]] += dS1[k];
  std::vector<int> a2(nouter);
  for (int b = 0; b < nouter; ++b) {
    const double d = dS2[b] + fp->beta[1] * blk_sum[b];
    a2[b] = u2[b] < std::exp(-d) ? 1 : 0;
    if (res->delta2) res->delta2[b] = d;
    if (res->accept2) res->accept2[b] = a2[b];
  }
  HIPCHK(hipMemcpyAsync(acc, a2.data(), sizeof(int) * nouter, hipMemcpyHostToDevice, out->st));
  launch_merge_links(out->st, go, go.b, acc, U, U1, U2);
  HIPCHK(hipStreamSynchronize(out->st));
  s = load_links(out, w2, U2);
  if (s != PSMS_OK && s != PSMS_ENOTSU3) return s;
  // step 3: global Schur filter of the outer blocks' decomposition, one noise field
  double dS3 = 0.0;
  s = psms_logdet_ratio(out, PSMS_OP_SCHUR, slot_U, &w2, 1, noise + size_t(out->V) * 24, 1, 1, &fp->solve, &dS3, &st3);
  if (s != PSMS_OK) return s;
  double blk_all = 0.0;
  for (int k = 0; k < nsmall; ++k)
    if (a1[k] && a2[small_outer[k]]) blk_all += dS1[k];
  const double d3 = dS3 + fp->beta[2] * blk_all;
  const int a3 = u3 < std::exp(-d3) ? 1 : 0;
  res->delta3 = d3;
  res->accept3 = a3;
  res->inner_iters = st2.inner_iters + st3.inner_iters;
  if (fp->slot_out >= 0) {
    REQUIRE(fp->slot_out < 64, "slot_out out of range");
    const double* fin = a3 ? U2 : U;
    s = load_links(in, fp->slot_out, fin);
    if (s != PSMS_OK && s != PSMS_ENOTSU3) return s;
    s = load_links(out, fp->slot_out, fin);
    if (s != PSMS_OK && s != PSMS_ENOTSU3) return s;
  }
  HIPCHK(hipStreamSynchronize(out->st));
  API_END(out)
  return PSMS_OK;
}

psms_status psms_log_ratio_estimate(const double* delta, int nprop, int nnoise, double* out) {
  if (!delta || !out || nprop < 1 || nnoise < 1) return PSMS_EINVAL;
  for (size_t i = 0; i < size_t(nprop) * nnoise; ++i)
    if (!std::isfinite(delta[i])) return PSMS_EINVAL;
  for (int p = 0; p < nprop; ++p) {
    const double* d = delta + size_t(p) * nnoise;
    double top = -d[0];
    for (int j = 1; j < nnoise; ++j) top = std::max(top, -d[j]);
    double sum = 0.0;
    for (int j = 0; j < nnoise; ++j) sum += std::exp(-d[j] - top);
    out[p] = top + std::log(sum / nnoise);
  }
  return PSMS_OK;
}

psms_status psms_net_init(psms_ctx* c, const int* channels, int nlayers, unsigned long long seed, double scale) {
  API_BEGIN(c)
  REQUIRE(channels != nullptr && nlayers >= 1 && nlayers <= 16, "bad network shape");
  std::vector<int> ch(channels, channels + nlayers + 1);
  net_alloc(c, ch);
  // small random weights plus the identity on the (t = 0, channel 0 -> 0) path, so
  // that the untrained network starts close to N(r) = r
  std::mt19937_64 rng(seed);
  std::normal_distribution<double> nd(0.0, 1.0);
  std::vector<float> w(c->net.nw * 2);
  for (int l = 0; l < c->net.nlayers; ++l) {
    const int cin = ch[l], cout = ch[l + 1];
    const double sd = scale / std::sqrt(9.0 * 4.0 * cin);
    const size_t o = c->net.woff[l];
    for (size_t k = 0; k < net_layer_size(cin, cout); ++k) {
      w[2 * (o + k)] = float(sd * nd(rng));
      w[2 * (o + k) + 1] = float(sd * nd(rng));
    }
    for (int s = 0; s < 4; ++s) w[2 * (o + s * 4 + s)] += 1.0f;  // t = 0, co = 0, ci = 0
  }
  HIPCHK(hipMemcpy(c->net.w, w.data(), w.size() * sizeof(float), hipMemcpyHostToDevice));
  c->net.packed = false;
  API_END(c)
  return PSMS_OK;
}

long long psms_net_num_weights(const psms_ctx* c) { return c ? (long long)c->net.nw : 0; }

psms_status psms_net_set_weights(psms_ctx* c, const double* w, long long n) {
  API_BEGIN(c)
  REQUIRE(c->net.nlayers > 0, "no network");
  REQUIRE(w != nullptr && n == (long long)c->net.nw, "weight count must equal psms_net_num_weights");
  std::vector<float> f(2 * n);
  for (long long i = 0; i < 2 * n; ++i) f[i] = float(w[i]);
  HIPCHK(hipMemcpy(c->net.w, f.data(), f.size() * sizeof(float), hipMemcpyHostToDevice));
  c->net.packed = false;
  API_END(c)
  return PSMS_OK;
}

psms_status psms_net_get_weights(psms_ctx* c, double* w, long long n) {
  API_BEGIN(c)
  REQUIRE(c->net.nlayers > 0, "no network");
  REQUIRE(w != nullptr && n == (long long)c->net.nw, "weight count must equal psms_net_num_weights");
  std::vector<float> f(2 * n);
  HIPCHK(hipStreamSynchronize(c->st));
  HIPCHK(hipMemcpy(f.data(), c->net.w, f.size() * sizeof(float), hipMemcpyDeviceToHost));
  for (long long i = 0; i < 2 * n; ++i) w[i] = f[i];
  API_END(c)
  return PSMS_OK;
}

psms_status psms_net_apply(psms_ctx* c, int slot, const double* in, double* out, int nrhs) {
  API_BEGIN(c)
  check_rhs(nrhs);
  REQUIRE(c->net.nlayers > 0, "no network");
  size_t nd = size_t(nrhs) * c->V * 24;
  const double* din = stage_in(c, in, nd, "stage_in");
  double* dout = stage_out(c, out, nd, "stage_out");
  Links L = links_of(c, &slot, 1, LK_F32C12);
  FieldBatch a = field(c, "api_a32", P_F32, 1, nrhs), b = field(c, "api_b32", P_F32, 1, nrhs);
  launch_pack(c->st, c->g, din, a);
  net_forward(c, L.p[0], a.p, nrhs, b.p, nullptr);
  launch_unpack(c->st, c->g, b, dout);
  finish_out(c, out, dout, nd);
  API_END(c)
  return PSMS_OK;
}

psms_status psms_net_loss_grad(psms_ctx* c, int slot, const double* r, const double* e, int npairs, double* loss,
                               double* grad) {
  API_BEGIN(c)
  check_rhs(npairs);
  REQUIRE(c->net.nlayers > 0, "no network");
  REQUIRE(loss != nullptr, "null loss");
  size_t nd = size_t(npairs) * c->V * 24;
  const double* dr = stage_in(c, r, nd, "stage_in");
  const double* de = stage_in(c, e, nd, "stage_in2");
  Links L = links_of(c, &slot, 1, LK_F32C12);
  FieldBatch r32 = field(c, "api_a32", P_F32, 1, npairs), e32 = field(c, "api_b32", P_F32, 1, npairs);
  FieldBatch e64 = field(c, "api_e64", P_F64, 1, npairs);
  launch_pack(c->st, c->g, dr, r32);
  launch_pack(c->st, c->g, de, e32);
  launch_pack(c->st, c->g, de, e64);
  double* en = dscratch<double>(c, "api_en", npairs);
  norm2(c, e64, en);
  std::vector<double> hen = to_host(c, en, npairs);
  *loss = net_loss_grad(c, L.p[0], r32, e32, hen.data(), npairs, false);
  if (grad) {
    HIPCHK(hipStreamSynchronize(c->st));
    HIPCHK(hipMemcpy(grad, c->net.grad, c->net.nw * 2 * sizeof(double), hipMemcpyDeviceToHost));
  }
  API_END(c)
  return PSMS_OK;
}

void psms_default_train_params(psms_train_params* p) {
  if (!p) return;
  p->npairs = 256;
  p->batch = 8;
  p->epochs = 2;
  p->chunk = 64;
  p->lr = 2e-3;
  p->solve_tol = 1e-6;
  p->seed = 12345;
  p->ckpt_path = nullptr;
  p->ckpt_every = 0;
}

static void net_write(psms_ctx* c, const char* path) {
  auto& n = c->net;
  std::vector<float> w(2 * n.nw), m(2 * n.nw), v(2 * n.nw);
  HIPCHK(hipStreamSynchronize(c->st));
  HIPCHK(hipMemcpy(w.data(), n.w, w.size() * 4, hipMemcpyDeviceToHost));
  HIPCHK(hipMemcpy(m.data(), n.m, m.size() * 4, hipMemcpyDeviceToHost));
  HIPCHK(hipMemcpy(v.data(), n.v, v.size() * 4, hipMemcpyDeviceToHost));
  std::string tmp = std::string(path) + ".tmp";
  FILE* f = std::fopen(tmp.c_str(), "wb");
  REQUIRE(f != nullptr, std::string("cannot write ") + path);
  int32_t hdr[2] = {n.nlayers, n.adam_step};
  std::fwrite("PSMSNET1", 1, 8, f);
  std::fwrite(hdr, 4, 2, f);
  std::fwrite(n.ch.data(), 4, n.ch.size(), f);
  std::fwrite(w.data(), 4, w.size(), f);
  std::fwrite(m.data(), 4, m.size(), f);
  std::fwrite(v.data(), 4, v.size(), f);
  bool ok = std::fclose(f) == 0;
  REQUIRE(ok && std::rename(tmp.c_str(), path) == 0, std::string("cannot write ") + path);
}

psms_status psms_net_save(psms_ctx* c, const char* path) {
  API_BEGIN(c)
  REQUIRE(c->net.nlayers > 0 && path != nullptr, "no network or null path");
  net_write(c, path);
  API_END(c)
  return PSMS_OK;
}

psms_status psms_net_load(psms_ctx* c, const char* path) {
  API_BEGIN(c)
  REQUIRE(path != nullptr, "null path");
  FILE* f = std::fopen(path, "rb");
  REQUIRE(f != nullptr, std::string("cannot open ") + path);
  char magic[8];
  int32_t hdr[2];
  bool ok = std::fread(magic, 1, 8, f) == 8 && std::memcmp(magic, "PSMSNET1", 8) == 0 && std::fread(hdr, 4, 2, f) == 2 &&
            hdr[0] >= 1 && hdr[0] <= 16;
  std::vector<int32_t> ch(ok ? hdr[0] + 1 : 0);
  ok = ok && std::fread(ch.data(), 4, ch.size(), f) == ch.size();
  if (!ok) {
    std::fclose(f);
    throw Err{PSMS_EINVAL, std::string("not a network checkpoint: ") + path};
  }
  net_alloc(c, std::vector<int>(ch.begin(), ch.end()));
  auto& n = c->net;
  std::vector<float> w(2 * n.nw), m(2 * n.nw), v(2 * n.nw);
  ok = std::fread(w.data(), 4, w.size(), f) == w.size() && std::fread(m.data(), 4, m.size(), f) == m.size() &&
       std::fread(v.data(), 4, v.size(), f) == v.size();
  std::fclose(f);
  REQUIRE(ok, std::string("truncated network checkpoint: ") + path);
  HIPCHK(hipMemcpy(n.w, w.data(), w.size() * 4, hipMemcpyHostToDevice));
  HIPCHK(hipMemcpy(n.m, m.data(), m.size() * 4, hipMemcpyHostToDevice));
  HIPCHK(hipMemcpy(n.v, v.data(), v.size() * 4, hipMemcpyHostToDevice));
  n.adam_step = hdr[1];
  n.packed = false;
  API_END(c)
  return PSMS_OK;
}

psms_status psms_net_train(psms_ctx* c, const int* slots, int nconf, const psms_train_params* tp, psms_train_stats* ts) {
  API_BEGIN(c)
  REQUIRE(c->net.nlayers > 0, "no network (psms_net_init or psms_net_load first)");
  REQUIRE(slots != nullptr && nconf >= 1 && tp != nullptr, "bad arguments");
  REQUIRE(tp->npairs >= 1 && tp->batch >= 1 && tp->chunk >= tp->batch && tp->epochs >= 1 && tp->lr > 0 &&
              tp->solve_tol > 0,
          "bad training parameters");
  auto t0 = std::chrono::steady_clock::now();
  double t_data = 0, t_train = 0, first = -1, last = 0;
  int steps = 0;
  const size_t fd = size_t(c->V) * 24;
  psms_solve_params sp;
  psms_default_params(&sp);
  sp.tol = tp->solve_tol;
  sp.prec = PSMS_MIXED;
  sp.pc = PSMS_PC_SAP;
  for (int k = 0, p0 = 0; p0 < tp->npairs; ++k, p0 += tp->chunk) {
    const int nc = std::min(tp->chunk, tp->npairs - p0);
    const int conf = slots[k % nconf];
    auto ta = std::chrono::steady_clock::now();
    // residual / correction pairs: Gaussian r, e = D^-1 r from the plain solver
    double* rb = dscratch<double>(c, "tr_rb", fd * nc);
    launch_gaussian(c->st, rb, fd / 2, nc, tp->seed, uint32_t(k));
    FieldBatch b64 = field(c, "tr_b64", P_F64, 1, nc), x64 = field(c, "tr_x64", P_F64, 1, nc);
    launch_pack(c->st, c->g, rb, b64);
    FullSolveOut so = solve_full(c, &conf, &sp, b64, x64);
    REQUIRE(!so.nan, "NaN while generating training pairs");
    FieldBatch r32 = field(c, "tr_r32", P_F32, 1, nc), e32 = field(c, "tr_e32", P_F32, 1, nc);
    launch_copy(c->st, c->g, b64, r32, nullptr);
    launch_copy(c->st, c->g, x64, e32, nullptr);
    double* en = dscratch<double>(c, "tr_en", nc);
    norm2(c, x64, en);
    std::vector<double> hen = to_host(c, en, nc);
    Links L = links_of(c, &conf, 1, LK_F32C12);
    auto tb = std::chrono::steady_clock::now();
    t_data += std::chrono::duration<double>(tb - ta).count();
    const size_t fb = bytes_per_field(P_F32, c->Vh);
    for (int ep = 0; ep < tp->epochs; ++ep) {
      for (int b0 = 0; b0 < nc; b0 += tp->batch) {
        const int nb = std::min(tp->batch, nc - b0);
        FieldBatch rb32{(char*)r32.p + b0 * fb, P_F32, 1, nb}, eb32{(char*)e32.p + b0 * fb, P_F32, 1, nb};
        double loss = net_loss_grad(c, L.p[0], rb32, eb32, hen.data() + b0, nb, true);
        {
          ProfScope ps(c, FAM_NET, 0);
          launch_adam(c->st, c->net.w, c->net.grad, c->net.m, c->net.v, int(2 * c->net.nw), float(tp->lr), 0.9f, 0.999f,
                      1e-8f, ++c->net.adam_step);
          c->net.packed = false;
        }
        if (first < 0) first = loss;
        last = loss;
        ++steps;
        if (tp->ckpt_path && tp->ckpt_every > 0 && steps % tp->ckpt_every == 0) net_write(c, tp->ckpt_path);
      }
    }
    t_train += std::chrono::duration<double>(std::chrono::steady_clock::now() - tb).count();
  }
  if (tp->ckpt_path) net_write(c, tp->ckpt_path);
  HIPCHK(hipStreamSynchronize(c->st));
  if (ts) {
    ts->first_loss = first;
    ts->final_loss = last;
    ts->steps = steps;
    ts->seconds_data = t_data;
    ts->seconds_train = t_train;
  }
  (void)t0;
  API_END(c)
  return PSMS_OK;
}

static int* tuning_slot(psms_ctx* c, const char* key) {
  if (!std::strcmp(key, "dslash_variant_f64")) return &c->variant[P_F64];
  if (!std::strcmp(key, "dslash_variant_f32")) return &c->variant[P_F32];
  if (!std::strcmp(key, "dslash_variant_bf16")) return &c->variant[P_BF16];
  if (!std::strcmp(key, "nr_f64")) return &c->nr_f64;
  if (!std::strcmp(key, "nr_low")) return &c->nr_low;
  if (!std::strcmp(key, "xcd_map")) return &c->xcd_map;
  if (!std::strcmp(key, "net_mfma")) return &c->net_mfma;
  if (!std::strcmp(key, "block_solver")) return &c->block_solver;
  if (!std::strcmp(key, "block_lanes")) return &c->block_lanes;
  if (!std::strcmp(key, "block_eo")) return &c->block_eo;
  if (!std::strcmp(key, "block_eo_lanes")) return &c->block_eo_lanes;
  if (!std::strcmp(key, "block_tol_prec")) return &c->block_tol_prec;
  if (!std::strcmp(key, "sap_bf16")) return &c->sap_bf16;
  if (!std::strcmp(key, "block_xcd")) return &c->block_xcd;
  if (!std::strcmp(key, "sap_link16")) return &c->sap_link16;
  return nullptr;
}
static const char* tuning_keys[] = {"dslash_variant_f64", "dslash_variant_f32", "dslash_variant_bf16", "nr_f64", "nr_low",
                                    "xcd_map", "net_mfma", "block_solver", "block_lanes", "block_eo",
                                    "block_eo_lanes", "block_tol_prec", "sap_bf16", "block_xcd", "sap_link16"};

psms_status psms_set_tuning(psms_ctx* c, const char* key, int value) {
  API_BEGIN(c)
  REQUIRE(key != nullptr, "null key");
  int* t = tuning_slot(c, key);
  REQUIRE(t != nullptr, std::string("unknown tuning key ") + key);
  if (std::strncmp(key, "dslash_variant", 14) == 0) REQUIRE(value >= 0 && value <= 8, "stencil variant must be in [0, 8]");
  else if (!std::strcmp(key, "block_eo"))
    REQUIRE(value >= 0 && value <= 3, "block_eo must be 0 (plain), 1 (even-odd), 2 (by launch shape) or 3 (even-odd, links from L2)");
  else if (!std::strcmp(key, "xcd_map") || !std::strcmp(key, "net_mfma") || !std::strcmp(key, "block_solver") ||
           !std::strcmp(key, "sap_bf16"))
    REQUIRE(value == 0 || value == 1, "flag must be 0 or 1");
  else if (!std::strcmp(key, "sap_link16"))
    REQUIRE(value >= 0 && value <= 2, "sap_link16 must be 0 (FP32 links), 1 (FP16 12-real links) or 2 (FP16 links and fields)");
  else if (!std::strcmp(key, "block_xcd"))
    REQUIRE(value >= 0 && value <= 2, "block_xcd must be 0 (launch order), 1 (by XCD) or 2 (by link footprint)");
  else if (!std::strcmp(key, "block_eo_lanes"))
    REQUIRE(value == 0 || value == 2 || value == 4, "even-odd lanes per site must be 0 (default), 2 or 4");
  else if (!std::strcmp(key, "block_tol_prec"))
    REQUIRE(value >= 0 && value <= 2, "block_tol_prec must be 0 (by block size), 1 (FP32 passes) or 2 (FP64)");
  else if (!std::strcmp(key, "block_lanes"))
    REQUIRE(value >= 0 && value <= 2, "lanes per site must be 0 (by grid size), 1 or 2");
  else REQUIRE(value == 1 || value == 2 || value == 4, "right-hand sides per thread must be 1, 2 or 4");
  *t = value;
  API_END(c)
  return PSMS_OK;
}

psms_status psms_get_tuning(psms_ctx* c, const char* key, int* value) {
  API_BEGIN(c)
  REQUIRE(key != nullptr && value != nullptr, "null argument");
  int* t = tuning_slot(c, key);
  REQUIRE(t != nullptr, std::string("unknown tuning key ") + key);
  *value = *t;
  API_END(c)
  return PSMS_OK;
}

static std::string tuning_key(psms_ctx* c) {
  hipDeviceProp_t prop;
  std::string arch = "unknown";
  if (hipGetDeviceProperties(&prop, c->device) == hipSuccess) arch = prop.gcnArchName;
  char buf[256];
  std::snprintf(buf, sizeof buf, "%s|L=%dx%dx%dx%d|b=%dx%dx%dx%d", arch.c_str(), c->g.L[0], c->g.L[1], c->g.L[2], c->g.L[3],
                c->g.b[0], c->g.b[1], c->g.b[2], c->g.b[3]);
  return buf;
}

// Mean time of `reps` full-lattice stencil launches with the current tuning.
static double time_dslash(psms_ctx* c, const Links& L, const FieldBatch& in, const FieldBatch& out, int reps) {
  for (int i = 0; i < 2; ++i) apply_D(c, L, in, out);
  hipEvent_t a = get_event(c), b = get_event(c);
  HIPCHK(hipEventRecord(a, c->st));
  for (int i = 0; i < reps; ++i) apply_D(c, L, in, out);
  HIPCHK(hipEventRecord(b, c->st));
  HIPCHK(hipEventSynchronize(b));
  float ms = 0;
  HIPCHK(hipEventElapsedTime(&ms, a, b));
  c->pool.push_back(a);
  c->pool.push_back(b);
  return ms / reps;
}

psms_status psms_autotune(psms_ctx* c, int slot, const char* cache_path) {
  API_BEGIN(c)
  const std::string key = tuning_key(c);
  if (cache_path) {
    if (FILE* f = std::fopen(cache_path, "r")) {
      char line[1024];
      while (std::fgets(line, sizeof line, f)) {
        if (!std::strstr(line, (std::string("\"key\": \"") + key + "\"").c_str())) continue;
        for (const char* k : tuning_keys) {
          const char* q = std::strstr(line, (std::string("\"") + k + "\": ").c_str());
          if (q) *tuning_slot(c, k) = std::atoi(q + std::strlen(k) + 4);
        }
        c->tuned_from = "cache";
      }
      std::fclose(f);
      if (c->tuned_from == "cache") return PSMS_OK;
    }
  }
  REQUIRE(slot >= 0 && slot < 64 && c->slots[slot].loaded, "autotune needs a loaded gauge slot");
  // kernel timing off while tuning; the setting and the tuning buffers are restored and
  // freed on every way out
  struct Restore {
    psms_ctx* c;
    bool prof;
    ~Restore() {
      c->prof = prof;
      for (const char* b : {"tune_in", "tune_out", "tune_raw"}) {
        auto it = c->bufs.find(b);
        if (it == c->bufs.end()) continue;
        if (it->second.p) {
          (void)hipStreamSynchronize(c->st);
          (void)hipFree(it->second.p);
          c->held -= it->second.n;
        }
        c->bufs.erase(it);
      }
    }
  } restore{c, c->prof};
  c->prof = false;
  // The solvers apply the stencil in their own layout when the Schwarz blocks differ from
  // the domain blocks (the 32^4 estimator: 4^4 inside 8^4): the forms are timed there.
  struct SolverView {
    psms_ctx* c;
    bool on;
    explicit SolverView(psms_ctx* cc) : c(cc), on(cc->split && !cc->solver_view) {
      if (on) {
        std::swap(c->g, c->gs);
        c->solver_view = true;
      }
    }
    ~SolverView() {
      if (on) {
        std::swap(c->g, c->gs);
        c->solver_view = false;
      }
    }
  } view(c);
  const int reps = c->V >= (1 << 20) ? 10 : 30;
  // Stencil forms are timed on two launch shapes the solvers make: one gauge field with
  // 16 right-hand sides (1 from 2^20 sites up, where one right-hand side is not bound by
  // launch latency), and the other loaded gauge fields as the proposals of one launch
  // (as the batched estimator launches them) with 128 right-hand sides in all (from 2^20
  // sites up 8 per proposal, the 32^4 estimator's launches; each tuning buffer within
  // 8 GiB). After a warm-up round, each form keeps its best time over three
  // interleaved rounds, so that clock changes during tuning favour no form. The pick is
  // the form whose worst slowdown against the fastest form of a shape is smallest: a form
  // that is fast on one shape and slow on the other loses to one that is good on both.
  const bool big = c->V >= (1 << 20);
  // Gaussian inputs (zeros draw less power, which can change clocks and so the ranking)
  auto fill = [&](const FieldBatch& in) {
    const size_t fd = size_t(c->V) * 24;
    const int nf = in.nprop * in.nrhs;
    double* raw = dscratch<double>(c, "tune_raw", fd * nf);
    launch_gaussian(c->st, raw, fd / 2, nf, 0x74756e65ULL, 0);
    launch_pack(c->st, c->g, raw, in);
  };
  for (int pr = 0; pr < 3; ++pr) {
    Prec P = Prec(pr);
    if (P != P_F64 && !c->slots[slot].su3) continue;
    // the proposals: every other loaded slot (the slot itself when there is none)
    std::vector<int> props;
    for (int i = 0; i < 64 && int(props.size()) < MAXPROP; ++i)
      if (i != slot && c->slots[i].loaded && (P == P_F64 || c->slots[i].su3)) props.push_back(i);
    if (props.empty()) props.push_back(slot);
    const int fmt = P == P_F64 ? LK_F64 : LK_F32C12;
    // Forms whose kernels spill registers to scratch are not timed while any form does not:
    // their cost depends on what else occupies the caches, so an isolated timing misleads.
    bool spills[NVAR], any_clean = false;
    for (int v = 0; v < NVAR; ++v) {
      spills[v] = dslash_variant_scratch(P, P, v) > 0 || (P == P_BF16 && dslash_variant_scratch(P, P_F32, v) > 0);
      any_clean |= !spills[v];
    }
    // BF16 inputs also meet FP32 outputs (a different kernel under the same form number):
    // a third measurement, the batched shape into FP32
    const int nsh = P == P_BF16 ? 3 : 2;
    double tv[NVAR][3];
    for (auto& row : tv) row[0] = row[1] = row[2] = 1e30;
    // each tuning buffer (input, output, Gaussian staging) is kept within 8 GiB
    const size_t cap = std::max<size_t>(1, (size_t(8) << 30) / (size_t(c->V) * 24 * sizeof(double)));
    for (int si = 0; si < nsh; ++si) {
      const int np = si == 0 ? 1 : int(std::min<size_t>(props.size(), cap));
      const int nrhs = int(std::min<size_t>(si == 0 ? (big ? 1 : 16) : (big ? 8 : std::max(1, 128 / np)),
                                            std::max<size_t>(1, cap / np)));
      Links L = links_of(c, si == 0 ? &slot : props.data(), np, fmt);
      FieldBatch in = field(c, "tune_in", P, np, nrhs);
      FieldBatch out = field(c, "tune_out", si == 2 ? P_F32 : P, np, nrhs);
      fill(in);
      const int r = si == 0 ? reps : std::max(3, reps / 4);
      for (int pass = 0; pass < 4; ++pass)  // pass 0 only warms up (clocks, first launches)
        for (int v = 0; v < NVAR; ++v) {
          if (any_clean && spills[v]) continue;
          c->variant[pr] = v;
          const double t = time_dslash(c, L, in, out, r);
          if (pass > 0) tv[v][si] = std::min(tv[v][si], t);
        }
    }
    double fastest[3] = {1e30, 1e30, 1e30};
    for (int v = 0; v < NVAR; ++v)
      for (int si = 0; si < nsh; ++si) fastest[si] = std::min(fastest[si], tv[v][si]);
    int best = -1;
    double worst_best = 1e30;
    for (int v = 0; v < NVAR; ++v) {
      if (any_clean && spills[v]) continue;
      double worst = 0;
      for (int si = 0; si < nsh; ++si) worst = std::max(worst, tv[v][si] / fastest[si]);
      if (worst < worst_best) {
        worst_best = worst;
        best = v;
      }
    }
    c->variant[pr] = best < 0 ? 0 : best;
  }
  // right-hand sides per thread for batched launches (8 right-hand sides)
  for (int pr = 0; pr < 2; ++pr) {
    Prec P = pr == 0 ? P_F64 : P_F32;
    if (P != P_F64 && !c->slots[slot].su3) continue;
    Links L = links_of(c, &slot, 1, P == P_F64 ? LK_F64 : LK_F32C12);
    FieldBatch in = field(c, "tune_in", P, 1, 8), out = field(c, "tune_out", P, 1, 8);
    fill(in);
    int* nr = pr == 0 ? &c->nr_f64 : &c->nr_low;
    double tn[3] = {1e30, 1e30, 1e30};
    const int cands[3] = {1, 2, 4};
    for (int round = 0; round < 3; ++round)
      for (int i = 0; i < 3; ++i) {
        *nr = cands[i];
        tn[i] = std::min(tn[i], time_dslash(c, L, in, out, std::max(3, reps / 4)));
      }
    int best = 0;
    for (int i = 1; i < 3; ++i)
      if (tn[i] < tn[best]) best = i;
    *nr = cands[best];
  }
  c->tuned_from = "autotune";
  if (cache_path) {
    if (FILE* f = std::fopen(cache_path, "a")) {
      std::fprintf(f, "{\"key\": \"%s\"", key.c_str());
      for (const char* k : tuning_keys) std::fprintf(f, ", \"%s\": %d", k, *tuning_slot(c, k));
      std::fprintf(f, "}\n");
      std::fclose(f);
    }
  }
  API_END(c)
  return PSMS_OK;
}

psms_status psms_profile(psms_ctx* c, int enable) {
  API_BEGIN(c)
  prof_collect(c);
  if (enable) {
    for (int f = 0; f < NFAM; ++f) {
      c->prof_ms[f] = 0;
      c->prof_n[f] = 0;
      c->prof_bytes[f] = 0;
    }
  }
  c->prof = enable != 0;
  API_END(c)
  return PSMS_OK;
}

psms_status psms_profile_read(psms_ctx* c, const char* family, double* total_ms, long long* launches,
                              double* algorithmic_bytes) {
  API_BEGIN(c)
  prof_collect(c);
  REQUIRE(family != nullptr, "null family");
  for (int f = 0; f < NFAM; ++f) {
    if (std::strcmp(family, fam_names[f]) == 0) {
      if (total_ms) *total_ms = c->prof_ms[f];
      if (launches) *launches = c->prof_n[f];
      if (algorithmic_bytes) *algorithmic_bytes = c->prof_bytes[f];
      return PSMS_OK;
    }
  }
  throw Err{PSMS_EINVAL, std::string("unknown kernel family ") + family};
  API_END(c)
  return PSMS_OK;
}

}  // extern "C"
