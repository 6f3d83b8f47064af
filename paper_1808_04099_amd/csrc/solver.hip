// Host orchestration of the projection path: workspace plan, multigrid V-cycle coarsened
// inside each cube down to one cell per cube (Sec. 3), where multigrid on the cube graph (or
// the paper's conjugate-gradient solve, Sec. 7) takes over, flexible CG wrapper, FP64
// iterative refinement of FP32 inner solves, projection step (Sec. 3) and its adjoint,
// exposed through the C ABI of bcm.h.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <climits>
#include <cmath>
#include <cstdio>
#include <cstring>
#include <mutex>
#include <string>
#include <vector>

#include "bcm_internal.hpp"
#include "kernels.hpp"

namespace bcm {

namespace {

__global__ void k_fill(double* p, size_t n, double v) {
  for (size_t e = blockIdx.x * size_t(blockDim.x) + threadIdx.x; e < n; e += size_t(gridDim.x) * blockDim.x)
    p[e] = v;
}
__global__ void k_fillf(float* p, size_t n, float v) {
  for (size_t e = blockIdx.x * size_t(blockDim.x) + threadIdx.x; e < n; e += size_t(gridDim.x) * blockDim.x)
    p[e] = v;
}

template <typename T>
hipError_t fill(T* p, size_t n, hipStream_t s) {
  const int blocks = int(std::min<size_t>((n + 255) / 256, 65536));
  if (n == 0) return hipSuccess;
  if constexpr (sizeof(T) == 8)
    hipLaunchKernelGGL(k_fill, dim3(blocks), dim3(256), 0, s, reinterpret_cast<double*>(p), n, 0.0);
  else
    hipLaunchKernelGGL(k_fillf, dim3(blocks), dim3(256), 0, s, reinterpret_cast<float*>(p), n, 0.0f);
  return hipGetLastError();
}

const char* const kTimerNames[] = {"presmooth16", "presmooth8", "presmooth4", "presmooth2",
                                   "postsmooth16", "postsmooth8", "postsmooth4", "postsmooth2", "restrict16",
                                   "restrict8", "restrict4", "restrict2", "apply16", "apply8",
                                   "apply4", "apply2", "update", "resid64", "ir", "coarse",
                                   "finalize", "force", "div", "correct", "adj_gp", "adj_rhs",
                                   "export", "xupdate", "momentum", "momentum_start", "ib", "codec",
                                   "preupd16", "preupd8", "preupd4", "preupd2", "rprobe", nullptr};

int level_index(int NL) { return NL == 16 ? 0 : NL == 8 ? 1 : NL == 4 ? 2 : 3; }

struct Status {
  int code = BCM_OK;
  std::string msg;
};

}  // namespace

struct Timer {
  int cls = -1;
  int every = 1;     // time one launch of the class in every `every`
  int64_t seen = 0;  // launches of the class since enabled
  std::vector<hipEvent_t> ev;
  size_t used = 0;
};

}  // namespace bcm

using namespace bcm;

struct bcm_plan {
  const HostMesh* M = nullptr;
  bcm_solver_opts o{};
  int n = 0, nlev = 0, nc = 0;
  size_t cells = 0;
  bool inner32 = false, fields32 = false;
  size_t ws_bytes = 0;
  char* ws = nullptr;
  // workspace offsets
  size_t o_meta = 0, o_launch = 0, o_part[3] = {0, 0, 0}, o_sc = 0, o_cw = 0;
  size_t o_nb27 = 0;  // 27-neighbourhoods (trilinear prolongation), 0 = not used
  // momentum sub-step (single-level meshes with n >= 4, else 0): two-layer faces of u^n and of
  // the two Crank-Nicolson iterates, its right-hand side and a second iterate
  size_t o_mfa[3] = {0, 0, 0}, o_mfv[2][3] = {{0, 0, 0}, {0, 0, 0}}, o_mrhs[3] = {0, 0, 0},
         o_mit[3] = {0, 0, 0};
  bool momentum = false;
  // Lagrangian-particle forcing: per-level point-location tables (finest level first)
  std::vector<int32_t> ib_table;
  std::vector<IbLevel> ib_levels;
  double ib_anchor[3] = {0, 0, 0};
  size_t o_ibtab = 0, o_iberr = 0;
  bool ib = false;
  size_t o_cflag = 0;  // wavelet codec: total bytes (u64) and error flags (u32)
  size_t o_ustar[3] = {0, 0, 0}, o_uf = 0, o_b64 = 0, o_pf = 0, o_lam = 0;
  size_t o_body = 0;  // per-cube forcing flags of the 16^3 projection (1 byte per cube)
  size_t o_r = 0, o_z = 0, o_p = 0, o_q = 0, o_d = 0;
  size_t o_zf[2] = {0, 0}, o_pfk[2] = {0, 0};
  std::vector<size_t> o_x, o_b, o_xf[2];  // per level (index 0 unused for x/b: level 0 = z/r)
  int pf_cur = 0;                         // ping-pong index of the Krylov search-direction faces
  // cube-graph multigrid (coarse_solver 1)
  bool graph = false;
  struct GOff {
    size_t col, val, diag, vol, parent, child, child_w, x, b, r, pcol;
    int lds_x, lds_b, lds_r;
  };
  std::vector<GOff> g_off;
  size_t o_glev = 0, o_gw = 0, o_perm0 = 0, o_ginv = 0;
  int g_lds = 0, g_lds_inv = -1;
  int g_split = 0;  // leading graph levels smoothed by the multi-workgroup kernels
  hipStream_t s2 = nullptr;        // Krylov x updates, beside the next V-cycle
  hipEvent_t ev_mid = nullptr, ev_x = nullptr;
  int side_wgs = 1;                // workgroups of a vector update carried by the coarse launch
  ScalarMirror* mirror = nullptr;  // pinned host copy of the scalars (nullptr: copy + sync)
  uint32_t mirror_seq = 0;         // sequence number of the last finalize
  Timer timer;
  template <typename P> P* at(size_t off) const { return reinterpret_cast<P*>(ws + off); }
};

namespace {

constexpr size_t kAlign = 256;

size_t take(size_t& top, size_t bytes) {
  const size_t off = top;
  top += (bytes + kAlign - 1) / kAlign * kAlign;
  return off;
}

int hip_fail(hipError_t e, const char* what) {
  set_error(std::string(what) + ": " + hipGetErrorString(e));
  return BCM_ERR_HIP;
}

#define HIPCHK(expr, what)                           \
  do {                                               \
    hipError_t _e = (expr);                          \
    if (_e != hipSuccess) return hip_fail(_e, what); \
  } while (0)

// Timed launch: when timing is enabled for `cls`, bracket the launch with events.
template <class F>
hipError_t timed(bcm_plan* P, int cls, hipStream_t s, F&& launch) {
  Timer& t = P->timer;
  const bool on = t.cls == cls && t.seen++ % t.every == 0;
  if (on) {
    if (t.used + 2 > t.ev.size()) {
      for (int i = 0; i < 256; ++i) {
        hipEvent_t e;
        hipError_t err = hipEventCreate(&e);
        if (err != hipSuccess) return err;
        t.ev.push_back(e);
      }
    }
    hipError_t err = hipEventRecord(t.ev[t.used], s);
    if (err != hipSuccess) return err;
  }
  hipError_t err = launch();
  if (on) {
    if (err == hipSuccess) err = hipEventRecord(t.ev[t.used + 1], s);
    t.used += 2;
  }
  return err;
}

int cls_of(const char* base, int NL) {
  char name[32];
  std::snprintf(name, sizeof(name), "%s%d", base, NL);
  for (int i = 0; kTimerNames[i]; ++i)
    if (!std::strcmp(kTimerNames[i], name) || !std::strcmp(kTimerNames[i], base)) return i;
  return -1;
}

Geom geom(const bcm_plan* P, int NL) {
  return Geom{P->at<const CubeMeta>(P->o_meta), P->at<const int32_t>(P->o_launch), P->nc,
              double(P->n) / double(NL), P->M->multilevel ? 1 : 0};
}

// Scalars of the last finalize.  With the pinned mirror the host polls its sequence number
// (checking the stream every 1024 polls, so that an error or a finished stream ends the wait)
// instead of synchronising the stream, which takes tens of microseconds longer to return.
int read_scalars(bcm_plan* P, Scalars* host, hipStream_t s) {
  if (P->mirror) {
    const uint32_t want = P->mirror_seq;
    auto ready = [&] { return __atomic_load_n(&P->mirror->seq, __ATOMIC_ACQUIRE) == want; };
    for (unsigned n = 1; !ready(); ++n) {
      if ((n & 1023) != 0) continue;
      const hipError_t e = hipStreamQuery(s);
      if (e == hipErrorNotReady) continue;
      if (e != hipSuccess) return hip_fail(e, "stream query");
      if (!ready()) {
        set_error("scalar readback: the stream finished without publishing the scalars");
        return BCM_ERR_HIP;
      }
    }
    std::memcpy(host, const_cast<const Scalars*>(&P->mirror->sc), sizeof(Scalars));
    return BCM_OK;
  }
  HIPCHK(hipMemcpyAsync(host, P->at<Scalars>(P->o_sc), sizeof(Scalars), hipMemcpyDeviceToHost, s),
         "scalar readback");
  HIPCHK(hipStreamSynchronize(s), "stream synchronize");
  return BCM_OK;
}

int finalize(bcm_plan* P, int op, int which0, int which1, int nparts, int first, hipStream_t s) {
  // the two recurrences in the middle of a Krylov iteration are never read by the host before
  // the next finalize: they skip the copy to the pinned mirror and its system-scope fence
  const bool publish = P->mirror && op != OP_ZRZQ && op != OP_PQ;
  FinalizeArgs a{P->at<double>(P->o_part[which0]), which1 >= 0 ? P->at<double>(P->o_part[which1]) : nullptr,
                 nparts, P->at<Scalars>(P->o_sc), op, first, publish ? P->mirror : nullptr,
                 publish ? ++P->mirror_seq : 0u};
  HIPCHK(timed(P, cls_of("finalize", 0), s, [&] { return launch_finalize(a, s); }), "k_finalize");
  return BCM_OK;
}

int n_wg(int NL, int nc) {
  const int c = cubes_per_wg(NL);
  return (nc + c - 1) / c;
}

// Export the faces of an FP64 field (kc_ir without an update).
int export64(bcm_plan* P, double* x, double* xf, hipStream_t s) {
  IrArgs<float> a{geom(P, P->n), x, nullptr, xf, 0.0};
  HIPCHK(timed(P, cls_of("export", 0), s, [&] { return launch_ir<float>(P->n, a, s); }), "export faces");
  return BCM_OK;
}

// Multigrid on the cube graph when its leading levels are large: those levels are smoothed by
// multi-workgroup kernels (one launch per colour), the rest by the single workgroup.
template <typename T>
int coarse_split(bcm_plan* P, const T* b_in, T* x_out, T* xf_out, hipStream_t s) {
  const auto& Ls = P->M->coarse.levels;
  const int S = P->g_split, pre = 2, post = 2;
  GStepArgs<T> ga{P->at<const GLevel<T>>(P->o_glev), 0, 0, 0, b_in, x_out, xf_out,
                  P->at<const int32_t>(P->o_perm0), P->nc};
  auto step = [&](int kind, int g, int n, int lo = 0, int hi = 0) -> int {
    ga.g = g;
    ga.lo = lo;
    ga.hi = hi;
    HIPCHK(timed(P, cls_of("coarse", 0), s, [&] { return launch_g_step<T>(kind, n, ga, s); }),
           "graph multigrid step");
    return BCM_OK;
  };
  auto sweep = [&](int g, bool forward) -> int {
    const auto& co = Ls[g].color_off;
    const int nc = int(co.size()) - 1;
    for (int k = 0; k < nc; ++k) {
      const int c = forward ? k : nc - 1 - k;
      if (int e = step(G_SMOOTH, g, co[c + 1] - co[c], co[c], co[c + 1])) return e;
    }
    return BCM_OK;
  };
  int st = step(G_GATHER, 0, P->nc);
  for (int cy = 0; cy < P->o.coarse_cycles && !st; ++cy) {
    for (int g = 0; g < S && !st; ++g) {
      for (int k = 0; k < pre && !st; ++k) st = sweep(g, true);
      if (!st) st = step(G_RESID, g, Ls[g].n);
      if (!st) st = step(G_RESTRICT, g, Ls[g + 1].n);
    }
    if (st) break;
    CoarseMGArgs<T> a{b_in, x_out, xf_out, P->at<const GLevel<T>>(P->o_glev),
                      P->at<const int32_t>(P->o_perm0), int(P->g_off.size()), S, 1, pre, post,
                      std::max(P->o.coarse_iters, 64), P->at<double>(P->o_gw),
                      P->M->coarse.bottom_inv.empty() ? nullptr : P->at<const T>(P->o_ginv), P->g_lds,
                      P->g_lds_inv};
    HIPCHK(timed(P, cls_of("coarse", 0), s, [&] { return launch_coarse_mg<T>(a, s); }), "k_coarse_mg");
    for (int g = S - 1; g >= 0 && !st; --g) {
      st = step(G_PROLONG, g, Ls[g].n);
      for (int k = 0; k < post && !st; ++k) st = sweep(g, false);
    }
  }
  if (!st) st = step(G_SCATTER, 0, P->nc);
  return st;
}

// The V-cycle's arrays: iterate, right-hand side and the two face buffers of level l.
template <typename T>
struct VLevels {
  bcm_plan* P;
  T* X(int l) const { return l == 0 ? P->at<T>(P->o_z) : P->at<T>(P->o_x[l]); }
  T* B(int l) const { return l == 0 ? P->at<T>(P->o_r) : P->at<T>(P->o_b[l]); }
  T* F(int ab, int l) const { return l == 0 ? P->at<T>(P->o_zf[ab]) : P->at<T>(P->o_xf[ab][l]); }
};

// The pre-smoother of level l (< nlev - 1): from zero, with the restriction of its residual
// fused in.  Its cross-cube terms need the neighbours' smoothed faces, so the next level's
// pre-smoother adds them (it reads nothing across faces itself: its iterate starts at zero),
// and kc_rfix only after the last such level.
// upd (level 0): the previous Krylov step's r update, applied by this launch to b (= r).
template <typename T>
int presmooth(bcm_plan* P, int l, hipStream_t s, const UpdateArgs<T>* upd = nullptr) {
  const VLevels<T> V{P};
  const int NL = P->n >> l;
  SmoothArgs<T> sa{};
  if (upd) {
    sa.upd_q = upd->q;
    sa.upd_sc = upd->sc;
    sa.part_rr = P->at<double>(P->o_part[0]);
  }
  sa.g = geom(P, NL);
  sa.x = V.X(l);
  sa.b = V.B(l);
  sa.xf_out = V.F(0, l);
  sa.sweeps = P->o.pre_sweeps;
  sa.black_first = 0;
  sa.zero_init = 1;
  sa.bc = V.B(l + 1);
  if (l > 0) {
    sa.rfx = V.F(0, l - 1);
    sa.b_fixed = V.B(l);
    sa.rfx_hscale = geom(P, NL * 2).hscale;
  }
  HIPCHK(timed(P, cls_of(upd ? "preupd" : "presmooth", NL), s, [&] { return launch_smooth<T>(NL, sa, s); }),
         "kc_smooth (pre)");
  return BCM_OK;
}

// One V-cycle on (b_0 = r, x_0 = z): per-cube levels NL = n, n/2, ..., 2 smoothed with
// red-black Gauss-Seidel, then the one-cell-per-cube level (cube-graph multigrid, or the
// paper's CG with coarse_solver 0).  At level 0 the final smoothing also accumulates <z, r>
// and (if q_dot) <z, q>.
//
// upd: the previous Krylov step's r update, applied by the level-0 pre-smoother (which needs
// nlev >= 2), after which after_pre0(stop) runs (the convergence check); stop = true ends the
// V-cycle there.
template <typename T, class Hook, class After>
int vcycle(bcm_plan* P, const T* q_dot, hipStream_t s, Hook&& before_coarse, const UpdateArgs<T>* upd,
           After&& after_pre0, bool& stop) {
  const int L = P->nlev;
  const VLevels<T> V{P};
  auto X = [&](int l) { return V.X(l); };
  auto B = [&](int l) { return V.B(l); };
  auto F = [&](int ab, int l) { return V.F(ab, l); };
  const bcm_solver_opts& o = P->o;
  stop = false;
  for (int l = 0; l < L - 1; ++l) {
    const int NL = P->n >> l;
    if (const int st = presmooth<T>(P, l, s, l == 0 ? upd : nullptr)) return st;
    if (l == L - 2) {
      RestrictFixArgs<T> ra{geom(P, NL), F(0, l), B(l + 1)};
      HIPCHK(timed(P, cls_of("restrict", NL), s, [&] { return launchc_rfix<T>(NL, ra, s); }), "kc_rfix");
    }
    if (l == 0) {
      if (const int st = after_pre0(stop)) return st;
      if (stop) return BCM_OK;
    }
  }
  if (P->graph && P->g_split > 0) {
    if (const int st = before_coarse(nullptr)) return st;
    if (int st = coarse_split<T>(P, B(L - 1), X(L - 1), F(1, L - 1), s)) return st;
  } else if (P->graph) {
    CoarseMGArgs<T> ga{B(L - 1), X(L - 1), F(1, L - 1), P->at<const GLevel<T>>(P->o_glev),
                       P->at<const int32_t>(P->o_perm0), int(P->g_off.size()), 0, o.coarse_cycles,
                       2, 2, std::max(o.coarse_iters, 64),  // the last graph level has <= 64 nodes
                       P->at<double>(P->o_gw),
                       P->M->coarse.bottom_inv.empty() ? nullptr : P->at<const T>(P->o_ginv), P->g_lds,
                      P->g_lds_inv};
    if (const int st = before_coarse(&ga)) return st;  // may hand it a vector update to carry
    HIPCHK(timed(P, cls_of("coarse", 0), s, [&] { return launch_coarse_mg<T>(ga, s); }), "k_coarse_mg");
  } else {
    if (const int st = before_coarse(nullptr)) return st;
    CoarseArgs<T> ca{P->at<const CubeMeta>(P->o_meta), P->nc, double(P->n), B(L - 1), X(L - 1),
                     F(1, L - 1), P->at<double>(P->o_cw), o.coarse_iters};
    HIPCHK(timed(P, cls_of("coarse", 0), s, [&] { return launch_coarse<T>(ca, s); }), "k_coarse");
  }
  for (int l = L - 2; l >= 0; --l) {
    const int NL = P->n >> l;
    SmoothArgs<T> sa{};
    sa.g = geom(P, NL);
    sa.x = X(l);
    sa.b = B(l);
    sa.xf_in = F(0, l);
    sa.xf_out = F(1, l);
    sa.xc = X(l + 1);
    sa.xcf = F(1, l + 1);
    sa.nb27 = P->o_nb27 ? P->at<const uint32_t>(P->o_nb27) : nullptr;
    sa.sweeps = o.post_sweeps;
    sa.black_first = 1;
    sa.zero_init = 0;
    if (l == 0) {
      sa.r_dot = B(0);
      sa.q_dot = q_dot;
      sa.part_zr = P->at<double>(P->o_part[0]);
      sa.part_zq = q_dot ? P->at<double>(P->o_part[1]) : nullptr;
    }
    HIPCHK(timed(P, cls_of("postsmooth", NL), s, [&] { return launch_smooth<T>(NL, sa, s); }), "kc_smooth (post)");
  }
  return BCM_OK;
}

struct SolveLog {
  bcm_report* rep;
  int iters = 0;
  bool stalled = false;  // a Krylov solve stopped because its residual stopped decreasing
  void push(double v) {
    if (rep && rep->history && rep->history_len < rep->history_cap) rep->history[rep->history_len++] = v;
  }
};

constexpr int kStallChecks = 10;      // checks without progress that count as stagnation
constexpr double kStallFactor = 0.99;  // progress = the residual norm falls below 0.99 x best

// Flexible CG (or plain V-cycle iteration) on A x = r0 with r (= P->o_r) holding the initial
// residual and x the accumulator (x_zero: x starts at zero and is not read before its first
// update).  Stops when the V-weighted <r, r> <= thr (recurrence).
// hist_scale converts sqrt(<r,r>) to the reported relative residual.
// defer: on a normal return the last pending x update is not launched but handed to the
// caller in *defer (defer->p != nullptr), which must apply it (the mixed path folds it into
// the refinement update).
template <typename T>
int krylov(bcm_plan* P, T* x, bool x_zero, double thr, int max_iter, double hist_scale, SolveLog& log,
           Scalars* hs, hipStream_t s, UpdateArgs<T>* defer = nullptr) {
  const int NL = P->n;
  const int nparts = partials_of(NL, P->nc);
  T* r = P->at<T>(P->o_r);
  T* z = P->at<T>(P->o_z);
  T* p = P->at<T>(P->o_p);
  T* q = P->at<T>(P->o_q);
  const bool fcg = P->o.krylov != 0;    // conjugate gradients (else V-cycle iteration)
  const bool flex = P->o.krylov == 1;  // flexible CG: beta from <z, q_old>
  // The x update of iteration it needs only alpha and p, which stay put until the apply of
  // iteration it + 1.  It is launched on the second stream when the next V-cycle reaches its
  // one-cell-per-cube solve, which occupies a single workgroup, and that apply waits for it.
  UpdateArgs<T> ux{};
  bool pending = false, in_flight = false;
  auto launch_x = [&](hipStream_t on) {
    return timed(P, cls_of("xupdate", 0), on, [&] { return launch_update<T>(ux, on); });
  };
  auto start_x = [&](bool beside, CoarseMGArgs<T>* carrier) -> int {
    if (!pending) return BCM_OK;
    pending = false;
    const bool vec_ok = (reinterpret_cast<uintptr_t>(ux.x) | reinterpret_cast<uintptr_t>(ux.p)) % 16 == 0;
    if (beside && carrier && vec_ok) {  // the single-workgroup coarse solve's launch carries it
                                        // (16-byte accesses: x and p must be 16-byte aligned)
      carrier->xu_x = ux.x;
      carrier->xu_p = ux.p;
      carrier->xu_alpha = &ux.sc->alpha;
      carrier->xu_n = size_t(ux.n_cubes) * size_t(ux.n3);
      carrier->xu_zero = ux.x_zero;
      carrier->xu_wgs = P->side_wgs;
      return BCM_OK;
    }
    if (!P->s2 || !beside) {
      HIPCHK(launch_x(s), "k_update (x)");
      return BCM_OK;
    }
    HIPCHK(hipEventRecord(P->ev_mid, s), "event record");
    HIPCHK(hipStreamWaitEvent(P->s2, P->ev_mid, 0), "stream wait");
    HIPCHK(launch_x(P->s2), "k_update (x)");
    HIPCHK(hipEventRecord(P->ev_x, P->s2), "event record");
    in_flight = true;
    return BCM_OK;
  };
  auto join_x = [&]() -> int {
    if (!in_flight) return BCM_OK;
    in_flight = false;
    HIPCHK(hipStreamWaitEvent(s, P->ev_x, 0), "stream wait");
    return BCM_OK;
  };
  auto finish = [&](int st) {  // every exit: no x update left behind
    int e = join_x();
    if (!e && !st && defer && pending) {  // the caller applies it
      *defer = ux;
      pending = false;
    }
    if (!e) e = start_x(false, nullptr);  // nothing left to run beside: on the caller's stream
    return st ? st : e;
  };
  // stagnation: kStallChecks convergence checks in a row without a 1% reduction of the best
  // residual norm seen so far end the solve early (the iterate stays valid)
  double best_rr = HUGE_VAL;
  int stall = 0;
  // The r update r -= alpha q of iteration it is applied by the first pre-smoother of V-cycle
  // it + 1 (which reads r anyway), and the convergence check after it sits between that
  // pre-smoother and the rest of the V-cycle; a converged solve drops the rest.  After the
  // last iteration, or without a per-cube level to smooth (nlev < 2), it runs on its own.
  // A fused launch whose check ends the solve does its pre-smoothing for nothing, so when the
  // residual's last reduction factor predicts convergence at the next check (with checks every
  // iteration), a probe computes that check's <r, r> alone, leaving r as it is (an ended solve
  // never reads r again); if the solve goes on, the fused launch still applies the update and
  // skips the check (probed).  After the last allowed iteration the probe also serves.
  const bool fuse = P->nlev >= 2;
  UpdateArgs<T> ur{};
  bool r_pending = false, probed = false;
  double rr_a = -1.0, rr_b = -1.0;  // the last two checked <r, r> (rr_b the latest)
  // <r, r> of the update of iteration it (partials: nrr), and the convergence checks every
  // check_every iterations and at the last one
  auto check = [&](int it, int nrr, bool& stop) -> int {
    stop = false;
    if (const int st = finalize(P, OP_RR, 0, -1, nrr, 0, s)) return st;
    log.iters++;
    if ((it + 1) % P->o.check_every != 0 && it + 1 < max_iter) return BCM_OK;
    if (const int st = read_scalars(P, hs, s)) return st;
    if (!std::isfinite(hs->rr)) {
      set_error("non-finite residual in the Krylov iteration");
      return BCM_ERR_NONFINITE;
    }
    log.push(std::sqrt(std::max(hs->rr, 0.0)) * hist_scale);
    rr_a = rr_b;
    rr_b = hs->rr;
    if (hs->rr <= thr) {
      stop = true;
    } else if (hs->rr < kStallFactor * kStallFactor * best_rr) {
      best_rr = hs->rr;
      stall = 0;
    } else if (++stall >= kStallChecks) {
      log.stalled = true;
      stop = true;
    }
    return BCM_OK;
  };
  // the pending r update on its own (probe: only its <r, r>), with per-cube partials
  auto update_alone = [&](int it, bool probe, bool& stop) -> int {
    UpdateArgs<T> a = ur;
    a.part_sel = probe ? 3 : 1;
    r_pending = probe;
    probed = probe;
    HIPCHK(timed(P, cls_of(probe ? "rprobe" : "update", 0), s, [&] { return launch_update<T>(a, s); }),
           "k_update");
    return check(it, P->nc, stop);
  };
  for (int it = 0; it < max_iter; ++it) {
    bool stop = false;
    bool alone = r_pending && !fuse;
    if (r_pending && fuse && P->o.check_every == 1 && rr_a > 0.0 && rr_b > 0.0 &&
        rr_b * (rr_b / rr_a) <= 3.0 * thr)
      alone = true;  // predicted to converge at this check
    if (alone) {
      if (const int st = update_alone(it - 1, fuse, stop)) return finish(st);
      if (stop) {  // an ended solve does not need the probed update
        r_pending = false;
        break;
      }
    }
    int st = vcycle<T>(P, (flex && it > 0) ? q : nullptr, s,
                       [&](CoarseMGArgs<T>* carrier) { return start_x(true, carrier); },
                       r_pending ? &ur : nullptr,
                       [&](bool& stop_) -> int {
                         if (!r_pending) return BCM_OK;
                         r_pending = false;
                         if (probed) {  // checked already
                           probed = false;
                           return BCM_OK;
                         }
                         return check(it - 1, nparts, stop_);
                       },
                       stop);
    if (st) return finish(st);
    if (stop) break;
    if ((st = finalize(P, OP_ZRZQ, 0, (flex && it > 0) ? 1 : -1, nparts, !fcg || it == 0, s))) return finish(st);
    if ((st = join_x())) return finish(st);
    ApplyArgs<T> aa{geom(P, NL), z, P->at<T>(P->o_zf[1]), p, P->at<T>(P->o_pfk[P->pf_cur]),
                    P->at<T>(P->o_pfk[P->pf_cur ^ 1]), q, P->at<const Scalars>(P->o_sc),
                    (!fcg || it == 0) ? 1 : 0, P->at<double>(P->o_part[2])};
    HIPCHK(timed(P, cls_of("apply", NL), s, [&] { return launch_apply<T>(NL, aa, s); }), "kc_apply");
    P->pf_cur ^= 1;
    if ((st = finalize(P, OP_PQ, 2, -1, nparts, 0, s))) return finish(st);
    if (!fcg) {  // stationary iteration: x += z, r -= A z  (alpha = 1)
      if ((st = finalize(P, OP_PQ, 0, -1, nparts, 0, s))) return finish(st);  // alpha = zr / zr
    }
    ur = UpdateArgs<T>{P->at<const CubeMeta>(P->o_meta), P->nc, NL * NL * NL, x, p, r, q,
                       P->at<const Scalars>(P->o_sc), P->at<double>(P->o_part[0]), x_zero && it == 0, 1};
    r_pending = true;
    ux = ur;
    ux.part_sel = 2;
    pending = true;
  }
  if (r_pending) {  // the last iteration's check (r itself is not needed any more)
    bool stop = false;
    if (const int st = update_alone(max_iter - 1, true, stop)) return finish(st);
  }
  return finish(BCM_OK);
}

// True FP64 residual of p (faces exported first unless they are current): <r,r>_V (and
// <b,b>_V) into the scalars.
template <typename TO>
int residual64(bcm_plan* P, const double* p, const double* b, TO* r, double rscale, hipStream_t s,
               bool faces_current = false) {
  const int NL = P->n;
  if (p && !faces_current) {
    int st = export64(P, const_cast<double*>(p), P->at<double>(P->o_pf), s);
    if (st) return st;
  }
  Resid64Args<TO> ra{geom(P, NL), p, P->at<const double>(P->o_pf), b, r,
                     P->at<double>(P->o_part[0]), P->at<double>(P->o_part[1]), rscale};
  HIPCHK(timed(P, cls_of("resid64", 0), s, [&] { return launch_resid64<TO>(NL, ra, s); }), "kc_resid64");
  return finalize(P, OP_BB, 0, 1, partials_of(NL, P->nc), 0, s);
}

constexpr double kFp64Floor = 64 * 2.220446049250313e-16;  // relative residual FP64 can reach

// Solve A p = b to opts.tol (relative, V-weighted, FP64).  p holds the guess if use_guess.
// Every return path reports the true FP64 residual of the returned p: a pass that updated p
// after the last residual evaluation (the limits were reached) is followed by one more
// evaluation.  The solve stops early with BCM_STAGNATED when a whole FP64 Krylov pass fails to
// halve the true residual norm, or two refinement steps in a row fail to (mixed).
int poisson(bcm_plan* P, const double* b, double* p, bool use_guess, bcm_report* rep, hipStream_t s) {
  const bcm_solver_opts& o = P->o;
  SolveLog log{rep};
  if (rep) rep->history_len = 0;
  Scalars hs{};
  int st = BCM_OK;
  int outer = 0;
  bool faces_ok = false;  // the face buffer holds the faces of the current p
  // Without a guess p starts at zero.  The mixed path never reads p before its first
  // refinement update, which then writes p = d instead of adding d to a zero-filled p; an exit
  // before that update fills p (p_unwritten).
  bool p_unwritten = !use_guess && P->inner32;
  if (!use_guess && !P->inner32) HIPCHK(fill<double>(p, P->cells, s), "zero fill");
  auto fail = [&](int e) {
    if (p_unwritten && fill<double>(p, P->cells, s) == hipSuccess) p_unwritten = false;
    return e;
  };
  double bb = 0.0, rr = 0.0;
  const double tol2 = o.tol * o.tol;
  bool converged = false, stagnated = false;
  bool unchecked = false;  // p changed since rr was evaluated
  auto nonfinite = [&]() {
    set_error("non-finite right-hand side or residual");
    return BCM_ERR_NONFINITE;
  };
  if (!P->inner32) {
    // FP64: flexible CG directly on p, restarted from the true residual if the recurrence
    // residual and the true one disagree at the end.
    double rr_prev = HUGE_VAL;
    for (outer = 0; outer < std::max(1, o.max_outer); ++outer) {
      if ((st = residual64<double>(P, p, b, P->at<double>(P->o_r), 1.0, s))) return st;
      if ((st = read_scalars(P, &hs, s))) return st;
      unchecked = false;
      bb = hs.bb;
      rr = hs.rr;
      if (!std::isfinite(rr) || !std::isfinite(bb)) return nonfinite();
      if (bb == 0.0) {
        HIPCHK(fill<double>(p, P->cells, s), "zero fill");
        rr = 0.0;
        converged = true;
        break;
      }
      log.push(std::sqrt(rr / bb));
      if (rr <= tol2 * bb) {
        converged = true;
        break;
      }
      if (outer > 0 && rr > 0.25 * rr_prev) {  // a whole Krylov pass did not halve it
        stagnated = true;
        break;
      }
      rr_prev = rr;
      if (log.iters >= o.max_iter) break;
      // the recurrence residual is not asked to go below what FP64 can resolve: a tolerance
      // under that floor ends in a restart whose true residual shows the stagnation
      const double thr = std::max(tol2 * 0.25, kFp64Floor * kFp64Floor) * bb;
      if ((st = krylov<double>(P, p, false, thr, o.max_iter - log.iters, 1.0 / std::sqrt(bb), log, &hs, s)))
        return st;
      unchecked = true;
    }
    if (unchecked) {  // the last restart's update has not been evaluated yet
      if ((st = residual64<double>(P, p, b, P->at<double>(P->o_r), 1.0, s))) return st;
      if ((st = read_scalars(P, &hs, s))) return st;
      rr = hs.rr;
      if (!std::isfinite(rr)) return nonfinite();
      log.push(std::sqrt(rr / bb));
      converged = rr <= tol2 * bb;
    }
  } else {
    // Mixed: FP64 residual and update, FP32 inner flexible CG.  The residual handed to the
    // inner solve is scaled to unit RMS (by the predicted norm) so FP32 range never matters.
    const double vol = double(P->cells);
    double rscale = 1.0, rr_prev = HUGE_VAL;
    int slow = 0;  // consecutive refinement steps that did not halve the residual norm
    for (outer = 0; outer < o.max_outer; ++outer) {
      float* r32 = P->at<float>(P->o_r);
      const double* pg = (use_guess || outer) ? p : nullptr;
      if ((st = residual64<float>(P, pg, b, r32, rscale, s, faces_ok))) return fail(st);
      faces_ok = pg != nullptr;
      if ((st = read_scalars(P, &hs, s))) return fail(st);
      unchecked = false;
      if (outer == 0) bb = hs.bb;
      rr = hs.rr;
      if (!std::isfinite(rr) || !std::isfinite(bb)) return fail(nonfinite());
      if (bb == 0.0) {
        HIPCHK(fill<double>(p, P->cells, s), "zero fill");
        p_unwritten = false;
        faces_ok = false;
        rr = 0.0;
        converged = true;
        break;
      }
      log.push(std::sqrt(rr / bb));
      if (rr <= tol2 * bb) {
        converged = true;
        break;
      }
      slow = rr > 0.25 * rr_prev ? slow + 1 : 0;
      if (slow >= 2) {
        stagnated = true;
        break;
      }
      rr_prev = rr;
      if (outer == 0 && !(rscale > 0 && std::fabs(std::log10(rr / vol)) < 20)) {
        // first pass unscaled and far from unit size: redo the conversion with the true norm
        rscale = 1.0 / std::sqrt(rr / vol);
        if ((st = residual64<float>(P, pg, b, r32, rscale, s, faces_ok))) return fail(st);
      }
      float* d = P->at<float>(P->o_d);
      // reduce the residual by inner_tol, or only by what is still missing to reach tol
      // (with a factor 0.3 of margin), whichever is the weaker requirement
      const double need = 0.3 * o.tol * std::sqrt(bb / rr);
      const double red_target = std::max(o.inner_tol, std::min(need, 0.1));
      const double thr = red_target * red_target * rr * rscale * rscale;
      UpdateArgs<float> last{};  // the inner solve's last x update, folded into kc_ir
      if ((st = krylov<float>(P, d, true, thr, o.max_iter, 1.0 / (rscale * std::sqrt(bb)), log, &hs, s,
                              &last)))
        return fail(st);
      IrArgs<float> ia{geom(P, P->n), p, d, P->at<double>(P->o_pf), 1.0 / rscale, p_unwritten ? 1 : 0,
                       last.p, last.sc, last.p ? last.x_zero : 0};
      HIPCHK(timed(P, cls_of("ir", 0), s, [&] { return launch_ir<float>(P->n, ia, s); }), "kc_ir");
      p_unwritten = false;
      faces_ok = true;  // kc_ir exports the faces of the updated p
      unchecked = true;
      const double rr_est = hs.rr / (rscale * rscale);
      if (rr_est > 0 && std::isfinite(rr_est)) rscale = 1.0 / std::sqrt(rr_est / vol);
    }
    if (p_unwritten) {  // converged without a refinement step (a tolerance of 1 or more)
      HIPCHK(fill<double>(p, P->cells, s), "zero fill");
      p_unwritten = false;
    }
    if (unchecked) {  // the last refinement step has not been evaluated yet
      if ((st = residual64<float>(P, p, b, P->at<float>(P->o_r), rscale, s, faces_ok))) return st;
      if ((st = read_scalars(P, &hs, s))) return st;
      rr = hs.rr;
      if (!std::isfinite(rr)) return nonfinite();
      log.push(std::sqrt(rr / bb));
      converged = rr <= tol2 * bb;
    }
  }
  const int status = converged ? BCM_OK : stagnated ? BCM_STAGNATED : BCM_NOT_CONVERGED;
  if (rep) {
    rep->n_outer = outer;
    rep->n_inner = log.iters;
    rep->final_rel_res = bb > 0 ? std::sqrt(std::max(rr, 0.0) / bb) : 0.0;
    rep->status = status;
  }
  // leave the faces of p exported for the correction kernels
  if (!faces_ok && (st = export64(P, p, P->at<double>(P->o_pf), s))) return st;
  return status;
}

// Forcing -> right-hand side -> Poisson -> correction (or, with p_given, forcing and
// correction only).
template <typename TF>
int project_impl(bcm_plan* P, const bcm_project_in* in, bcm_project_out* out, bcm_report* rep,
                 hipStream_t s, const double* p_given) {
  const int NL = P->n;
  const double c = in->dt / in->rho;
  ForceArgs<TF> fa{};
  fa.g = geom(P, NL);
  fa.alpha = static_cast<const TF*>(in->alpha);
  for (int d = 0; d < 3; ++d) {
    fa.u[d] = static_cast<const TF*>(in->u[d]);
    fa.us[d] = static_cast<const TF*>(in->us[d]);
    fa.usc[d] = in->us_const[d];
    fa.ustar[d] = P->at<TF>(P->o_ustar[d]);
  }
  fa.uf = P->at<TF>(P->o_uf);
  // 16^3 kernels: force and store u* only in cubes that hold some alpha != 0; the others pass
  // u~ on (the face-velocity output needs the generic correction, which reads u* everywhere)
  const bool sel = NL == 16 && !out->face_u[0] && !out->face_u[1] && !out->face_u[2];
  fa.body = sel ? P->at<uint8_t>(P->o_body) : nullptr;
  HIPCHK(timed(P, cls_of("force", 0), s, [&] { return launch_force<TF>(NL, fa, s); }), "k_force");
  double* p = out->p;
  int st = BCM_OK;
  if (!p_given) {
    DivArgs<TF> da{};
    da.g = geom(P, NL);
    for (int d = 0; d < 3; ++d) {
      da.ustar[d] = fa.ustar[d];
      da.u[d] = fa.u[d];
    }
    da.body = fa.body;
    da.uf = fa.uf;
    da.U_in = in->U_in;
    da.inv_c = 1.0 / c;
    da.b = P->at<double>(P->o_b64);
    HIPCHK(timed(P, cls_of("div", 0), s, [&] { return launch_div<TF>(NL, da, s); }), "k_div");
    bool guess = false;
    if (in->p0) {
      if (in->p0 != p)
        HIPCHK(hipMemcpyAsync(p, in->p0, P->cells * sizeof(double), hipMemcpyDeviceToDevice, s), "copy p0");
      guess = true;
    }
    st = poisson(P, P->at<const double>(P->o_b64), p, guess, rep, s);
    if (st < 0) return st;
    if (out->b)
      HIPCHK(hipMemcpyAsync(out->b, P->at<const double>(P->o_b64), P->cells * sizeof(double),
                            hipMemcpyDeviceToDevice, s), "copy b");
  } else {
    p = const_cast<double*>(p_given);
    int e = export64(P, p, P->at<double>(P->o_pf), s);
    if (e) return e;
  }
  CorrectArgs<TF> ca{};
  ca.g = geom(P, NL);
  ca.p = p;
  ca.pf = P->at<const double>(P->o_pf);
  for (int d = 0; d < 3; ++d) {
    ca.ustar[d] = fa.ustar[d];
    ca.u[d] = fa.u[d];
    ca.unew[d] = static_cast<TF*>(out->u_new[d]);
    ca.face_u[d] = static_cast<TF*>(out->face_u[d]);
  }
  ca.uf = fa.uf;
  ca.body = fa.body;
  ca.U_in = in->U_in;
  ca.c = c;
  HIPCHK(timed(P, cls_of("correct", 0), s, [&] { return launch_correct<TF>(NL, ca, s); }), "k_correct");
  return st;
}

// Adjoint of project_impl: g_p = -c G^T G_c^T g_u (+ g_p); lam = V A^{-1} (g_p / V);
// g_u* = g_u + (1/c) W^T D^T lam; g_u~ = (1 - alpha) g_u*; g_alpha; g_U_in.
template <typename TF>
int adjoint_impl(bcm_plan* P, const bcm_adjoint_in* in, bcm_adjoint_out* out, bcm_report* rep,
                 hipStream_t s) {
  const int NL = P->n;
  const double c = in->dt / in->rho;
  TF* vf = P->at<TF>(P->o_uf);
  ExportArgs<TF, TF> ea{};
  ea.g = geom(P, NL);
  ea.xf = vf;
  ea.comp_faces = 1;
  for (int d = 0; d < 3; ++d) ea.x3[d] = static_cast<const TF*>(in->g_u_new[d]);
  HIPCHK(timed(P, cls_of("export", 0), s, [&] { return launch_export<TF, TF>(NL, ea, s); }), "export g_u faces");
  AdjGpArgs<TF> ga{};
  ga.g = geom(P, NL);
  for (int d = 0; d < 3; ++d) ga.v[d] = ea.x3[d];
  ga.vf = vf;
  ga.gp_in = in->g_p;
  ga.c = c;
  ga.out = P->at<double>(P->o_b64);
  HIPCHK(timed(P, cls_of("adj_gp", 0), s, [&] { return launch_adj_gp<TF>(NL, ga, s); }), "k_adj_gp");
  double* lam = P->at<double>(P->o_lam);
  int st = poisson(P, P->at<const double>(P->o_b64), lam, false, rep, s);
  if (st < 0) return st;
  if (P->M->multilevel) {
    ScaleArgs sa{P->at<const CubeMeta>(P->o_meta), P->nc, NL * NL * NL, lam, lam, +1};
    HIPCHK(launch_scale(sa, s), "k_scale");
  }
  int e = export64(P, lam, P->at<double>(P->o_pf), s);
  if (e) return e;
  AdjRhsArgs<TF> ra{};
  ra.g = geom(P, NL);
  ra.lam = lam;
  ra.lamf = P->at<const double>(P->o_pf);
  ra.alpha = static_cast<const TF*>(in->alpha);
  for (int d = 0; d < 3; ++d) {
    ra.gun[d] = ea.x3[d];
    ra.u[d] = static_cast<const TF*>(in->u[d]);
    ra.us[d] = static_cast<const TF*>(in->us[d]);
    ra.usc[d] = in->us_const[d];
    ra.gu[d] = static_cast<TF*>(out->g_u[d]);
  }
  ra.galpha = static_cast<TF*>(out->g_alpha);
  ra.accumulate = out->accumulate != 0;
  ra.inv_c = 1.0 / c;
  ra.part_gU = P->at<double>(P->o_part[0]);
  HIPCHK(timed(P, cls_of("adj_rhs", 0), s, [&] { return launch_adj_rhs<TF>(NL, ra, s); }), "k_adj_rhs");
  if ((e = finalize(P, OP_GU, 0, -1, n_wg(NL, P->nc), 0, s))) return e;
  Scalars hs{};
  if ((e = read_scalars(P, &hs, s))) return e;
  out->g_U_in = (out->accumulate ? out->g_U_in : 0.0) + hs.gU;
  if (out->lambda)
    HIPCHK(hipMemcpyAsync(out->lambda, lam, P->cells * sizeof(double), hipMemcpyDeviceToDevice, s), "copy lambda");
  return st;
}

// J = (rho/2) sum_i V_i |u_i|^2 and the seed cotangent g_scale rho V_i u_i.
template <typename TF>
int kinetic_impl(bcm_plan* P, const void* const u[3], double rho, double g_scale, double* J,
                 void* const g_u[3], hipStream_t s) {
  KineticArgs<TF> ka{};
  ka.meta = P->at<const CubeMeta>(P->o_meta);
  ka.n_cubes = P->nc;
  ka.n3 = P->n * P->n * P->n;
  for (int d = 0; d < 3; ++d) {
    ka.u[d] = static_cast<const TF*>(u[d]);
    ka.gu[d] = g_u ? static_cast<TF*>(g_u[d]) : nullptr;
  }
  ka.gscale = g_scale * rho;
  const int grid = std::min(P->nc, 2048);  // the partial buffers hold >= n_cubes values
  ka.part = J ? P->at<double>(P->o_part[0]) : nullptr;
  HIPCHK(launch_kinetic<TF>(ka, grid, s), "k_kinetic");
  if (!J) return BCM_OK;
  if (int e = finalize(P, OP_VUU, 0, -1, grid, 0, s)) return e;
  Scalars hs{};
  if (int e = read_scalars(P, &hs, s)) return e;
  if (!std::isfinite(hs.vuu)) {
    set_error("bcm_kinetic_energy: non-finite velocity");
    return BCM_ERR_NONFINITE;
  }
  *J = 0.5 * rho * hs.vuu;
  return BCM_OK;
}

// Momentum sub-step (Eq. (substep1)): export the two-layer faces of u^n, then one explicit pass
// (Euler, AB2) or the Crank-Nicolson start and its Jacobi iterations, which alternate between
// the caller's output and the plan's second iterate.
template <typename TF>
int momentum_impl(bcm_plan* P, const bcm_momentum_in* in, bcm_momentum_out* out, bcm_report* rep,
                  hipStream_t s) {
  const int NL = P->n, nc = P->nc;
  const int units = nc;  // cubes or groups of cubes; the grid never exceeds the partial buffers
  const int grid = std::min(units, 2048);
  MomExportArgs<TF> ea{};
  ea.n_cubes = nc;
  for (int d = 0; d < 3; ++d) {
    ea.x[d] = static_cast<const TF*>(in->u[d]);
    ea.xf[d] = P->at<TF>(P->o_mfa[d]);
  }
  HIPCHK(timed(P, cls_of("momentum_start", 0), s, [&] { return launch_mom_export<TF>(NL, ea, grid, s); }),
         "k_mom_export");
  MomArgs<TF> ma{};
  ma.meta = P->at<const CubeMeta>(P->o_meta);
  ma.n_cubes = nc;
  for (int d = 0; d < 3; ++d) {
    ma.v[d] = static_cast<const TF*>(in->u[d]);
    ma.vf[d] = P->at<const TF>(P->o_mfa[d]);
    ma.a[d] = static_cast<const TF*>(in->u[d]);
    ma.af[d] = P->at<const TF>(P->o_mfa[d]);
    ma.hprev[d] = static_cast<const TF*>(in->h_prev[d]);
    ma.rhs[d] = P->at<TF>(P->o_mrhs[d]);
    ma.out[d] = static_cast<TF*>(out->u_tilde[d]);
    ma.hout[d] = static_cast<TF*>(out->h[d]);
  }
  ma.U_in = in->U_in;
  ma.nu = in->nu;
  ma.dt = in->dt;
  SolveLog log{rep};
  if (rep) rep->history_len = 0;
  auto launch = [&](int mode) {  // timer class "momentum": the passes over H (explicit step or
                                 // Crank-Nicolson sweep); "momentum_start": export and CN start
    const int cls = cls_of(mode == MOM_CN_START ? "momentum_start" : "momentum", 0);
    return timed(P, cls, s, [&] { return launch_mom<TF>(NL, mode, ma, grid, s); });
  };
  if (in->scheme != BCM_CN) {
    const bool ab2 = in->scheme == BCM_AB2 && in->h_prev[0];
    ma.c1 = ab2 ? 1.5 : 1.0;
    ma.c2 = ab2 ? -0.5 : 0.0;
    if (!ab2)
      for (int d = 0; d < 3; ++d) ma.hprev[d] = nullptr;
    HIPCHK(launch(MOM_EXPLICIT), "k_mom (explicit)");
    if (rep) {
      rep->status = BCM_OK;
      rep->n_outer = 0;
      rep->n_inner = 0;
      rep->final_rel_res = 0.0;
    }
    return BCM_OK;
  }
  const double tol = in->cn_tol > 0 ? in->cn_tol : 1e-12;
  const int max_iter = in->cn_max_iter > 0 ? in->cn_max_iter : 200;
  // start: rhs = u^n + dt/2 H(u^n), first iterate (Euler predictor) into the caller's output
  for (int d = 0; d < 3; ++d) ma.outf[d] = P->at<TF>(P->o_mfv[0][d]);
  ma.part = P->at<double>(P->o_part[0]);
  HIPCHK(launch(MOM_CN_START), "k_mom (Crank-Nicolson start)");
  if (int e = finalize(P, OP_B0, 0, -1, grid, 0, s)) return e;
  for (int d = 0; d < 3; ++d) ma.hout[d] = nullptr;
  TF* bufs[2][3];
  for (int d = 0; d < 3; ++d) {
    bufs[0][d] = static_cast<TF*>(out->u_tilde[d]);
    bufs[1][d] = P->at<TF>(P->o_mit[d]);
  }
  Scalars hs{};
  double bb = 0.0, rr = 0.0;
  bool converged = false;
  int cur = 0, it = 0;
  for (it = 0; it < max_iter; ++it) {
    for (int d = 0; d < 3; ++d) {
      ma.v[d] = bufs[cur][d];
      ma.vf[d] = P->at<const TF>(P->o_mfv[cur][d]);
      ma.out[d] = bufs[cur ^ 1][d];
      ma.outf[d] = P->at<TF>(P->o_mfv[cur ^ 1][d]);
    }
    HIPCHK(launch(MOM_CN_ITER), "k_mom (Crank-Nicolson iteration)");
    cur ^= 1;
    if (int e = finalize(P, OP_RR, 0, -1, grid, 0, s)) return e;
    log.iters++;
    if ((it + 1) % P->o.check_every != 0 && it + 1 < max_iter) continue;
    if (int e = read_scalars(P, &hs, s)) return e;
    bb = hs.bb;
    rr = hs.rr;
    if (!std::isfinite(rr) || !std::isfinite(bb)) {
      set_error("bcm_momentum: non-finite residual of the Crank-Nicolson iteration");
      return BCM_ERR_NONFINITE;
    }
    const double rel = bb > 0 ? std::sqrt(rr / bb) : 0.0;
    log.push(rel);
    if (rr <= tol * tol * bb) {
      converged = true;
      ++it;
      break;
    }
  }
  if (cur == 1)  // the last iterate is in the plan's buffer
    for (int d = 0; d < 3; ++d)
      HIPCHK(hipMemcpyAsync(out->u_tilde[d], bufs[1][d], P->cells * sizeof(TF), hipMemcpyDeviceToDevice, s),
             "copy iterate");
  const int status = converged ? BCM_OK : BCM_NOT_CONVERGED;
  if (rep) {
    rep->status = status;
    rep->n_outer = 0;
    rep->n_inner = log.iters;
    rep->final_rel_res = bb > 0 ? std::sqrt(std::max(rr, 0.0) / bb) : 0.0;
  }
  return status;
}

// Lagrangian-particle forcing: u* = u~, then every particle adds its spread constraint force.
template <typename TF>
int ib_force_impl(bcm_plan* P, const bcm_particles* pt, const void* const u_tilde[3], void* const u_star[3],
                  double dt, double rho, double* Up, double* Fp, hipStream_t s) {
  IbArgs<TF> a{};
  a.meta = P->at<const CubeMeta>(P->o_meta);
  a.n_cubes = P->nc;
  a.n = P->n;
  a.table = P->at<const int32_t>(P->o_ibtab);
  a.n_levels = int(P->ib_levels.size());
  for (int l = 0; l < a.n_levels; ++l) a.lev[l] = P->ib_levels[l];
  for (int d = 0; d < 3; ++d) {
    a.anchor[d] = P->ib_anchor[d];
    a.usc[d] = pt->us_const[d];
    a.u[d] = static_cast<const TF*>(u_tilde[d]);
    a.ustar[d] = static_cast<TF*>(u_star[d]);
    HIPCHK(hipMemcpyAsync(u_star[d], u_tilde[d], P->cells * sizeof(TF), hipMemcpyDeviceToDevice, s), "copy u~");
  }
  a.n_particles = pt->n;
  a.X = pt->X;
  a.dV = pt->dV;
  a.Us = pt->Us;
  a.rho_dt = rho / dt;
  a.dt_rho = dt / rho;
  a.Up = Up;
  a.Fp = Fp;
  a.errors = P->at<unsigned int>(P->o_iberr);
  HIPCHK(launch_zero_u32(a.errors, s), "zero the skip counter");
  HIPCHK(timed(P, cls_of("ib", 0), s, [&] { return launch_ib_force<TF>(a, s); }), "k_ib_force");
  unsigned int skipped = 0;
  HIPCHK(hipMemcpyAsync(&skipped, a.errors, sizeof(skipped), hipMemcpyDeviceToHost, s), "skip counter readback");
  HIPCHK(hipStreamSynchronize(s), "stream synchronize");
  if (skipped) {
    set_error("bcm_ib_force: " + std::to_string(skipped) +
              " particles skipped (outside the mesh, or their 3x3x3 support leaves their cube's level"
              " or the domain); u_star holds the forcing of the others");
    return BCM_ERR_INVALID_ARG;
  }
  return BCM_OK;
}

// Wavelet codec: header bytes, the worst case of a cube's stream, transform levels.
size_t codec_header_bytes(const bcm_plan* P) { return 32 + 8 * (size_t(P->nc) + 1); }
size_t codec_cube_bound(int n) {
  const size_t G = size_t(n) * n * n / 32;
  return (G + 3) / 4 * 4 + 4 * 32 * G;
}
int codec_levels(int n) { return n == 16 ? 4 : n == 8 ? 3 : 2; }

CodecArgs codec_args(bcm_plan* P, double step) {
  CodecArgs a{};
  a.n_cubes = P->nc;
  a.n = P->n;
  a.levels = codec_levels(P->n);
  a.step = step;
  a.codes = P->at<uint32_t>(P->o_r);   // the Krylov vectors are free between solves
  a.widths = P->at<uint8_t>(P->o_z);
  a.sizes = P->at<unsigned long long>(P->o_part[1]);
  a.total = P->at<unsigned long long>(P->o_cflag);
  a.flags = reinterpret_cast<unsigned int*>(P->at<char>(P->o_cflag) + 8);
  return a;
}

// ---- no-allocation variant of the kinetic-energy objective --------------------------------
// Its scratch (the per-workgroup partial sums and the scalar block of the final sum) lives in a
// file-scope device array instead of the plan's workspace.  Every GPU that runs it holds its own
// copy of the array until the process ends; host code reaches a device's copy only through the
// address hipGetSymbolAddress returns with that device current (kept per device below), never
// through the array's name.
constexpr int kNoAllocParts = 2048;  // partial sums (the objective's grid never exceeds it)
constexpr size_t kNoAllocBytes = kNoAllocParts * sizeof(double) + sizeof(Scalars);
__device__ __align__(256) unsigned char scratch[kNoAllocBytes];

constexpr int kMaxDevices = 64;
std::mutex g_scratch_mu;
void* g_scratch_ptr[kMaxDevices] = {};

// Device address of this device's scratch array (looked up once per device).
int scratch_address(void** out) {
  int dev = 0;
  HIPCHK(hipGetDevice(&dev), "hipGetDevice");
  if (dev < 0 || dev >= kMaxDevices) {
    set_error("bcm_kinetic_energy_noalloc: device index beyond the supported 64");
    return BCM_ERR_UNSUPPORTED;
  }
  std::lock_guard<std::mutex> lock(g_scratch_mu);
  if (!g_scratch_ptr[dev]) {
    void* p = nullptr;
    HIPCHK(hipGetSymbolAddress(&p, HIP_SYMBOL(scratch)), "hipGetSymbolAddress(scratch)");
    g_scratch_ptr[dev] = p;
  }
  *out = g_scratch_ptr[dev];
  return BCM_OK;
}

template <typename TF>
int kinetic_noalloc_impl(bcm_plan* P, const void* const u[3], double rho, double g_scale, double* J,
                         void* const g_u[3], hipStream_t s) {
  void* base = nullptr;
  if (int e = scratch_address(&base)) return e;
  double* part = static_cast<double*>(base);
  Scalars* sc = reinterpret_cast<Scalars*>(static_cast<char*>(base) + kNoAllocParts * sizeof(double));
  KineticArgs<TF> ka{};
  ka.meta = P->at<const CubeMeta>(P->o_meta);
  ka.n_cubes = P->nc;
  ka.n3 = P->n * P->n * P->n;
  for (int d = 0; d < 3; ++d) {
    ka.u[d] = static_cast<const TF*>(u[d]);
    ka.gu[d] = g_u ? static_cast<TF*>(g_u[d]) : nullptr;
  }
  ka.gscale = g_scale * rho;
  const int grid = std::min(P->nc, 2048);  // the same grid as bcm_kinetic_energy
  if (grid > kNoAllocParts) {
    set_error("bcm_kinetic_energy_noalloc: more partial sums than the scratch array holds");
    return BCM_ERR_UNSUPPORTED;
  }
  ka.part = J ? part : nullptr;
  HIPCHK(launch_kinetic<TF>(ka, grid, s), "k_kinetic");
  if (!J) return BCM_OK;
  FinalizeArgs fa{part, nullptr, grid, sc, OP_VUU, 0, nullptr, 0u};
  HIPCHK(launch_finalize(fa, s), "k_finalize");
  double vuu = 0.0;
  HIPCHK(hipMemcpyAsync(&vuu, &sc->vuu, sizeof(double), hipMemcpyDeviceToHost, s), "objective readback");
  HIPCHK(hipStreamSynchronize(s), "stream synchronize");
  if (!std::isfinite(vuu)) {
    set_error("bcm_kinetic_energy_noalloc: non-finite velocity");
    return BCM_ERR_NONFINITE;
  }
  *J = 0.5 * rho * vuu;
  return BCM_OK;
}

// Upload the cube-graph hierarchy (converted to the inner precision T) and its level table.
template <typename T>
int upload_graph(bcm_plan* P, hipStream_t s) {
  const auto& Ls = P->M->coarse.levels;
  std::vector<std::vector<T>> keep;
  std::vector<GLevel<T>> lev(Ls.size());
  auto put = [&](size_t off, const void* src, size_t bytes) -> hipError_t {
    if (bytes == 0) return hipSuccess;
    return hipMemcpyAsync(P->ws + off, src, bytes, hipMemcpyHostToDevice, s);
  };
  auto conv = [&](const std::vector<double>& v) -> const std::vector<T>& {
    keep.emplace_back(v.begin(), v.end());
    return keep.back();
  };
  keep.reserve(4 * Ls.size() + 1);
  for (size_t g = 0; g < Ls.size(); ++g) {
    const CoarseLevel& L = Ls[g];
    const bcm_plan::GOff& o = P->g_off[g];
    HIPCHK(put(o.col, L.e_col.data(), L.e_col.size() * 4), "upload graph columns");
    HIPCHK(put(o.val, conv(L.e_val).data(), L.e_val.size() * sizeof(T)), "upload graph values");
    HIPCHK(put(o.diag, conv(L.e_diag).data(), L.e_diag.size() * sizeof(T)), "upload graph diagonal");
    HIPCHK(put(o.vol, conv(L.e_vol).data(), L.e_vol.size() * sizeof(T)), "upload graph volumes");
    HIPCHK(put(o.parent, L.e_parent.data(), L.e_parent.size() * 4), "upload graph parents");
    if (!L.e_pcol.empty())
      HIPCHK(put(o.pcol, L.e_pcol.data(), L.e_pcol.size() * 4), "upload packed graph columns");
    if (g > 0) {
      HIPCHK(put(o.child, L.e_child.data(), L.e_child.size() * 4), "upload graph children");
      HIPCHK(put(o.child_w, conv(L.e_child_w).data(), L.e_child_w.size() * sizeof(T)), "upload graph weights");
    }
    GLevel<T>& d = lev[g];
    std::memset(&d, 0, sizeof(d));
    d.n = L.n;
    d.ncol = int(L.color_off.size()) - 1;
    d.W = L.W;
    d.CW = L.CW;
    for (int c = 0; c <= d.ncol; ++c) d.color_off[c] = L.color_off[c];
    d.lds_x = o.lds_x;
    d.lds_b = o.lds_b;
    d.lds_r = o.lds_r;
    d.col = P->at<const int32_t>(o.col);
    d.val = P->at<const T>(o.val);
    d.diag = P->at<const T>(o.diag);
    d.vol = P->at<const T>(o.vol);
    d.parent = L.e_parent.empty() ? nullptr : P->at<const int32_t>(o.parent);
    d.child = g > 0 ? P->at<const int32_t>(o.child) : nullptr;
    d.child_w = g > 0 ? P->at<const T>(o.child_w) : nullptr;
    d.x = P->at<T>(o.x);
    d.b = P->at<T>(o.b);
    d.r = P->at<T>(o.r);
    d.pcol = L.e_pcol.empty() ? nullptr : P->at<const uint32_t>(o.pcol);
    d.uval = T(L.uval);
  }
  HIPCHK(put(P->o_perm0, Ls[0].perm.data(), Ls[0].perm.size() * 4), "upload graph permutation");
  HIPCHK(put(P->o_ginv, conv(P->M->coarse.bottom_inv).data(), P->M->coarse.bottom_inv.size() * sizeof(T)),
         "upload bottom inverse");
  HIPCHK(put(P->o_glev, lev.data(), lev.size() * sizeof(GLevel<T>)), "upload graph levels");
  HIPCHK(hipStreamSynchronize(s), "stream synchronize");
  return BCM_OK;
}

int check_bound(const bcm_plan* P) {
  if (!P) {
    set_error("NULL plan");
    return BCM_ERR_INVALID_ARG;
  }
  if (!P->ws) {
    set_error("no workspace bound to the plan (bcm_plan_bind)");
    return BCM_ERR_WORKSPACE;
  }
  return BCM_OK;
}

}  // namespace

extern "C" {

void bcm_default_opts(bcm_solver_opts* o) {
  if (!o) return;
  o->precision = BCM_FP64;
  o->tol = 1e-10;
  o->max_iter = 50;
  o->max_outer = 10;
  o->inner_tol = 1e-3;
  o->pre_sweeps = 2;
  o->post_sweeps = 2;
  o->coarse_iters = 10;
  o->krylov = 1;
  o->coarse_solver = 1;
  o->coarse_cycles = 1;
  o->graph_split = -1;
  o->prolong = 1;
  o->check_every = 1;
}

int bcm_plan_create(const bcm_mesh* mesh, const bcm_solver_opts* opts, bcm_plan** out,
                    size_t* workspace_bytes) {
  if (!mesh || !out) {
    set_error("bcm_plan_create: NULL argument");
    return BCM_ERR_INVALID_ARG;
  }
  *out = nullptr;
  bcm_solver_opts o;
  if (opts)
    o = *opts;
  else
    bcm_default_opts(&o);
  if (o.precision < BCM_FP64 || o.precision > BCM_MIXED_F32FIELDS || !(o.tol > 0.0) || o.max_iter < 1 ||
      o.max_outer < 1 || !(o.inner_tol > 0.0 && o.inner_tol < 1.0) || o.pre_sweeps < 0 ||
      o.post_sweeps < 0 || o.coarse_iters < 0 || o.pre_sweeps > 16 || o.post_sweeps > 16 ||
      o.coarse_solver < 0 || o.coarse_solver > 1 || o.coarse_cycles < 1 || o.graph_split < -1 || o.krylov < 0 || o.krylov > 2 ||
      o.prolong < 0 || o.prolong > 1 || o.check_every < 1) {
    set_error("bcm_plan_create: invalid solver options");
    return BCM_ERR_INVALID_ARG;
  }
  auto* P = new (std::nothrow) bcm_plan;
  if (!P) {
    set_error("bcm_plan_create: out of host memory");
    return BCM_ERR_INVALID_ARG;
  }
  const HostMesh& M = mesh->m;
  P->M = &M;
  P->o = o;
  P->n = M.n;
  P->nc = M.n_cubes;
  P->nlev = 1;
  while ((M.n >> (P->nlev - 1)) > 1) P->nlev++;
  P->cells = size_t(M.n_cubes) * M.n * M.n * M.n;
  P->inner32 = o.precision != BCM_FP64;
  P->fields32 = o.precision == BCM_MIXED_F32FIELDS;
  const size_t Ti = P->inner32 ? 4 : 8, Tf = P->fields32 ? 4 : 8;
  const size_t nc = size_t(M.n_cubes), cells = P->cells;
  size_t top = 0;
  P->o_meta = take(top, nc * sizeof(CubeMeta));
  P->o_launch = take(top, nc * sizeof(int32_t));
  if (o.prolong == 1 && !M.nb27.empty()) P->o_nb27 = take(top, M.nb27.size() * sizeof(uint32_t));
  const size_t nparts = std::max(nc, size_t(partials_of(P->n, int(nc))));
  for (int i = 0; i < 3; ++i) P->o_part[i] = take(top, nparts * sizeof(double));
  P->o_sc = take(top, sizeof(Scalars));
  P->o_cw = take(top, 4 * nc * sizeof(double));
  for (int d = 0; d < 3; ++d) P->o_ustar[d] = take(top, cells * Tf);
  P->o_uf = take(top, size_t(face_stride(M.n)) * nc * Tf);
  P->o_body = take(top, nc);
  P->o_b64 = take(top, cells * 8);
  P->o_pf = take(top, size_t(face_stride(M.n)) * nc * 8);
  P->o_lam = take(top, cells * 8);
  P->o_r = take(top, cells * Ti);
  P->o_z = take(top, cells * Ti);
  P->o_p = take(top, cells * Ti);
  P->o_q = take(top, cells * Ti);
  P->o_d = P->inner32 ? take(top, cells * 4) : 0;
  for (int i = 0; i < 2; ++i) {
    P->o_zf[i] = take(top, size_t(face_stride(M.n)) * nc * Ti);
    P->o_pfk[i] = take(top, size_t(face_stride(M.n)) * nc * Ti);
  }
  P->o_x.assign(P->nlev, 0);
  P->o_b.assign(P->nlev, 0);
  P->o_xf[0].assign(P->nlev, 0);
  P->o_xf[1].assign(P->nlev, 0);
  for (int l = 1; l < P->nlev; ++l) {
    const size_t NL = size_t(M.n >> l);
    P->o_x[l] = take(top, nc * NL * NL * NL * Ti);
    P->o_b[l] = take(top, nc * NL * NL * NL * Ti);
    P->o_xf[0][l] = take(top, size_t(face_stride(int(NL))) * nc * Ti);
    P->o_xf[1][l] = take(top, size_t(face_stride(int(NL))) * nc * Ti);
  }
  P->momentum = !M.multilevel && M.n >= 4;
  if (P->momentum) {
    const size_t mfs = size_t(4) * M.n * M.n * nc * Tf;  // two x layers per face (kernels_mom.hip)
    for (int d = 0; d < 3; ++d) {
      P->o_mfa[d] = take(top, mfs);
      P->o_mfv[0][d] = take(top, mfs);
      P->o_mfv[1][d] = take(top, mfs);
      P->o_mrhs[d] = take(top, cells * Tf);
      P->o_mit[d] = take(top, cells * Tf);
    }
  }
  // point-location tables of the particle forcing: per level, a dense table over the bounding
  // box of its cubes on its lattice (skipped when a level's box exceeds 2^26 entries)
  {
    int lmin = 127, lmax = -1;
    for (int c = 0; c < int(nc); ++c) {
      lmin = std::min<int>(lmin, M.level[c]);
      lmax = std::max<int>(lmax, M.level[c]);
    }
    for (int d = 0; d < 3; ++d) P->ib_anchor[d] = HUGE_VAL;
    for (int c = 0; c < int(nc); ++c)
      if (M.level[c] == lmin)
        for (int d = 0; d < 3; ++d) P->ib_anchor[d] = std::min(P->ib_anchor[d], M.origin[3 * c + d]);
    bool ok = lmax >= 0 && lmax - lmin + 1 <= kIbMaxLevels;
    for (int L = lmax; L >= lmin && ok; --L) {
      IbLevel lv{};
      lv.level = L;
      lv.edge = M.root_edge / std::ldexp(1.0, L);
      int lo[3] = {INT32_MAX, INT32_MAX, INT32_MAX}, hi[3] = {INT32_MIN, INT32_MIN, INT32_MIN};
      bool any = false;
      for (int c = 0; c < int(nc); ++c) {
        if (M.level[c] != L) continue;
        any = true;
        for (int d = 0; d < 3; ++d) {
          const int q = int(std::lround((M.origin[3 * c + d] - P->ib_anchor[d]) / lv.edge));
          lo[d] = std::min(lo[d], q);
          hi[d] = std::max(hi[d], q);
        }
      }
      if (!any) continue;
      long long cnt = 1;
      for (int d = 0; d < 3; ++d) {
        lv.lo[d] = lo[d];
        lv.dims[d] = hi[d] - lo[d] + 1;
        cnt *= lv.dims[d];
      }
      if (cnt > (1LL << 26)) {
        ok = false;
        break;
      }
      lv.offset = (long long)P->ib_table.size();
      P->ib_table.resize(P->ib_table.size() + size_t(cnt), -1);
      for (int c = 0; c < int(nc); ++c) {
        if (M.level[c] != L) continue;
        int q[3];
        for (int d = 0; d < 3; ++d) q[d] = int(std::lround((M.origin[3 * c + d] - P->ib_anchor[d]) / lv.edge)) - lv.lo[d];
        P->ib_table[size_t(lv.offset + ((long long)q[2] * lv.dims[1] + q[1]) * lv.dims[0] + q[0])] = c;
      }
      P->ib_levels.push_back(lv);
    }
    P->ib = ok && !P->ib_levels.empty();
    if (P->ib) {
      P->o_ibtab = take(top, P->ib_table.size() * sizeof(int32_t));
      P->o_iberr = take(top, 256);
    } else {
      P->ib_table.clear();
      P->ib_levels.clear();
    }
  }
  P->o_cflag = take(top, 256);
  P->graph = o.coarse_solver == 1 && M.coarse.ok && !M.coarse.levels.empty();
  if (P->graph) {
    const auto& Ls = M.coarse.levels;
    for (size_t g = 0; g < Ls.size(); ++g) {
      const CoarseLevel& L = Ls[g];
      bcm_plan::GOff go{};
      const size_t n = size_t(L.n);
      go.col = take(top, L.e_col.size() * 4);
      go.val = take(top, L.e_val.size() * Ti);
      go.diag = take(top, n * Ti);
      go.vol = take(top, n * Ti);
      go.parent = take(top, std::max<size_t>(L.e_parent.size(), 1) * 4);
      if (g > 0) {
        go.child = take(top, L.e_child.size() * 4);
        go.child_w = take(top, L.e_child.size() * Ti);
      }
      go.x = take(top, n * Ti);
      go.b = take(top, n * Ti);
      go.r = take(top, n * Ti);
      go.pcol = L.e_pcol.empty() ? 0 : take(top, L.e_pcol.size() * 4);
      go.lds_x = go.lds_b = go.lds_r = -1;
      P->g_off.push_back(go);
    }
    // leading levels above o.graph_split nodes (automatic: those whose x, b and r do not fit
    // in the LDS budget) are smoothed by multi-workgroup kernels; never the last one, which
    // the single workgroup solves directly or by CG
    auto large = [&](int g) {
      return o.graph_split >= 0 ? Ls[g].n > o.graph_split
                                : size_t(3) * Ls[g].n * Ti > size_t(kGraphLdsBudget);
    };
    P->g_split = 0;
    while (P->g_split + 1 < int(Ls.size()) && large(P->g_split)) ++P->g_split;
    // LDS placement of the single workgroup's levels, smallest first: x, then b and r,
    // while the budget lasts
    int lds = 0;
    auto place = [&](int& slot, size_t n) {
      const int bytes = int((n * Ti + 15) / 16 * 16);
      if (lds + bytes <= kGraphLdsBudget) {
        slot = lds;
        lds += bytes;
      }
    };
    for (int g = int(Ls.size()) - 1; g >= P->g_split; --g) place(P->g_off[g].lds_x, Ls[g].n);
    for (int g = int(Ls.size()) - 1; g >= P->g_split; --g) {
      place(P->g_off[g].lds_b, Ls[g].n);
      place(P->g_off[g].lds_r, Ls[g].n);
    }
    // the bottom level's inverse too, when it fits beside them
    P->g_lds_inv = -1;
    if (!M.coarse.bottom_inv.empty()) {
      const int bytes = int((M.coarse.bottom_inv.size() * Ti + 15) / 16 * 16);
      if (lds + bytes <= kGraphLdsTotal) {
        P->g_lds_inv = lds;
        lds += bytes;
      }
    }
    P->g_lds = lds;
    P->o_glev = take(top, Ls.size() * sizeof(GLevel<double>));
    P->o_gw = take(top, 4 * size_t(Ls.back().n) * sizeof(double));
    P->o_perm0 = take(top, Ls[0].perm.size() * 4);
    P->o_ginv = take(top, M.coarse.bottom_inv.size() * sizeof(double));
  }
  P->ws_bytes = top;
  if (workspace_bytes) *workspace_bytes = top;
  *out = P;
  return BCM_OK;
}

void bcm_plan_destroy(bcm_plan* P) {
  if (!P) return;
  for (hipEvent_t e : P->timer.ev) (void)hipEventDestroy(e);
  if (P->mirror) (void)hipHostFree(P->mirror);
  if (P->ev_mid) (void)hipEventDestroy(P->ev_mid);
  if (P->ev_x) (void)hipEventDestroy(P->ev_x);
  if (P->s2) (void)hipStreamDestroy(P->s2);
  delete P;
}

int bcm_plan_bind(bcm_plan* P, void* d_ws, size_t bytes, void* stream) {
  if (!P || !d_ws) {
    set_error("bcm_plan_bind: NULL argument");
    return BCM_ERR_INVALID_ARG;
  }
  if (bytes < P->ws_bytes || (reinterpret_cast<uintptr_t>(d_ws) % kAlign) != 0) {
    set_error("bcm_plan_bind: workspace smaller than bcm_plan_create reported, or not 256-byte aligned");
    return BCM_ERR_WORKSPACE;
  }
  hipStream_t s = static_cast<hipStream_t>(stream);
  P->ws = static_cast<char*>(d_ws);
  const HostMesh& M = *P->M;
  HIPCHK(hipMemcpyAsync(P->ws + P->o_meta, M.meta.data(), M.meta.size() * sizeof(CubeMeta),
                        hipMemcpyHostToDevice, s), "upload cube metadata");
  HIPCHK(hipMemcpyAsync(P->ws + P->o_launch, M.launch.data(), M.launch.size() * sizeof(int32_t),
                        hipMemcpyHostToDevice, s), "upload launch order");
  if (P->o_nb27)
    HIPCHK(hipMemcpyAsync(P->ws + P->o_nb27, M.nb27.data(), M.nb27.size() * sizeof(uint32_t),
                          hipMemcpyHostToDevice, s), "upload 27-neighbourhoods");
  if (P->ib)
    HIPCHK(hipMemcpyAsync(P->ws + P->o_ibtab, P->ib_table.data(), P->ib_table.size() * sizeof(int32_t),
                          hipMemcpyHostToDevice, s), "upload point-location tables");
  HIPCHK(hipStreamSynchronize(s), "stream synchronize");
  if (!P->mirror) {
    // pinned, coherent host memory for the scalar mirror; without it the scalars are copied
    // back and the stream synchronised
    void* hm = nullptr;
    if (hipHostMalloc(&hm, sizeof(ScalarMirror), hipHostMallocMapped | hipHostMallocCoherent) == hipSuccess) {
      P->mirror = static_cast<ScalarMirror*>(hm);
      std::memset(hm, 0, sizeof(ScalarMirror));
      P->mirror_seq = 0;
    } else {
      (void)hipGetLastError();
    }
  }
  if (!P->s2) {
    // second stream (default priority) and its two events for the Krylov x updates; without
    // them the x updates stay on the caller's stream
    hipStream_t s2 = nullptr;
    hipEvent_t e1 = nullptr, e2 = nullptr;
    if (hipStreamCreateWithFlags(&s2, hipStreamNonBlocking) == hipSuccess &&
        hipEventCreateWithFlags(&e1, hipEventDisableTiming) == hipSuccess &&
        hipEventCreateWithFlags(&e2, hipEventDisableTiming) == hipSuccess) {
      P->s2 = s2;
      P->ev_mid = e1;
      P->ev_x = e2;
    } else {
      if (e1) (void)hipEventDestroy(e1);
      if (s2) (void)hipStreamDestroy(s2);
      (void)hipGetLastError();
    }
  }
  {
    // a carried vector update gets every CU but the coarse solve's (one workgroup per CU: the
    // launch reserves the coarse solve's LDS for each)
    int dev = 0, cus = 0;
    if (hipGetDevice(&dev) == hipSuccess &&
        hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev) == hipSuccess && cus > 1)
      P->side_wgs = cus - 1;
    else
      (void)hipGetLastError();
  }
  if (P->graph) return P->inner32 ? upload_graph<float>(P, s) : upload_graph<double>(P, s);
  return BCM_OK;
}

int bcm_project(bcm_plan* P, const bcm_project_in* in, bcm_project_out* out, bcm_report* rep,
                void* stream) {
  int st = check_bound(P);
  if (st) return st;
  if (!in || !out || !out->p || !in->u[0] || !in->u[1] || !in->u[2] || !(in->dt > 0) || !(in->rho > 0)) {
    set_error("bcm_project: NULL field or non-positive dt / rho");
    return BCM_ERR_INVALID_ARG;
  }
  hipStream_t s = static_cast<hipStream_t>(stream);
  st = P->fields32 ? project_impl<float>(P, in, out, rep, s, nullptr)
                   : project_impl<double>(P, in, out, rep, s, nullptr);
  if (rep) rep->status = st;
  return st;
}

int bcm_project_recompute(bcm_plan* P, const bcm_project_in* in, const double* d_p,
                          bcm_project_out* out, void* stream) {
  int st = check_bound(P);
  if (st) return st;
  if (!in || !out || !d_p || !in->u[0] || !in->u[1] || !in->u[2] || !(in->dt > 0) || !(in->rho > 0)) {
    set_error("bcm_project_recompute: NULL field or non-positive dt / rho");
    return BCM_ERR_INVALID_ARG;
  }
  hipStream_t s = static_cast<hipStream_t>(stream);
  return P->fields32 ? project_impl<float>(P, in, out, nullptr, s, d_p)
                     : project_impl<double>(P, in, out, nullptr, s, d_p);
}

int bcm_project_adjoint(bcm_plan* P, const bcm_adjoint_in* in, bcm_adjoint_out* out,
                        bcm_report* rep, void* stream) {
  int st = check_bound(P);
  if (st) return st;
  if (!in || !out || !in->u[0] || !in->u[1] || !in->u[2] || !in->g_u_new[0] || !in->g_u_new[1] ||
      !in->g_u_new[2] || !out->g_u[0] || !out->g_u[1] || !out->g_u[2] || !(in->dt > 0) ||
      !(in->rho > 0) || (in->alpha && !out->g_alpha)) {
    set_error("bcm_project_adjoint: NULL field or non-positive dt / rho");
    return BCM_ERR_INVALID_ARG;
  }
  hipStream_t s = static_cast<hipStream_t>(stream);
  st = P->fields32 ? adjoint_impl<float>(P, in, out, rep, s) : adjoint_impl<double>(P, in, out, rep, s);
  if (rep) rep->status = st;
  return st;
}

int bcm_momentum(bcm_plan* P, const bcm_momentum_in* in, bcm_momentum_out* out, bcm_report* rep,
                 void* stream) {
  int st = check_bound(P);
  if (st) return st;
  if (!in || !out || !in->u[0] || !in->u[1] || !in->u[2] || !out->u_tilde[0] || !out->u_tilde[1] ||
      !out->u_tilde[2] || !(in->dt > 0) || !(in->nu >= 0) || !std::isfinite(in->U_in) ||
      in->scheme < BCM_EULER || in->scheme > BCM_CN || in->cn_tol < 0 || in->cn_max_iter < 0 ||
      (in->h_prev[0] || in->h_prev[1] || in->h_prev[2]) != (in->h_prev[0] && in->h_prev[1] && in->h_prev[2]) ||
      (out->h[0] || out->h[1] || out->h[2]) != (out->h[0] && out->h[1] && out->h[2])) {
    set_error("bcm_momentum: NULL field, dt <= 0, nu < 0, unknown scheme or a partial field triple");
    return BCM_ERR_INVALID_ARG;
  }
  if (!P->momentum) {
    set_error("bcm_momentum: single-level meshes with n >= 4 only");
    return BCM_ERR_UNSUPPORTED;
  }
  for (int d = 0; d < 3; ++d)
    if (out->u_tilde[d] == in->u[d]) {
      set_error("bcm_momentum: u_tilde must not alias u");
      return BCM_ERR_INVALID_ARG;
    }
  hipStream_t s = static_cast<hipStream_t>(stream);
  st = P->fields32 ? momentum_impl<float>(P, in, out, rep, s) : momentum_impl<double>(P, in, out, rep, s);
  if (rep) rep->status = st;
  return st;
}

int bcm_kinetic_energy(bcm_plan* P, const void* const u[3], double rho, double g_scale, double* J,
                       void* const g_u[3], void* stream) {
  int st = check_bound(P);
  if (st) return st;
  if (!u || !u[0] || !u[1] || !u[2] || !(rho > 0) || !std::isfinite(g_scale) ||
      (g_u && (!g_u[0] || !g_u[1] || !g_u[2]))) {
    set_error("bcm_kinetic_energy: NULL field, non-positive rho or non-finite g_scale");
    return BCM_ERR_INVALID_ARG;
  }
  hipStream_t s = static_cast<hipStream_t>(stream);
  return P->fields32 ? kinetic_impl<float>(P, u, rho, g_scale, J, g_u, s)
                     : kinetic_impl<double>(P, u, rho, g_scale, J, g_u, s);
}

int bcm_ib_force(bcm_plan* P, const bcm_particles* pt, const void* const u_tilde[3], void* const u_star[3],
                 double dt, double rho, double* U_p, double* F_p, void* stream) {
  int st = check_bound(P);
  if (st) return st;
  if (!pt || !u_tilde || !u_star || pt->n < 0 || pt->n >= (1 << 26) || (pt->n > 0 && !pt->X) ||
      !(dt > 0) || !(rho > 0)) {
    set_error("bcm_ib_force: NULL argument, particle count negative or not below 2^26, or dt / rho "
              "not positive");
    return BCM_ERR_INVALID_ARG;
  }
  for (int d = 0; d < 3; ++d)
    if (!u_tilde[d] || !u_star[d] || u_tilde[d] == u_star[d]) {
      set_error("bcm_ib_force: NULL field, or u_star aliasing u_tilde");
      return BCM_ERR_INVALID_ARG;
    }
  if (!P->ib) {
    set_error("bcm_ib_force: no point-location tables for this mesh (a level's bounding box is too large)");
    return BCM_ERR_UNSUPPORTED;
  }
  hipStream_t s = static_cast<hipStream_t>(stream);
  return P->fields32 ? ib_force_impl<float>(P, pt, u_tilde, u_star, dt, rho, U_p, F_p, s)
                     : ib_force_impl<double>(P, pt, u_tilde, u_star, dt, rho, U_p, F_p, s);
}

int bcm_compress_bound(const bcm_plan* P, size_t* bytes) {
  if (!P || !bytes) {
    set_error("bcm_compress_bound: NULL argument");
    return BCM_ERR_INVALID_ARG;
  }
  if (P->n < 4) {
    set_error("bcm_compress_bound: the codec needs n >= 4");
    return BCM_ERR_UNSUPPORTED;
  }
  *bytes = codec_header_bytes(P) + size_t(P->nc) * codec_cube_bound(P->n);
  return BCM_OK;
}

int bcm_compress(bcm_plan* P, const double* d_field, double step, void* d_stream, size_t capacity,
                 size_t* bytes, void* stream) {
  int st = check_bound(P);
  if (st) return st;
  if (!d_field || !d_stream || !bytes || !(step > 0) || !std::isfinite(step) ||
      (reinterpret_cast<uintptr_t>(d_stream) % 8) != 0) {
    set_error("bcm_compress: NULL argument, step not positive and finite, or stream not 8-byte aligned");
    return BCM_ERR_INVALID_ARG;
  }
  if (P->n < 4) {
    set_error("bcm_compress: the codec needs n >= 4");
    return BCM_ERR_UNSUPPORTED;
  }
  const size_t head = codec_header_bytes(P);
  if (capacity < head) {
    *bytes = head;
    set_error("bcm_compress: stream buffer smaller than the header");
    return BCM_ERR_INVALID_ARG;
  }
  hipStream_t s = static_cast<hipStream_t>(stream);
  CodecArgs a = codec_args(P, step);
  a.field = d_field;
  a.stream = d_stream;
  const int grid = std::min(P->nc, 4096);
  HIPCHK(launch_zero_u32(a.flags, s), "zero the codec flags");
  HIPCHK(timed(P, cls_of("codec", 0), s, [&] { return launch_wc_encode(P->n, a, grid, s); }), "k_wc_encode");
  HIPCHK(launch_wc_header(a, s), "k_wc_header");
  struct {
    unsigned long long total;
    unsigned int flags, pad;
  } back{};
  HIPCHK(hipMemcpyAsync(&back, a.total, sizeof(back), hipMemcpyDeviceToHost, s), "codec readback");
  HIPCHK(hipStreamSynchronize(s), "stream synchronize");
  if (back.flags & 1u) {
    set_error("bcm_compress: step too small for the field (a code reaches 2^30) or a non-finite value");
    return BCM_ERR_INVALID_ARG;
  }
  *bytes = head + size_t(back.total);
  if (*bytes > capacity) {
    set_error("bcm_compress: stream buffer too small (the needed size is in *bytes)");
    return BCM_ERR_INVALID_ARG;
  }
  HIPCHK(timed(P, cls_of("codec", 0), s, [&] { return launch_wc_pack(P->n, a, grid, s); }), "k_wc_pack");
  return BCM_OK;
}

int bcm_decompress(bcm_plan* P, const void* d_stream, size_t bytes, double* d_field, void* stream) {
  int st = check_bound(P);
  if (st) return st;
  if (!d_stream || !d_field || (reinterpret_cast<uintptr_t>(d_stream) % 8) != 0) {
    set_error("bcm_decompress: NULL argument or stream not 8-byte aligned");
    return BCM_ERR_INVALID_ARG;
  }
  if (P->n < 4) {
    set_error("bcm_decompress: the codec needs n >= 4");
    return BCM_ERR_UNSUPPORTED;
  }
  const size_t head = codec_header_bytes(P);
  if (bytes < head) {
    set_error("bcm_decompress: stream shorter than its header");
    return BCM_ERR_INVALID_ARG;
  }
  hipStream_t s = static_cast<hipStream_t>(stream);
  unsigned char h[32];
  unsigned long long last = 0;
  HIPCHK(hipMemcpyAsync(h, d_stream, 32, hipMemcpyDeviceToHost, s), "header readback");
  HIPCHK(hipMemcpyAsync(&last, static_cast<const char*>(d_stream) + 32 + 8 * size_t(P->nc), 8,
                        hipMemcpyDeviceToHost, s), "header readback");
  HIPCHK(hipStreamSynchronize(s), "stream synchronize");
  uint32_t hw[6];
  double step = 0;
  std::memcpy(hw, h, 24);
  std::memcpy(&step, h + 24, 8);
  if (hw[0] != 0x574D4342u || hw[1] != 1u || int(hw[2]) != P->nc || int(hw[3]) != P->n ||
      int(hw[4]) != codec_levels(P->n) || !(step > 0) || !std::isfinite(step) || last != bytes - head) {
    set_error("bcm_decompress: not a stream of this mesh (magic, version, cube count, n, levels, "
              "step or total size)");
    return BCM_ERR_INVALID_ARG;
  }
  CodecArgs a = codec_args(P, step);
  a.stream_in = d_stream;
  a.data_bytes = bytes - head;
  a.field_out = d_field;
  HIPCHK(launch_zero_u32(a.flags, s), "zero the codec flags");
  HIPCHK(timed(P, cls_of("codec", 0), s,
               [&] { return launch_wc_decode(P->n, a, std::min(P->nc, 4096), s); }), "k_wc_decode");
  unsigned int flags = 0;
  HIPCHK(hipMemcpyAsync(&flags, a.flags, sizeof(flags), hipMemcpyDeviceToHost, s), "codec readback");
  HIPCHK(hipStreamSynchronize(s), "stream synchronize");
  if (flags & 2u) {
    set_error("bcm_decompress: malformed cube stream(s); those cubes decode to zero");
    return BCM_ERR_INVALID_ARG;
  }
  return BCM_OK;
}

int bcm_kinetic_energy_noalloc(bcm_plan* P, const void* const u[3], double rho, double g_scale,
                               double* J, void* const g_u[3], void* stream) {
  int st = check_bound(P);
  if (st) return st;
  if (!u || !u[0] || !u[1] || !u[2] || !(rho > 0) || !std::isfinite(g_scale) ||
      (g_u && (!g_u[0] || !g_u[1] || !g_u[2]))) {
    set_error("bcm_kinetic_energy_noalloc: NULL field, non-positive rho or non-finite g_scale");
    return BCM_ERR_INVALID_ARG;
  }
  hipStream_t s = static_cast<hipStream_t>(stream);
  return P->fields32 ? kinetic_noalloc_impl<float>(P, u, rho, g_scale, J, g_u, s)
                     : kinetic_noalloc_impl<double>(P, u, rho, g_scale, J, g_u, s);
}

int bcm_poisson_solve(bcm_plan* P, const double* d_b, double* d_p, int use_guess, bcm_report* rep,
                      void* stream) {
  int st = check_bound(P);
  if (st) return st;
  if (!d_b || !d_p) {
    set_error("bcm_poisson_solve: NULL field");
    return BCM_ERR_INVALID_ARG;
  }
  st = poisson(P, d_b, d_p, use_guess != 0, rep, static_cast<hipStream_t>(stream));
  if (rep) rep->status = st;
  return st;
}

int bcm_apply_laplacian(bcm_plan* P, const double* d_p, double* d_Ap, void* stream) {
  int st = check_bound(P);
  if (st) return st;
  if (!d_p || !d_Ap) {
    set_error("bcm_apply_laplacian: NULL field");
    return BCM_ERR_INVALID_ARG;
  }
  hipStream_t s = static_cast<hipStream_t>(stream);
  if ((st = export64(P, const_cast<double*>(d_p), P->at<double>(P->o_pf), s))) return st;
  Resid64Args<double> ra{geom(P, P->n), d_p, P->at<const double>(P->o_pf), nullptr, d_Ap, nullptr, nullptr, 1.0};
  HIPCHK(timed(P, cls_of("resid64", 0), s, [&] { return launch_resid64<double>(P->n, ra, s); }), "kc_resid64 (apply)");
  return BCM_OK;
}

int bcm_timing_enable(bcm_plan* P, const char* name) {
  if (!P) {
    set_error("bcm_timing_enable: NULL plan");
    return BCM_ERR_INVALID_ARG;
  }
  P->timer.used = 0;
  P->timer.cls = -1;
  P->timer.every = 1;
  P->timer.seen = 0;
  if (!name || !*name) return BCM_OK;
  for (int i = 0; kTimerNames[i]; ++i)
    if (!std::strcmp(kTimerNames[i], name)) {
      P->timer.cls = i;
      return BCM_OK;
    }
  set_error(std::string("bcm_timing_enable: unknown kernel class ") + name);
  return BCM_ERR_INVALID_ARG;
}

int bcm_timing_sample(bcm_plan* P, int32_t every) {
  if (!P || every < 1) {
    set_error("bcm_timing_sample: NULL plan or every < 1");
    return BCM_ERR_INVALID_ARG;
  }
  P->timer.every = every;
  P->timer.seen = 0;
  return BCM_OK;
}

int bcm_timing_read(bcm_plan* P, int64_t* launches, double* total_ms) {
  if (!P || !launches || !total_ms) {
    set_error("bcm_timing_read: NULL argument");
    return BCM_ERR_INVALID_ARG;
  }
  double tot = 0.0;
  for (size_t i = 0; i + 1 < P->timer.used; i += 2) {
    HIPCHK(hipEventSynchronize(P->timer.ev[i + 1]), "event synchronize");
    float ms = 0.f;
    HIPCHK(hipEventElapsedTime(&ms, P->timer.ev[i], P->timer.ev[i + 1]), "event elapsed time");
    tot += ms;
  }
  *launches = int64_t(P->timer.used / 2);
  *total_ms = tot;
  return BCM_OK;
}

const char* bcm_timing_name(int i) {
  if (i < 0) return nullptr;
  for (int k = 0; kTimerNames[k]; ++k)
    if (k == i) return kTimerNames[k];
  return nullptr;
}

}  // extern "C"
