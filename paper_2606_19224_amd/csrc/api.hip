// Host side of the C ABI declared in include/cgd_enkf.h.
#include <math.h>
#include <string.h>

#include <algorithm>
#include <mutex>
#include <vector>

#include "internal.h"
#include "modes.h"

namespace cgd {

size_t cg_smem_bytes(int RB, int N, int prec);

namespace {

inline size_t al256(size_t x) { return (x + 255) & ~size_t(255); }

// The caller's options with the tuning overrides flattened in (NULL tuning:
// all automatic).
struct Opts : cgd_options {
  int grid, solver, rows_per_block, cooperative;
  unsigned census_ticks;
  void* prof_events;
  unsigned long long* trace;
};

Opts resolve_options(const cgd_options* opt) {
  Opts o;
  memset(&o, 0, sizeof(o));
  if (opt) {
    static_cast<cgd_options&>(o) = *opt;
  } else {
    o.prec = CGD_FP64;
  }
  if (o.tuning) {
    o.grid = o.tuning->grid;
    o.solver = o.tuning->solver;
    o.rows_per_block = o.tuning->rows_per_block;
    o.cooperative = o.tuning->cooperative;
    o.census_ticks = o.tuning->census_ticks;
    o.prof_events = o.tuning->prof_events;
    o.trace = o.tuning->trace;
  }
  return o;
}

bool sizes_ok(int n, int m, int N, int k) {
  if (n < 1 || m < 1 || N < 2 || k < 1) return false;
  // 32-bit element offsets inside tiles; keep every array below 2^31 elements
  if ((long long)n * N >= (1LL << 31) || (long long)m * N >= (1LL << 31) ||
      (long long)m * k >= (1LL << 31))
    return false;
  return true;
}

int solver_rows(int N, int prec) {
  // three RB x N tiles in LDS, about 48 KiB in total
  const size_t esz = prec == CGD_FP64 ? 8 : 4;
  long r = (long)((48 * 1024) / (3 * esz * (size_t)N + esz));
  if (r > 256) r = 256;
  if (r < 1) r = 1;
  return (int)r;
}

// N padded for the resident solver's MFMA tiles; the workspace strides and
// the kernel variant must use the same value.
int resident_pad(int N, int prec) {
  if (N <= 16) return 16;
  if (N <= 32) return 32;
  if (N <= 64) return 64;
  if (prec != CGD_FP64 && N <= 128) return 128;
  return 0;  // resident solver not available: streaming only
}

int reduced_rows(int N) {
  long r = (long)((48 * 1024) / (2 * 8 * (size_t)N + 16));
  if (r > 128) r = 128;
  if (r < 1) r = 1;
  return (int)r;
}

}  // namespace

// The precisions the library knows; the float-data ones the row-block x
// member-group solver runs.
inline bool prec_known(int p) {
  return p == CGD_FP64 || p == CGD_FP32 || p == CGD_MIXED_BF16 || p == CGD_BF16_SPLIT;
}
inline bool prec_tile(int p) { return p == CGD_FP32 || p == CGD_MIXED_BF16 || p == CGD_BF16_SPLIT; }

Layout make_layout(int n, int m, int N, int k, int prec, int mode) {
  Layout L;
  memset(&L, 0, sizeof(L));
  const size_t esz = prec == CGD_FP64 ? 8 : 4;
  const size_t mN = (size_t)m * N, NN = (size_t)N * N;
  size_t o = 0;
  auto take = [&](size_t bytes) {
    size_t at = o;
    o += al256(bytes);
    return at;
  };
  const bool tri = (mode & 2) != 0;
  mode &= 1;
  if (mode == 0) {
    L.RB = solver_rows(N, prec);
    L.nblk = (m + L.RB - 1) / L.RB;
    L.nwg_max = L.nblk < kMaxGrid ? L.nblk : kMaxGrid;
    {
      const int rp = resident_pad(N, prec);
      L.NP = rp > N ? rp : N;  // >= both solvers' partial strides
    }
    // partial buffers serve both solvers: the streaming one (stride N, at most
    // nwg_max workgroups) and the resident one (stride NP, one workgroup per
    // block of >= 16 rows)
    const size_t NPa = (size_t)L.NP;
    size_t nres = (size_t)(m + 15) / 16;
    if (nres > (size_t)kMaxResidentGrid) nres = kMaxResidentGrid;
    const size_t nw = nres > (size_t)L.nwg_max ? nres : (size_t)L.nwg_max;
    const size_t NNa = NPa * NPa;
    // column solver: S in plane layout (mp x NPc) and D transposed (N x mp)
    int mp = 0, npc = 0, gv = 0;
    const int mix = prec == CGD_MIXED_BF16;
    const int col_ok = prec == CGD_FP64 ? columns_shape<double>(m, N, 0, &mp, &npc, &gv)
                                        : columns_shape<float>(m, N, mix, &mp, &npc, &gv);
    L.mp = col_ok ? mp : 0;
    L.NPc = col_ok ? npc : 0;
    L.gv = col_ok ? gv : 0;
    const size_t dN = col_ok && (size_t)N * mp > mN ? (size_t)N * mp : mN;
    L.S = take(esz * mN);
    L.D = take(esz * dN);
    L.Z = take(esz * mN);
    L.R = take(esz * mN);
    L.P = take(esz * mN);
    L.partG = take(esz * NNa * nw);
    L.partG2 = take(esz * NNa * nres);
    L.partS = take(sizeof(double) * PS_NS * NPa * nw);
    L.Gt = take(esz * 2 * NNa);
    L.Gd = take(esz * NNa);
    L.partW = take(sizeof(double) * NNa * nw);
    L.col = take(sizeof(double) * CF_NF * N);
    L.coli = take(sizeof(int) * CI_NI * N);
    L.ctr = take(sizeof(int) * 4);
    L.Wd = take(sizeof(double) * NN);
    L.relres = take(sizeof(double) * N);
    L.flags = take(sizeof(int) * 4);
    L.xflags = take(sizeof(unsigned) * kResidentFlagWords);
    L.pend = take(sizeof(int) * kMaxResidentGrid);
    L.err = take(sizeof(int) * 4);
    L.Scol = col_ok ? take(esz * (size_t)mp * npc) : 0;
    L.Scol16 = (col_ok && mix) ? take(2 * (size_t)mp * npc) : 0;
    L.Vz = L.gv ? take(esz * (size_t)N * mp) : 0;
    L.Vr = L.gv ? take(esz * (size_t)N * mp) : 0;
    L.Vp = L.gv ? take(esz * (size_t)N * mp) : 0;
    L.Rp = L.gv ? take(esz * (size_t)mp) : 0;
    // split solver, when a row slice of S fits the LDS: S in slices, D
    // transposed over the slices' padded rows, exchange slots
    int sp = 0, sms = 0;
    const int split_ok = !mix && (prec == CGD_FP64 ? split_shape<double>(m, N, &sp, &sms)
                                                   : split_shape<float>(m, N, &sp, &sms));
    L.splitP = split_ok ? sp : 0;
    L.splitMs = split_ok ? sms : 0;
    const int np = N <= 16 ? 16 : N <= 32 ? 32 : 64;
    L.Ssplit = split_ok ? take(esz * (size_t)sp * sms * np) : 0;
    L.Dsplit = split_ok ? take(esz * (size_t)N * sp * sms) : 0;
    // published W (both per-member solvers), then the exchange slots
    // (the last word is the start-up census of a plain launch)
    L.xwords =
        (col_ok || split_ok) ? 2 * NN + (split_ok ? split_exchange_words(N, sp) : 0) + 1 : 0;
    L.xw = L.xwords ? take(sizeof(unsigned long long) * L.xwords) : 0;
    // per-workgroup error words of their gather launch (at least 8 padded rows each)
    {
      size_t rows = (size_t)m;
      if ((size_t)L.mp > rows) rows = (size_t)L.mp;
      if ((size_t)L.splitP * L.splitMs > rows) rows = (size_t)L.splitP * L.splitMs;
      L.gerr = L.xwords ? take(sizeof(int) * (rows / 8 + 1)) : 0;
    }
    // row-block x member-group solver (FP32 only)
    if (prec_tile(prec) && tile_shape(m, N, &L.tNP, &L.tRB, &L.tNG, &L.tnblk)) {
      L.tx = take(sizeof(unsigned long long) * tile_words(L.tNP, L.tNG, L.tnblk));
      L.tS = take(sizeof(float) * (size_t)m * L.tNP);
      L.tR = take(sizeof(float) * (size_t)m);
    }
  } else {
    int np = 0, mpad = 0, kc = 0, sc = 0;
    if (reduced_shape(m, N, &np, &mpad, &kc, &sc)) {
      L.rNP = np;
      L.rmpad = mpad;
      L.rKC = kc;
      L.rS = sc;
      const size_t lg = np < 64 ? 64 : (size_t)np, nr = lg;
      L.rQ = np > 64 ? take(esz * (size_t)mpad * 2 * np) : 0;  // NP <= 64: Q stays on chip
      L.rpart = take(esz * (size_t)sc * np * 2 * np);
      L.rG = take(sizeof(double) * nr * lg);
      L.rWt = take(esz * (size_t)np * np);
      L.rerr = take(sizeof(int) * (size_t)mpad);  // one word per gather workgroup
    } else {
      L.RB = reduced_rows(N);
      L.nblk = (m + L.RB - 1) / L.RB;
      L.nwg_max = L.nblk < kMaxGrid ? L.nblk : kMaxGrid;
      L.rpart = take(sizeof(double) * 2 * NN * L.nwg_max);
      L.rG = take(sizeof(double) * NN);
    }
    L.rB = take(sizeof(double) * NN);
    L.Wd = take(sizeof(double) * NN);
    L.riters = take(sizeof(int) * N);
    L.rstat = take(sizeof(int) * N);  // per-column ColStatus of the N x N CG
    L.flags = take(sizeof(int) * 4);
    L.err = take(sizeof(int) * 4);
  }
  if (tri) {
    L.tSd = take(sizeof(double) * mN);
    L.tDd = take(sizeof(double) * mN);
    L.tXp = take(esz * mN);
    L.tEp = take(esz * mN);
    L.tidx = take(sizeof(int32_t) * (size_t)m);
    L.tw = take(esz * (size_t)m);
    L.ty = take(esz * (size_t)m);
    L.tr = take(esz * (size_t)m);
    L.tzt = take(esz * mN);
    L.terr = take(sizeof(int) * 4);
  }
  (void)n;
  (void)k;
  L.total = o;
  return L;
}

namespace {

cgd_status validate_inputs(int prec, int n, int m, int N, int k, const void* Xf,
                           const int32_t* idx, const void* w, const void* y, const void* r,
                           const void* eps, const void* z0, void* ws, const Layout& L,
                           hipStream_t s) {
  int* flags = (int*)((unsigned char*)ws + L.flags);
  if (hipMemsetAsync(flags, 0, sizeof(int), s) != hipSuccess) return CGD_ERR_HIP;
  hipError_t e;
  if (prec == CGD_FP64)
    e = launch_validate<double>(n, m, N, k, (const double*)Xf, idx, (const double*)w,
                                (const double*)y, (const double*)r, (const double*)eps,
                                (const double*)z0, flags, s);
  else
    e = launch_validate<float>(n, m, N, k, (const float*)Xf, idx, (const float*)w,
                               (const float*)y, (const float*)r, (const float*)eps,
                               (const float*)z0, flags, s);
  if (e != hipSuccess) return CGD_ERR_HIP;
  int h = 0;
  if (hipMemcpyAsync(&h, flags, sizeof(int), hipMemcpyDeviceToHost, s) != hipSuccess)
    return CGD_ERR_HIP;
  if (hipStreamSynchronize(s) != hipSuccess) return CGD_ERR_HIP;
  if (h & VF_INDEX) return CGD_ERR_INDEX;
  if (h & VF_NONPOS_R) return CGD_ERR_NONPOS_R;
  if (h & VF_NONFINITE) return CGD_ERR_NONFINITE;
  return CGD_OK;
}

cgd_status common_checks(int n, int m, int N, int k, const void* Xf, void* Xa, const int32_t* idx,
                         const void* w, const void* y, const void* r, double tol, int maxit,
                         const Opts& o, void* ws, size_t ws_bytes, const Layout& L) {
  if (!sizes_ok(n, m, N, k)) return CGD_ERR_ARG;
  if (!Xf || !Xa || !idx || !w || !y || !r) return CGD_ERR_ARG;
  if (!(tol >= 0.0) || !isfinite(tol) || maxit < 0) return CGD_ERR_ARG;
  if (!prec_known(o.prec)) return CGD_ERR_ARG;
  if (o.grid < 0 || o.rr_period < 0) return CGD_ERR_ARG;
  if (o.precond != CGD_PRECOND_NONE && o.precond != CGD_PRECOND_DIAG_R) return CGD_ERR_ARG;
  if (!ws || ws_bytes < L.total) return CGD_ERR_WORKSPACE;
  if (((uintptr_t)ws & 255) != 0) return CGD_ERR_WORKSPACE;
  return CGD_OK;
}

// Solver variant for the full analysis.
//   kind 4: split solver (P workgroups per member, S slices in LDS) when the
//           column solver would stream much of S through L2 every pass, a
//           slice fits and the N * P workgroups fit co-resident;
//   kind 3: column-parallel solver (one workgroup per member, S through L2)
//           when the column layout applies and N workgroups fit co-resident;
//   kind 5: row-block x member-group solver (FP32, N <= 128, cold start,
//           no stall fallback) when its NG * nblk workgroups fit co-resident;
//   kind 2: resident row-block solver when N and the row blocks fit on chip
//           (NP = padded N, RB rows per workgroup, nwg workgroups);
//   kind 1: streaming cooperative solver otherwise.
// Lnp is the padded N the workspace was laid out for.
struct SolverChoice {
  int kind, NP, RB, nwg;
};
// The automatic choice takes the split solver when the column solver would
// stream more than this many bytes of S per member and pass through L2
// (measured on gfx950 at N = 64: split faster at m = 2048, 448 KiB streamed;
// column solver faster at m = 1024, 128 KiB, and at N = 32, m = 2048, 192 KiB).
constexpr size_t kSplitStreamBytes = 256 * 1024;

template <typename T>
cgd_status choose_solver(int m, int N, const Opts& o, const Layout& L,
                         SolverChoice* out) {
  SolverChoice c = {0, 0, 0, 0};
  if (o.solver < 0 || o.solver > 5) return CGD_ERR_ARG;
  const int mix = o.prec == CGD_MIXED_BF16;
  if (mix && o.solver != 0 && o.solver != 3 && o.solver != 5) return CGD_ERR_UNSUPPORTED;
  if (o.prec == CGD_BF16_SPLIT) {
    // the split-BF16 products run on the row-block x member-group solver only
    const bool ok = (o.solver == 0 || o.solver == 5) && L.tx && !o.z0 && !o.fallback_on_stall &&
                    o.rr_period == 0 && L.tNG * L.tnblk <= tile_coresident(L.tNP, L.tRB, 2);
    if (!ok) return CGD_ERR_UNSUPPORTED;
    c.kind = 5;
    c.NP = L.tNP;
    c.RB = L.tRB;
    c.nwg = L.tNG * L.tnblk;
    *out = c;
    return CGD_OK;
  }
  if ((o.solver == 0 || o.solver == 4) && !mix) {
    const bool want = o.solver == 4 || columns_streamed_bytes<T>(m, N) > kSplitStreamBytes;
    if (want && L.splitP > 0 &&
        N * L.splitP <= split_coresident<T>(N, L.splitP, L.splitMs)) {
      c.kind = 4;
      c.NP = L.splitP;   // workgroups per member
      c.RB = L.splitMs;  // rows per workgroup
      c.nwg = N * L.splitP;
      *out = c;
      return CGD_OK;
    }
    if (o.solver == 4) return CGD_ERR_UNSUPPORTED;
  }
  if (o.solver == 0 || o.solver == 3) {
    // with its vectors in global memory (large m) the column solver is the
    // automatic choice only where no other solver applies
    const bool auto_ok = !L.gv || o.solver == 3;
    if (L.NPc > 0 && auto_ok && columns_coresident<T>(m, N, mix) >= N) {
      c.kind = 3;
      c.NP = L.NPc;
      c.nwg = N;
      *out = c;
      return CGD_OK;
    }
    if (o.solver == 3) return CGD_ERR_UNSUPPORTED;
  }
  if (mix) {
    // the mixed mode runs on the row-block x member-group solver (BF16 inner
    // CG on the MFMA) or on the column solver
    const bool ok = (o.solver == 0 || o.solver == 5) && L.tx && !o.z0 &&
                    !o.fallback_on_stall && o.rr_period == 0 &&
                    L.tNG * L.tnblk <= tile_coresident(L.tNP, L.tRB, 1);
    if (ok) {
      c.kind = 5;
      c.NP = L.tNP;
      c.RB = L.tRB;
      c.nwg = L.tNG * L.tnblk;
    } else if (o.solver == 0 && L.NPc > 0 && columns_coresident<T>(m, N, mix) >= N) {
      c.kind = 3;
      c.NP = L.NPc;
      c.nwg = N;
    } else {
      return CGD_ERR_UNSUPPORTED;
    }
    *out = c;
    return CGD_OK;
  }
  if (o.solver == 0 || o.solver == 5) {
    const bool ok = L.tx && o.prec == CGD_FP32 && !o.z0 && !o.fallback_on_stall &&
                    o.rr_period == 0 && L.tNG * L.tnblk <= tile_coresident(L.tNP, L.tRB, 0);
    if (ok) {
      c.kind = 5;
      c.NP = L.tNP;
      c.RB = L.tRB;
      c.nwg = L.tNG * L.tnblk;
      *out = c;
      return CGD_OK;
    }
    if (o.solver == 5) return CGD_ERR_UNSUPPORTED;
  }
  if (o.solver != 1) {
    const int NP = resident_pad(N, o.prec);
    if (NP != resident_np<T>(N) || NP > L.NP) return CGD_ERR_UNSUPPORTED;  // layout guard
    if (NP > 0) {
      const int choices[3] = {16, 32, 64};
      for (int i = 0; i < 3 && !c.RB; ++i) {
        const int rb = choices[i];
        if (o.rows_per_block > 0 && rb != o.rows_per_block) continue;
        if (NP == 128 && rb > 16) continue;  // the only N <= 128 instance
        const int nw = (m + rb - 1) / rb;
        // automatic choice: the smallest block giving at most 64 workgroups,
        // else the largest block that fits (each flag exchange costs more
        // with more workgroups than the extra rows per workgroup do)
        if (o.rows_per_block == 0 && nw > 64 && rb < 64 && NP != 128) continue;
        if (nw > kMaxResidentGrid) continue;
        const int cap = resident_coresident<T>(NP, rb);
        if (nw <= cap) {
          c.kind = 2;
          c.NP = NP;
          c.RB = rb;
          c.nwg = nw;
        }
      }
    }
    if (!c.RB && o.solver == 2) return CGD_ERR_UNSUPPORTED;
  }
  if (!c.kind) {
    int nwg = L.nwg_max;
    if (o.grid > 0 && o.grid < nwg) nwg = o.grid;
    const int cap = cg_max_coresident<T>(L.RB, N);
    if (cap <= 0) return CGD_ERR_HIP;
    c.kind = 1;
    c.RB = L.RB;
    c.nwg = nwg < cap ? nwg : cap;
  }
  *out = c;
  return CGD_OK;
}

// The solvers write the solution of the scaled system when preconditioned.
template <typename T>
cgd_status unscale_z_out(int m, int N, const void* r, const Opts& o, hipStream_t s) {
  if (o.precond != CGD_PRECOND_DIAG_R || !o.z_out) return CGD_OK;
  return launch_unscale_rows<T>(m, N, (T*)o.z_out, (const T*)r, s) == hipSuccess ? CGD_OK
                                                                                  : CGD_ERR_HIP;
}

template <typename T>
cgd_status run_full(int n, int m, int N, int k, const void* Xf, void* Xa, const void* Xg, int ng,
                    const int32_t* idx, const void* w, const void* y, const void* r,
                    const void* eps, double tol, int maxit, const Opts& o, void* ws,
                    const Layout& L, bool need_relres, hipStream_t s) {
  unsigned char* b = (unsigned char*)ws;
  CGArgs<T> a;
  memset(&a, 0, sizeof(a));
  a.n = n; a.m = m; a.N = N; a.k = k; a.RB = L.RB; a.nblk = L.nblk;
  a.Xg = (const T*)Xg; a.ng = ng;
  a.Xf = (const T*)Xf; a.Xa = (T*)Xa; a.idx = idx; a.hw = (const T*)w; a.y = (const T*)y;
  a.rdiag = (const T*)r; a.eps = (const T*)eps; a.z0 = (const T*)o.z0;
  a.S = (T*)(b + L.S); a.D = (T*)(b + L.D); a.Z = (T*)(b + L.Z); a.R = (T*)(b + L.R);
  a.P = (T*)(b + L.P);
  a.partG = (T*)(b + L.partG); a.partS = (double*)(b + L.partS); a.Gt = (T*)(b + L.Gt);
  a.Gd = (T*)(b + L.Gd); a.partW = (double*)(b + L.partW); a.col = (double*)(b + L.col);
  a.coli = (int*)(b + L.coli); a.ctr = (int*)(b + L.ctr); a.Wd = (double*)(b + L.Wd);
  a.relres = (double*)(b + L.relres);
  a.z_out = (T*)o.z_out; a.iters_out = o.iters_out; a.relres_out = o.relres_out;
  a.tol = tol; a.maxit = maxit; a.fallback = o.fallback_on_stall ? 1 : 0;
  a.want_relres = need_relres ? 1 : 0;
  a.rr_period = o.rr_period;
  a.precond = o.precond == CGD_PRECOND_DIAG_R ? 1 : 0;

  a.partG2 = (T*)(b + L.partG2);
  a.arrive = (unsigned*)(b + L.xflags);
  a.done = a.arrive + kMaxResidentGrid;
  a.pend = (int*)(b + L.pend);
  a.err = (int*)(b + L.err);
  a.trace = o.trace;

  SolverChoice sc;
  const cgd_status cs = choose_solver<T>(m, N, o, L, &sc);
  if (cs != CGD_OK) return cs;
  hipEvent_t* ev = (hipEvent_t*)o.prof_events;
  if (sc.kind == 3 || sc.kind == 4) {
    // two launches: the gather (which also clears the published-W words, the
    // exchange slots and the error word) and the solver, which also applies
    // the update
    unsigned long long* wb = (unsigned long long*)(b + L.xw);
    a.census = o.cooperative ? nullptr : wb + (L.xwords - 1);
    a.census_ticks = o.census_ticks ? o.census_ticks : kCensusTicks;
    a.gerr = (int*)(b + L.gerr);
    a.zp = (unsigned*)wb;
    a.zn = (long)(2 * L.xwords);
    // the launcher records ev[0] between the gather and the solver launch
    hipError_t e;
    if (sc.kind == 4) {
      e = launch_cg_split<T>(a, sc.NP, sc.RB, (T*)(b + L.Ssplit), (T*)(b + L.Dsplit),
                             wb + 2 * (size_t)N * N, wb, ev, s);
    } else {
      __bf16* Sh = o.prec == CGD_MIXED_BF16 ? (__bf16*)(b + L.Scol16) : nullptr;
      auto vec = [&](size_t off) { return L.gv ? (T*)(b + off) : nullptr; };
      e = launch_cg_columns<T>(a, (T*)(b + L.Scol), Sh, wb, vec(L.Vz), vec(L.Vr), vec(L.Vp),
                               vec(L.Rp), ev, s);
    }
    if (e != hipSuccess) return CGD_ERR_HIP;
    if (ev && hipEventRecord(ev[1], s) != hipSuccess) return CGD_ERR_HIP;
    return unscale_z_out<T>(m, N, r, o, s);
  }
  if (sc.kind == 5) {
    if constexpr (sizeof(T) == 4) {
      a.txp = (unsigned long long*)(b + L.tx);
      a.txr = a.txp + tile_part_words(L.tNP, L.tNG, L.tnblk);
      a.tNG = L.tNG;
      a.tnblk = L.tnblk;
      a.tS = (T*)(b + L.tS);
      a.tR = (T*)(b + L.tR);
      // the census word is the last exchange word (zeroed by the launcher)
      a.census = o.cooperative ? nullptr
                               : a.txp + tile_words(L.tNP, L.tNG, L.tnblk) - 1;
      a.census_ticks = o.census_ticks ? o.census_ticks : kCensusTicks;
      if (launch_zero_u32((unsigned*)a.err, 1, s) != hipSuccess) return CGD_ERR_HIP;
      if (ev && hipEventRecord(ev[0], s) != hipSuccess) return CGD_ERR_HIP;
      const int variant = o.prec == CGD_MIXED_BF16 ? 1 : o.prec == CGD_BF16_SPLIT ? 2 : 0;
      if (launch_cg_tile(a, sc.NP, sc.RB, variant, s) != hipSuccess)
        return CGD_ERR_HIP;
      if (ev && hipEventRecord(ev[1], s) != hipSuccess) return CGD_ERR_HIP;
      if (launch_update<T>(n, N, (const T*)Xf, (T*)Xa, a.Wd, 0, s,
                           a.census ? a.err : nullptr) != hipSuccess)
        return CGD_ERR_HIP;
      return unscale_z_out<T>(m, N, r, o, s);
    }
    return CGD_ERR_UNSUPPORTED;
  }
  // the resident solver runs under a plain launch with its start-up census
  // unless cooperative launch is asked for; the streaming one synchronises
  // the grid through the cooperative API and always takes it
  a.census = (sc.kind == 2 && !o.cooperative)
                 ? (unsigned long long*)(a.arrive + 2 * kMaxResidentGrid)
                 : nullptr;
  a.census_ticks = o.census_ticks ? o.census_ticks : kCensusTicks;
  if (launch_zero_u32((unsigned*)a.err, 1, s) != hipSuccess) return CGD_ERR_HIP;
  if (ev && hipEventRecord(ev[0], s) != hipSuccess) return CGD_ERR_HIP;
  if (sc.kind == 2) {
    if (launch_cg_resident<T>(a, sc.NP, sc.RB, sc.nwg, s) != hipSuccess) return CGD_ERR_HIP;
  } else {
    if (launch_cg_solve<T>(a, sc.nwg, s) != hipSuccess) return CGD_ERR_HIP;
  }
  if (ev && hipEventRecord(ev[1], s) != hipSuccess) return CGD_ERR_HIP;
  if (launch_update<T>(n, N, (const T*)Xf, (T*)Xa, a.Wd, 0, s, a.census ? a.err : nullptr) !=
      hipSuccess)
    return CGD_ERR_HIP;
  return unscale_z_out<T>(m, N, r, o, s);
}

// Non-diagonal R: the whitened problem the solvers run on (whiten.hip).
template <typename T>
TriBuffers<T> tri_buffers(const Layout& L, void* ws, bool warm) {
  unsigned char* b = (unsigned char*)ws;
  TriBuffers<T> t;
  t.Sd = (double*)(b + L.tSd);
  t.Dd = (double*)(b + L.tDd);
  t.Xp = (T*)(b + L.tXp);
  t.Ep = (T*)(b + L.tEp);
  t.idxp = (int32_t*)(b + L.tidx);
  t.wp = (T*)(b + L.tw);
  t.yp = (T*)(b + L.ty);
  t.rp = (T*)(b + L.tr);
  t.zt = warm ? (T*)(b + L.tzt) : nullptr;
  t.err = (int*)(b + L.terr);
  return t;
}

// The analysis with R = L L^T (L lower bidiagonal): whiten, solve the
// whitened problem with the chosen solver (or the reduced mode), fold the
// whitening pass's index error in, map z_out back.
template <typename T>
cgd_status run_tri(int n, int m, int N, int k, const void* Xf, void* Xa, const int32_t* idx,
                   const void* w, const void* y, const void* eps, double tol, int maxit,
                   const Opts& o, void* ws, const Layout& L, bool need_relres, bool reduced,
                   hipStream_t s) {
  const T* Lf = (const T*)o.r_factor;
  const TriBuffers<T> tb = tri_buffers<T>(L, ws, !reduced && o.z0 != nullptr);
  if (launch_tri_whiten<T>(n, m, N, k, (const T*)Xf, idx, (const T*)w, (const T*)y,
                           (const T*)eps, Lf, reduced ? nullptr : (const T*)o.z0, tb, tb.err,
                           s) != hipSuccess)
    return CGD_ERR_HIP;
  int* err = (int*)((unsigned char*)ws + L.err);
  if (reduced) {
    if (launch_reduced<T>(n, m, N, 1, (const T*)Xf, (T*)Xa, tb.Xp, m, tb.idxp, tb.wp, tb.yp,
                          tb.rp, tb.Ep, tol, maxit, ws, L, o.iters_out, s) != hipSuccess)
      return CGD_ERR_HIP;
    return launch_or_u32(err, tb.err, s) == hipSuccess ? CGD_OK : CGD_ERR_HIP;
  }
  Opts q = o;
  q.z0 = tb.zt;
  q.precond = CGD_PRECOND_NONE;  // the whitened problem has R' = I
  const cgd_status st = run_full<T>(n, m, N, 1, Xf, Xa, tb.Xp, m, tb.idxp, tb.wp, tb.yp, tb.rp,
                                    tb.Ep, tol, maxit, q, ws, L, need_relres, s);
  if (st != CGD_OK) return st;
  if (launch_or_u32(err, tb.err, s) != hipSuccess) return CGD_ERR_HIP;
  if (o.z_out && launch_tri_back<T>(m, N, Lf, (T*)o.z_out, s) != hipSuccess) return CGD_ERR_HIP;
  return CGD_OK;
}

cgd_status fill_stats(const Layout& L, void* ws, int N, int reduced, int maxit, hipStream_t s,
                      cgd_stats* st) {
  unsigned char* b = (unsigned char*)ws;
  if (hipStreamSynchronize(s) != hipSuccess) return CGD_ERR_HIP;
  memset(st, 0, sizeof(*st));
  int xerr = 0;
  if (hipMemcpy(&xerr, b + L.err, sizeof(int), hipMemcpyDeviceToHost) != hipSuccess)
    return CGD_ERR_HIP;
  if (xerr & 2) return CGD_ERR_INDEX;
  if (xerr & 4) return CGD_ERR_BUSY;
  if (xerr) return CGD_ERR_HIP;
  if (reduced) {
    std::vector<int> it(N), cs(N);
    if (hipMemcpy(it.data(), b + L.riters, sizeof(int) * N, hipMemcpyDeviceToHost) != hipSuccess ||
        hipMemcpy(cs.data(), b + L.rstat, sizeof(int) * N, hipMemcpyDeviceToHost) != hipSuccess)
      return CGD_ERR_HIP;
    bool nonfinite = false;
    st->iters_min = it[0];
    for (int j = 0; j < N; ++j) {
      st->iters_max = it[j] > st->iters_max ? it[j] : st->iters_max;
      st->iters_min = it[j] < st->iters_min ? it[j] : st->iters_min;
      if (cs[j] == COL_CONVERGED) st->n_converged++;
      if (cs[j] == COL_NONFINITE) nonfinite = true;
    }
    if (nonfinite) return CGD_ERR_NONFINITE;
    return st->n_converged == N ? CGD_OK : CGD_NOT_CONVERGED;
  }
  std::vector<int> ci((size_t)CI_NI * N);
  std::vector<double> rr(N);
  if (hipMemcpy(ci.data(), b + L.coli, sizeof(int) * ci.size(), hipMemcpyDeviceToHost) !=
          hipSuccess ||
      hipMemcpy(rr.data(), b + L.relres, sizeof(double) * N, hipMemcpyDeviceToHost) != hipSuccess)
    return CGD_ERR_HIP;
  bool nonfinite = false;
  st->iters_min = ci[CI_ITERS * N];
  for (int j = 0; j < N; ++j) {
    const int it = ci[CI_ITERS * N + j];
    st->iters_max = it > st->iters_max ? it : st->iters_max;
    st->iters_min = it < st->iters_min ? it : st->iters_min;
    if (ci[CI_STATUS * N + j] == COL_CONVERGED) st->n_converged++;
    if (ci[CI_STATUS * N + j] == COL_NONFINITE) nonfinite = true;
    st->n_fallbacks += ci[CI_FALLBACK * N + j];
    st->relres_max = rr[j] > st->relres_max ? rr[j] : st->relres_max;
    if (!isfinite(rr[j])) nonfinite = true;
  }
  if (nonfinite) return CGD_ERR_NONFINITE;
  return st->n_converged == N ? CGD_OK : CGD_NOT_CONVERGED;
}

// ---------------------------------------------------------------------------
// Batched analyses
// ---------------------------------------------------------------------------
struct BatchLayout {
  size_t hdr, desc, gtab, stab, utab, prefix, coli, col, total;
  std::vector<size_t> Sp, Dt, Vz, Vr, Vp, Rp, Wd;
  std::vector<int> NP, mp, RL, gr, ur;
  int ngather, nsolve, nupdate;
  long long sumN;
};

// Rows per gather / update work-table entry of a problem (0 = default); -1
// for a value outside the documented ranges.
int batch_gather_rows(const cgd_problem& q) {
  if (q.gather_rows == 0) return kBatchRowsDefault;
  return (q.gather_rows >= 32 && q.gather_rows <= 4096 && q.gather_rows % 32 == 0) ? q.gather_rows
                                                                                  : -1;
}
int batch_update_rows(const cgd_problem& q) {
  if (q.update_rows == 0) return kBatchRowsDefault;
  return (q.update_rows >= 64 && q.update_rows <= 4096 && q.update_rows % 64 == 0) ? q.update_rows
                                                                                  : -1;
}

bool batch_problem_ok(const cgd_problem& q) {
  if (!sizes_ok(q.n, q.m, q.N, q.k) || q.N > 64) return false;
  if (batch_gather_rows(q) < 0 || batch_update_rows(q) < 0) return false;
  return q.X_f && q.X_a && q.idx && q.w && q.y && q.r_diag;
}

bool batch_shape(int prec, int m, int N, int* NP, int* mp, int* RL) {
  return prec == CGD_FP64 ? batched_shape<double>(m, N, NP, mp, RL) != 0
                          : batched_shape<float>(m, N, NP, mp, RL) != 0;
}

// Workspace of a batch: header (error word), problem descriptors, the three
// work tables, the prefix sums of N, per-member int and double fields, then
// per problem S (plane layout), D^T, the CG vectors z, r, p, diag(R) and W.
bool batch_layout(int count, const cgd_problem* probs, int prec, BatchLayout* out) {
  BatchLayout& B = *out;
  const size_t esz = prec == CGD_FP64 ? 8 : 4;
  const size_t dsz = prec == CGD_FP64 ? sizeof(BProb<double>) : sizeof(BProb<float>);
  size_t o = 0;
  auto take = [&](size_t bytes) {
    const size_t at = o;
    o += al256(bytes);
    return at;
  };
  B.ngather = B.nsolve = B.nupdate = 0;
  B.sumN = 0;
  for (int b = 0; b < count; ++b) {
    int NP = 0, mp = 0, RL = 0;
    if (!batch_shape(prec, probs[b].m, probs[b].N, &NP, &mp, &RL)) return false;
    const int gr = batch_gather_rows(probs[b]), ur = batch_update_rows(probs[b]);
    if (gr < 0 || ur < 0) return false;
    B.NP.push_back(NP);
    B.mp.push_back(mp);
    B.RL.push_back(RL);
    B.gr.push_back(gr);
    B.ur.push_back(ur);
    B.ngather += (mp + gr - 1) / gr;
    B.nsolve += probs[b].N;
    B.nupdate += (probs[b].n + ur - 1) / ur;
    B.sumN += probs[b].N;
  }
  B.hdr = take(256);
  B.desc = take(dsz * count);
  B.gtab = take(sizeof(int2) * (size_t)B.ngather);
  // member entries, padded per XCD queue (see batch_prepare): at most 8 per member
  B.stab = take(sizeof(int2) * 8 * (size_t)B.nsolve);
  B.utab = take(sizeof(int2) * (size_t)B.nupdate);
  B.prefix = take(sizeof(int) * ((size_t)count + 1));
  B.coli = take(sizeof(int) * CI_NI * (size_t)B.sumN);
  B.col = take(sizeof(double) * CF_NF * (size_t)B.sumN);
  for (int b = 0; b < count; ++b) {
    const size_t mp = (size_t)B.mp[b], N = (size_t)probs[b].N;
    B.Sp.push_back(take(esz * mp * B.NP[b]));
    B.Dt.push_back(take(esz * mp * N));
    B.Vz.push_back(take(esz * mp * N));
    B.Vr.push_back(take(esz * mp * N));
    B.Vp.push_back(take(esz * mp * N));
    B.Rp.push_back(take(esz * mp));
    B.Wd.push_back(take(sizeof(double) * N * N));
  }
  B.total = o;
  return true;
}

template <typename T>
cgd_status batch_prepare(int count, const cgd_problem* probs, void* ws, const BatchLayout& B,
                         cgd_batch_plan* plan, int prec, hipStream_t s) {
  unsigned char* base = (unsigned char*)ws;
  // member solves ordered by decreasing work per member (m N^2: row pass
  // cost m NP times the iteration bound ~N), so the longest start first
  std::vector<int> order(count);
  for (int b = 0; b < count; ++b) order[b] = b;
  std::stable_sort(order.begin(), order.end(), [&](int x, int y) {
    const double cx = (double)B.mp[x] * B.NP[x] * probs[x].N;
    const double cy = (double)B.mp[y] * B.NP[y] * probs[y].N;
    return cx > cy;
  });
  std::vector<int> prefix(count + 1, 0);
  for (int b = 0; b < count; ++b) prefix[b + 1] = prefix[b] + probs[b].N;
  std::vector<BProb<T>> desc(count);
  std::vector<int2> gtab, stab, utab;
  gtab.reserve(B.ngather);
  stab.reserve(B.nsolve);
  utab.reserve(B.nupdate);
  for (int b = 0; b < count; ++b) {
    const cgd_problem& q = probs[b];
    BProb<T>& d = desc[b];
    d.n = q.n; d.m = q.m; d.N = q.N; d.k = q.k;
    d.NP = B.NP[b]; d.mp = B.mp[b]; d.RL = B.RL[b]; d.gr = B.gr[b]; d.ur = B.ur[b];
    d.Xf = (const T*)q.X_f; d.Xa = (T*)q.X_a; d.idx = q.idx; d.hw = (const T*)q.w;
    d.y = (const T*)q.y; d.rdiag = (const T*)q.r_diag; d.eps = (const T*)q.eps;
    d.Sp = (T*)(base + B.Sp[b]); d.Dt = (T*)(base + B.Dt[b]);
    d.Vz = (T*)(base + B.Vz[b]); d.Vr = (T*)(base + B.Vr[b]); d.Vp = (T*)(base + B.Vp[b]);
    d.Rp = (T*)(base + B.Rp[b]); d.Wd = (double*)(base + B.Wd[b]);
    d.coli = (int*)(base + B.coli) + (size_t)CI_NI * prefix[b];
    d.col = (double*)(base + B.col) + (size_t)CF_NF * prefix[b];
    d.iters_out = q.iters_out;
    for (int i0 = 0; i0 < B.mp[b]; i0 += B.gr[b]) gtab.push_back(make_int2(b, i0));
    for (int i0 = 0; i0 < q.n; i0 += B.ur[b]) utab.push_back(make_int2(b, i0));
  }
  // Member solves: workgroup w runs on XCD w % 8, so all members of a problem
  // go to one XCD and its S stays in that XCD's L2 while they run.  Problems
  // go, in decreasing order of work, to the XCD with the least work so far;
  // the eight queues are interleaved and padded with empty entries (-1) to
  // equal length.
  {
    constexpr int kXcd = 8;
    std::vector<std::vector<int2>> q(kXcd);
    std::vector<double> load(kXcd, 0.0);
    for (int pos = 0; pos < count; ++pos) {
      const int b = order[pos];
      int x = 0;
      for (int t = 1; t < kXcd; ++t)
        if (load[t] < load[x]) x = t;
      for (int j = 0; j < probs[b].N; ++j) q[x].push_back(make_int2(b, j));
      load[x] += (double)B.mp[b] * B.NP[b] * probs[b].N;
    }
    size_t len = 0;
    for (const auto& v : q) len = v.size() > len ? v.size() : len;
    for (size_t t = 0; t < len; ++t)
      for (int x = 0; x < kXcd; ++x) stab.push_back(t < q[x].size() ? q[x][t] : make_int2(-1, 0));
  }
  if (hipMemcpyAsync(base + B.desc, desc.data(), sizeof(BProb<T>) * count, hipMemcpyHostToDevice,
                     s) != hipSuccess ||
      hipMemcpyAsync(base + B.gtab, gtab.data(), sizeof(int2) * gtab.size(),
                     hipMemcpyHostToDevice, s) != hipSuccess ||
      hipMemcpyAsync(base + B.stab, stab.data(), sizeof(int2) * stab.size(),
                     hipMemcpyHostToDevice, s) != hipSuccess ||
      hipMemcpyAsync(base + B.utab, utab.data(), sizeof(int2) * utab.size(),
                     hipMemcpyHostToDevice, s) != hipSuccess ||
      hipMemcpyAsync(base + B.prefix, prefix.data(), sizeof(int) * prefix.size(),
                     hipMemcpyHostToDevice, s) != hipSuccess ||
      hipStreamSynchronize(s) != hipSuccess)
    return CGD_ERR_HIP;
  memset(plan, 0, sizeof(*plan));
  plan->count = count;
  plan->prec = prec;
  plan->n_gather = B.ngather;
  plan->n_solve = (int)stab.size();
  plan->n_update = B.nupdate;
  plan->off_desc = B.desc;
  plan->off_gtab = B.gtab;
  plan->off_stab = B.stab;
  plan->off_utab = B.utab;
  plan->off_prefix = B.prefix;
  plan->off_coli = B.coli;
  plan->ws_bytes = B.total;
  return CGD_OK;
}

}  // namespace
}  // namespace cgd

using namespace cgd;

// Static scratch of cgd_enkf_analysis_static: the workspace of callers that
// cannot allocate device memory.  Each GPU the library runs on holds its own
// copy for the life of the process.  In host code `scratch` is only a
// stand-in for the symbol: its device address comes from
// hipGetSymbolAddress, taken once per device on that device's first call.
constexpr size_t kStaticScratchBytes = size_t(32) << 20;
static __device__ __align__(256) unsigned char scratch[kStaticScratchBytes];

namespace {

constexpr int kMaxDevices = 64;
std::mutex g_scratch_mu;
void* g_scratch_ptr[kMaxDevices] = {};

// The current device's address of `scratch` (CGD_ERR_HIP if it cannot be had).
cgd_status static_scratch(void** out) {
  int dev = -1;
  if (hipGetDevice(&dev) != hipSuccess || dev < 0 || dev >= kMaxDevices) return CGD_ERR_HIP;
  std::lock_guard<std::mutex> lock(g_scratch_mu);
  if (!g_scratch_ptr[dev]) {
    void* p = nullptr;
    if (hipGetSymbolAddress(&p, HIP_SYMBOL(scratch)) != hipSuccess || !p) return CGD_ERR_HIP;
    g_scratch_ptr[dev] = p;
  }
  *out = g_scratch_ptr[dev];
  return CGD_OK;
}

}  // namespace

extern "C" {

void cgd_options_default(cgd_options* opt) {
  if (!opt) return;
  memset(opt, 0, sizeof(*opt));
  opt->prec = CGD_FP64;
}

size_t cgd_enkf_workspace_bytes(int n, int m, int N, int k, int prec, int mode) {
  if (!sizes_ok(n, m, N, k) || mode < 0 || mode > 3) return 0;
  if (!prec_known(prec)) return 0;
  return make_layout(n, m, N, k, prec, mode).total;
}

cgd_status cgd_enkf_analysis(int n, int m, int N, int k, const void* X_f, void* X_a,
                             const int32_t* idx, const void* w, const void* y,
                             const void* r_diag, const void* eps, double tol, int maxit,
                             const cgd_options* opt, void* workspace, size_t ws_bytes,
                             cgd_stats* stats, void* stream) {
  const Opts o = resolve_options(opt);
  if (!sizes_ok(n, m, N, k)) return CGD_ERR_ARG;
  const Layout L = make_layout(n, m, N, k, o.prec, o.r_factor ? 2 : 0);
  cgd_status st = common_checks(n, m, N, k, X_f, X_a, idx, w, y, r_diag, tol, maxit, o, workspace,
                                ws_bytes, L);
  if (st != CGD_OK) return st;
  // the refinement loop of the mixed mode has no warm-start restart rule
  if (o.prec == CGD_MIXED_BF16 && o.z0 && o.fallback_on_stall) return CGD_ERR_UNSUPPORTED;
  hipStream_t s = (hipStream_t)stream;
  if (o.validate) {
    st = validate_inputs(o.prec, n, m, N, k, X_f, idx, w, y, r_diag, eps, o.z0, workspace, L, s);
    if (st != CGD_OK) return st;
  }
  const bool need_relres = stats != nullptr || o.relres_out != nullptr;
  if (o.r_factor) {
    st = o.prec == CGD_FP64
             ? run_tri<double>(n, m, N, k, X_f, X_a, idx, w, y, eps, tol, maxit, o, workspace, L,
                               need_relres, false, s)
             : run_tri<float>(n, m, N, k, X_f, X_a, idx, w, y, eps, tol, maxit, o, workspace, L,
                              need_relres, false, s);
  } else if (o.prec == CGD_FP64) {
    st = run_full<double>(n, m, N, k, X_f, X_a, X_f, n, idx, w, y, r_diag, eps, tol, maxit, o,
                          workspace, L, need_relres, s);
  } else {
    st = run_full<float>(n, m, N, k, X_f, X_a, X_f, n, idx, w, y, r_diag, eps, tol, maxit, o,
                         workspace, L, need_relres, s);
  }
  if (st != CGD_OK) return st;
  if (stats) return fill_stats(L, workspace, N, 0, maxit, s, stats);
  return CGD_OK;
}

cgd_status cgd_tridiag_cholesky(int m, const void* r_diag, const void* r_offdiag, void* factor,
                                int prec, void* stream) {
  if (m < 1 || !r_diag || (m > 1 && !r_offdiag) || !factor) return CGD_ERR_ARG;
  if (prec != CGD_FP64 && prec != CGD_FP32 && prec != CGD_MIXED_BF16) return CGD_ERR_ARG;
  hipStream_t s = (hipStream_t)stream;
  // a pivot that is not positive leaves factor[0] = -1, read back here
  double d0 = 0.0;
  float f0 = 0.f;
  hipError_t e;
  if (prec == CGD_FP64) {
    e = launch_tri_chol<double>(m, (const double*)r_diag, (const double*)r_offdiag,
                                (double*)factor, nullptr, s);
    if (e == hipSuccess) e = hipMemcpyAsync(&d0, factor, sizeof(double), hipMemcpyDeviceToHost, s);
  } else {
    e = launch_tri_chol<float>(m, (const float*)r_diag, (const float*)r_offdiag, (float*)factor,
                               nullptr, s);
    if (e == hipSuccess) e = hipMemcpyAsync(&f0, factor, sizeof(float), hipMemcpyDeviceToHost, s);
  }
  if (e != hipSuccess || hipStreamSynchronize(s) != hipSuccess) return CGD_ERR_HIP;
  if (prec != CGD_FP64) d0 = f0;
  return d0 > 0.0 && isfinite(d0) ? CGD_OK : CGD_ERR_NONPOS_R;
}

size_t cgd_enkf_static_scratch_bytes(void) { return kStaticScratchBytes; }

cgd_status cgd_enkf_analysis_static(int n, int m, int N, int k, const void* X_f, void* X_a,
                                    const int32_t* idx, const void* w, const void* y,
                                    const void* r_diag, const void* eps, double tol, int maxit,
                                    const cgd_options* opt, cgd_stats* stats, void* stream) {
  const Opts o = resolve_options(opt);
  if (!sizes_ok(n, m, N, k)) return CGD_ERR_ARG;
  if (!prec_known(o.prec)) return CGD_ERR_ARG;
  if (make_layout(n, m, N, k, o.prec, o.r_factor ? 2 : 0).total > kStaticScratchBytes)
    return CGD_ERR_WORKSPACE;
  void* ws = nullptr;
  const cgd_status st = static_scratch(&ws);
  if (st != CGD_OK) return st;
  return cgd_enkf_analysis(n, m, N, k, X_f, X_a, idx, w, y, r_diag, eps, tol, maxit, opt, ws,
                           kStaticScratchBytes, stats, stream);
}

cgd_status cgd_enkf_reduced_analysis(int n, int m, int N, int k, const void* X_f, void* X_a,
                                     const int32_t* idx, const void* w, const void* y,
                                     const void* r_diag, const void* eps, double tol, int maxit,
                                     const cgd_options* opt, void* workspace, size_t ws_bytes,
                                     cgd_stats* stats, void* stream) {
  const Opts o = resolve_options(opt);
  if (!sizes_ok(n, m, N, k)) return CGD_ERR_ARG;
  // (the split-BF16 products exist in the full mode only)
  if (o.prec == CGD_BF16_SPLIT) return CGD_ERR_UNSUPPORTED;
  const Layout L = make_layout(n, m, N, k, o.prec, o.r_factor ? 3 : 1);
  cgd_status st = common_checks(n, m, N, k, X_f, X_a, idx, w, y, r_diag, tol, maxit, o, workspace,
                                ws_bytes, L);
  if (st != CGD_OK) return st;
  hipStream_t s = (hipStream_t)stream;
  if (o.validate) {
    st = validate_inputs(o.prec, n, m, N, k, X_f, idx, w, y, r_diag, eps, nullptr, workspace, L, s);
    if (st != CGD_OK) return st;
  }
  hipEvent_t* ev = (hipEvent_t*)o.prof_events;
  if (ev && hipEventRecord(ev[0], s) != hipSuccess) return CGD_ERR_HIP;
  if (o.r_factor) {
    st = o.prec == CGD_FP64 ? run_tri<double>(n, m, N, k, X_f, X_a, idx, w, y, eps, tol, maxit, o,
                                              workspace, L, false, true, s)
                            : run_tri<float>(n, m, N, k, X_f, X_a, idx, w, y, eps, tol, maxit, o,
                                             workspace, L, false, true, s);
    if (st != CGD_OK) return st;
  } else {
    hipError_t e;
    if (o.prec == CGD_FP64)
      e = launch_reduced<double>(n, m, N, k, (const double*)X_f, (double*)X_a, (const double*)X_f,
                                 n, idx, (const double*)w, (const double*)y,
                                 (const double*)r_diag, (const double*)eps, tol, maxit, workspace,
                                 L, o.iters_out, s);
    else
      e = launch_reduced<float>(n, m, N, k, (const float*)X_f, (float*)X_a, (const float*)X_f, n,
                                idx, (const float*)w, (const float*)y, (const float*)r_diag,
                                (const float*)eps, tol, maxit, workspace, L, o.iters_out, s);
    if (e != hipSuccess) return CGD_ERR_HIP;
  }
  if (ev && hipEventRecord(ev[1], s) != hipSuccess) return CGD_ERR_HIP;
  if (stats) return fill_stats(L, workspace, N, 1, maxit, s, stats);
  return CGD_OK;
}

cgd_status cgd_senkf_analysis(int n, int m, int N, int k, const void* X_f, void* X_a,
                              const int32_t* idx, const void* w, const void* y,
                              const void* r_diag, const void* eps, const cgd_options* opt,
                              void* workspace, size_t ws_bytes, cgd_stats* stats, void* stream) {
  const Opts o = resolve_options(opt);
  if (!sizes_ok(n, m, N, k)) return CGD_ERR_ARG;
  // no system is solved, so there is nothing for a refinement to refine
  if (o.prec != CGD_FP64 && o.prec != CGD_FP32) return prec_known(o.prec) ? CGD_ERR_UNSUPPORTED
                                                                          : CGD_ERR_ARG;
  const Layout L = make_layout(n, m, N, k, o.prec, 1);
  cgd_status st = common_checks(n, m, N, k, X_f, X_a, idx, w, y, r_diag, 0.0, 0, o, workspace,
                                ws_bytes, L);
  if (st != CGD_OK) return st;
  hipStream_t s = (hipStream_t)stream;
  if (o.validate) {
    st = validate_inputs(o.prec, n, m, N, k, X_f, idx, w, y, r_diag, eps, nullptr, workspace, L, s);
    if (st != CGD_OK) return st;
  }
  hipEvent_t* ev = (hipEvent_t*)o.prof_events;
  if (ev && hipEventRecord(ev[0], s) != hipSuccess) return CGD_ERR_HIP;
  hipError_t e =
      o.prec == CGD_FP64
          ? launch_senkf<double>(n, m, N, k, (const double*)X_f, (double*)X_a, idx,
                                 (const double*)w, (const double*)y, (const double*)r_diag,
                                 (const double*)eps, workspace, L, o.iters_out, s)
          : launch_senkf<float>(n, m, N, k, (const float*)X_f, (float*)X_a, idx, (const float*)w,
                                (const float*)y, (const float*)r_diag, (const float*)eps,
                                workspace, L, o.iters_out, s);
  if (e != hipSuccess) return CGD_ERR_HIP;
  if (ev && hipEventRecord(ev[1], s) != hipSuccess) return CGD_ERR_HIP;
  if (!stats) return CGD_OK;
  if (hipStreamSynchronize(s) != hipSuccess) return CGD_ERR_HIP;
  memset(stats, 0, sizeof(*stats));
  int xerr = 0;
  if (hipMemcpy(&xerr, (unsigned char*)workspace + L.err, sizeof(int), hipMemcpyDeviceToHost) !=
      hipSuccess)
    return CGD_ERR_HIP;
  if (xerr & 2) return CGD_ERR_INDEX;
  if (xerr) return CGD_ERR_HIP;
  stats->n_converged = N;
  return CGD_OK;
}

size_t cgd_enkf_gain_workspace_bytes(int n, int m, int N, int k, int prec) {
  if (!sizes_ok(n, m, N, k)) return 0;
  return kt_layout(n, m, N, prec).total;
}

cgd_status cgd_enkf_gain_analysis(int n, int m, int N, int k, const void* X_f, void* X_a,
                                  const int32_t* idx, const void* w, const void* y,
                                  const void* r_diag, const void* eps, double tol, int maxit,
                                  const cgd_options* opt, void* kt_out, double* hist_out,
                                  void* workspace, size_t ws_bytes, cgd_stats* stats,
                                  void* stream) {
  const Opts o = resolve_options(opt);
  if (!sizes_ok(n, m, N, k)) return CGD_ERR_ARG;
  if (!X_f || !X_a || !idx || !w || !y || !r_diag) return CGD_ERR_ARG;
  if (!(tol >= 0.0) || !isfinite(tol) || maxit < 0) return CGD_ERR_ARG;
  if (!prec_known(o.prec)) return CGD_ERR_ARG;
  if (o.prec != CGD_FP64 && o.prec != CGD_FP32) return CGD_ERR_UNSUPPORTED;
  if (N > 128) return CGD_ERR_UNSUPPORTED;
  // a non-diagonal R changes Psi_z; this form takes diag(R) only
  if (o.r_factor) return CGD_ERR_UNSUPPORTED;
  const KtLayout L = kt_layout(n, m, N, o.prec);
  if (!workspace || ws_bytes < L.total || ((uintptr_t)workspace & 255) != 0)
    return CGD_ERR_WORKSPACE;
  hipStream_t s = (hipStream_t)stream;
  unsigned char* b = (unsigned char*)workspace;
  if (o.validate) {
    Layout Lv{};
    Lv.flags = L.err + sizeof(int);  // the second of the four error words
    const cgd_status st = validate_inputs(o.prec, n, m, N, k, X_f, idx, w, y, r_diag, eps,
                                          nullptr, workspace, Lv, s);
    if (st != CGD_OK) return st;
  }
  int* iters = o.iters_out ? o.iters_out : (int*)(b + L.iters);
  hipEvent_t* ev = (hipEvent_t*)o.prof_events;
  if (ev && hipEventRecord(ev[0], s) != hipSuccess) return CGD_ERR_HIP;
  const hipError_t e =
      o.prec == CGD_FP64
          ? launch_kt<double>(n, m, N, k, (const double*)X_f, (double*)X_a, idx,
                              (const double*)w, (const double*)y, (const double*)r_diag,
                              (const double*)eps, tol, maxit, (double*)kt_out, iters, hist_out,
                              L, workspace, s)
          : launch_kt<float>(n, m, N, k, (const float*)X_f, (float*)X_a, idx, (const float*)w,
                             (const float*)y, (const float*)r_diag, (const float*)eps, tol,
                             maxit, (float*)kt_out, iters, hist_out, L, workspace, s);
  if (e != hipSuccess) return CGD_ERR_HIP;
  if (ev && hipEventRecord(ev[1], s) != hipSuccess) return CGD_ERR_HIP;
  if (!stats) return CGD_OK;
  if (hipStreamSynchronize(s) != hipSuccess) return CGD_ERR_HIP;
  memset(stats, 0, sizeof(*stats));
  int xerr = 0;
  std::vector<int> it(n), cs(n);
  if (hipMemcpy(&xerr, b + L.err, sizeof(int), hipMemcpyDeviceToHost) != hipSuccess ||
      hipMemcpy(it.data(), iters, sizeof(int) * n, hipMemcpyDeviceToHost) != hipSuccess ||
      hipMemcpy(cs.data(), b + L.status, sizeof(int) * n, hipMemcpyDeviceToHost) != hipSuccess)
    return CGD_ERR_HIP;
  if (xerr & 2) return CGD_ERR_INDEX;
  if (xerr) return CGD_ERR_HIP;
  bool nonfinite = false;
  stats->iters_min = it[0];
  for (int i = 0; i < n; ++i) {
    stats->iters_max = it[i] > stats->iters_max ? it[i] : stats->iters_max;
    stats->iters_min = it[i] < stats->iters_min ? it[i] : stats->iters_min;
    if (cs[i] == COL_CONVERGED) stats->n_converged++;
    if (cs[i] == COL_NONFINITE) nonfinite = true;
  }
  if (nonfinite) return CGD_ERR_NONFINITE;
  return stats->n_converged == n ? CGD_OK : CGD_NOT_CONVERGED;
}

size_t cgd_enkf_batched_workspace_bytes(int count, const cgd_problem* probs, int prec) {
  if (count < 1 || !probs || (prec != CGD_FP64 && prec != CGD_FP32)) return 0;
  for (int b = 0; b < count; ++b)
    if (!sizes_ok(probs[b].n, probs[b].m, probs[b].N, probs[b].k) || probs[b].N > 64 ||
        batch_gather_rows(probs[b]) < 0 || batch_update_rows(probs[b]) < 0)
      return 0;
  BatchLayout B;
  return batch_layout(count, probs, prec, &B) ? B.total : 0;
}

cgd_status cgd_enkf_batched_prepare(int count, const cgd_problem* probs, int prec,
                                    void* workspace, size_t ws_bytes, cgd_batch_plan* plan,
                                    void* stream) {
  if (count < 1 || !probs || !plan) return CGD_ERR_ARG;
  if (prec != CGD_FP64 && prec != CGD_FP32) return CGD_ERR_UNSUPPORTED;
  for (int b = 0; b < count; ++b)
    if (!batch_problem_ok(probs[b])) return probs[b].N > 64 ? CGD_ERR_UNSUPPORTED : CGD_ERR_ARG;
  BatchLayout B;
  if (!batch_layout(count, probs, prec, &B)) return CGD_ERR_ARG;
  if (!workspace || ws_bytes < B.total || ((uintptr_t)workspace & 255) != 0)
    return CGD_ERR_WORKSPACE;
  hipStream_t s = (hipStream_t)stream;
  return prec == CGD_FP64 ? batch_prepare<double>(count, probs, workspace, B, plan, prec, s)
                          : batch_prepare<float>(count, probs, workspace, B, plan, prec, s);
}

cgd_status cgd_enkf_batched_run(const cgd_batch_plan* plan, void* workspace, double tol,
                                int maxit, const cgd_options* opt, cgd_stats* stats,
                                void* stream) {
  if (!plan || !workspace || plan->count < 1) return CGD_ERR_ARG;
  if (!(tol >= 0.0) || !isfinite(tol) || maxit < 0) return CGD_ERR_ARG;
  const Opts o = resolve_options(opt);
  if (o.prec != plan->prec) return CGD_ERR_ARG;
  if (o.precond != CGD_PRECOND_NONE && o.precond != CGD_PRECOND_DIAG_R) return CGD_ERR_ARG;
  if (o.z0 || o.z_out || o.relres_out || o.r_factor) return CGD_ERR_UNSUPPORTED;
  hipStream_t s = (hipStream_t)stream;
  unsigned char* base = (unsigned char*)workspace;
  int* err = (int*)base;
  hipEvent_t* ev = (hipEvent_t*)o.prof_events;
  if (launch_zero_u32((unsigned*)err, 1, s) != hipSuccess) return CGD_ERR_HIP;
  hipError_t e;
  const int2* gt = (const int2*)(base + plan->off_gtab);
  const int2* st = (const int2*)(base + plan->off_stab);
  const int2* ut = (const int2*)(base + plan->off_utab);
  const int pc = o.precond == CGD_PRECOND_DIAG_R ? 1 : 0;
  if (plan->prec == CGD_FP64)
    e = launch_batched<double>((const BProb<double>*)(base + plan->off_desc), gt, plan->n_gather,
                               st, plan->n_solve, ut, plan->n_update, tol, maxit, pc, err, ev, s);
  else
    e = launch_batched<float>((const BProb<float>*)(base + plan->off_desc), gt, plan->n_gather,
                              st, plan->n_solve, ut, plan->n_update, tol, maxit, pc, err, ev, s);
  if (e != hipSuccess) return CGD_ERR_HIP;
  if (!stats) return CGD_OK;
  if (hipStreamSynchronize(s) != hipSuccess) return CGD_ERR_HIP;
  int xerr = 0;
  std::vector<int> pre(plan->count + 1);
  if (hipMemcpy(&xerr, err, sizeof(int), hipMemcpyDeviceToHost) != hipSuccess ||
      hipMemcpy(pre.data(), base + plan->off_prefix, sizeof(int) * pre.size(),
                hipMemcpyDeviceToHost) != hipSuccess)
    return CGD_ERR_HIP;
  const size_t sumN = (size_t)pre[plan->count];
  std::vector<int> ci((size_t)CI_NI * sumN);
  if (hipMemcpy(ci.data(), base + plan->off_coli, sizeof(int) * ci.size(),
                hipMemcpyDeviceToHost) != hipSuccess)
    return CGD_ERR_HIP;
  if (xerr & 2) return CGD_ERR_INDEX;
  if (xerr) return CGD_ERR_HIP;
  bool all = true, nonfinite = false;
  for (int b = 0; b < plan->count; ++b) {
    cgd_stats& sb = stats[b];
    memset(&sb, 0, sizeof(sb));
    sb.relres_max = -1.0;  // not evaluated for batches
    const int N = pre[b + 1] - pre[b];
    const int* it = ci.data() + (size_t)CI_NI * pre[b] + (size_t)CI_ITERS * N;
    const int* stt = ci.data() + (size_t)CI_NI * pre[b] + (size_t)CI_STATUS * N;
    sb.iters_min = it[0];
    for (int j = 0; j < N; ++j) {
      sb.iters_max = it[j] > sb.iters_max ? it[j] : sb.iters_max;
      sb.iters_min = it[j] < sb.iters_min ? it[j] : sb.iters_min;
      if (stt[j] == COL_CONVERGED) sb.n_converged++;
      if (stt[j] == COL_NONFINITE) nonfinite = true;
    }
    if (sb.n_converged != N) all = false;
  }
  if (nonfinite) return CGD_ERR_NONFINITE;
  return all ? CGD_OK : CGD_NOT_CONVERGED;
}

cgd_status cgd_enkf_analysis_batched(int count, const cgd_problem* probs, double tol, int maxit,
                                     const cgd_options* opt, void* workspace, size_t ws_bytes,
                                     cgd_stats* per_problem_stats, void* stream) {
  if (count < 1 || !probs) return CGD_ERR_ARG;
  const int prec = opt ? opt->prec : CGD_FP64;
  cgd_batch_plan plan;
  const cgd_status st =
      cgd_enkf_batched_prepare(count, probs, prec, workspace, ws_bytes, &plan, stream);
  if (st != CGD_OK) return st;
  return cgd_enkf_batched_run(&plan, workspace, tol, maxit, opt, per_problem_stats, stream);
}

cgd_status cgd_enkf_solver_info(int n, int m, int N, int k, const cgd_options* opt,
                                int* solver, int* rows_per_block, int* workgroups) {
  const Opts o = resolve_options(opt);
  if (!sizes_ok(n, m, N, k) || !solver || !rows_per_block || !workgroups) return CGD_ERR_ARG;
  if (!prec_known(o.prec)) return CGD_ERR_ARG;
  const Layout L = make_layout(n, m, N, k, o.prec, 0);
  SolverChoice sc;
  const cgd_status cs = o.prec == CGD_FP64 ? choose_solver<double>(m, N, o, L, &sc)
                                           : choose_solver<float>(m, N, o, L, &sc);
  if (cs != CGD_OK) return cs;
  *solver = sc.kind;
  *rows_per_block = sc.RB;
  *workgroups = sc.nwg;
  return CGD_OK;
}

int cgd_layout_selfcheck(int n, int m, int N, int k, int prec) {
  // For every solver variant the host could launch on these sizes, the
  // largest element index each kernel uses in each workspace region must lie
  // inside that region.  Returns 0 when all fit, else the number of misfits.
  if (!sizes_ok(n, m, N, k)) return -1;
  const Layout L = make_layout(n, m, N, k, prec, 0);
  const size_t esz = prec == CGD_FP64 ? 8 : 4;
  auto region = [&](size_t off) {  // bytes up to the next region start
    size_t next = L.total;
    const size_t offs[] = {L.S, L.D, L.Z, L.R, L.P, L.partG, L.partG2, L.partS, L.Gt, L.Gd,
                           L.partW, L.col, L.coli, L.ctr, L.Wd, L.relres, L.flags, L.xflags,
                           L.pend, L.err, L.Scol, L.Scol16, L.xw, L.gerr, L.Ssplit, L.Dsplit,
                           L.Vz, L.Vr, L.Vp, L.Rp, L.tx, L.tS, L.tR};
    for (size_t o : offs)
      if (o > off && o < next) next = o;
    return next - off;
  };
  int bad = 0;
  auto need = [&](size_t off, size_t bytes) {
    if (bytes > region(off)) ++bad;
  };
  // streaming solver: stride N, nwg <= nwg_max
  const size_t NN = (size_t)N * N, nws = (size_t)L.nwg_max;
  need(L.partG, esz * NN * nws);
  need(L.partS, sizeof(double) * PS_NS * (size_t)N * nws);
  need(L.partW, sizeof(double) * NN * nws);
  need(L.Gt, esz * 2 * NN);
  need(L.Gd, esz * NN);
  // resident solver: stride NP, one workgroup per block of RB rows
  const int NP = resident_pad(N, prec);
  if (NP > 0) {
    for (int rb : {16, 32, 64}) {
      const size_t nres = (size_t)(m + rb - 1) / rb;
      if (nres > (size_t)kMaxResidentGrid) continue;
      const size_t NN2 = (size_t)NP * NP;
      need(L.partG, esz * NN2 * nres);
      need(L.partG2, esz * NN2 * nres);
      need(L.partS, sizeof(double) * PS_NS * (size_t)NP * nres);
      need(L.partW, sizeof(double) * NN2 * nres);
      need(L.Gt, esz * 2 * NN2);
      need(L.Gd, esz * NN2);
      need(L.xflags, sizeof(unsigned) * kResidentFlagWords);  // cleared whole every launch
      need(L.pend, sizeof(int) * nres);
    }
  }
  need(L.Wd, sizeof(double) * NN);
  need(L.col, sizeof(double) * CF_NF * (size_t)N);
  need(L.coli, sizeof(int) * CI_NI * (size_t)N);
  need(L.S, esz * (size_t)m * N);
  need(L.D, esz * (size_t)m * N);
  // column solver: S in plane layout, D transposed over padded rows, N flags
  int mp = 0, npc = 0, gv = 0;
  const int col_ok = prec == CGD_FP64 ? columns_shape<double>(m, N, 0, &mp, &npc, &gv)
                                      : columns_shape<float>(m, N, prec == CGD_MIXED_BF16, &mp,
                                                             &npc, &gv);
  if (col_ok) {
    if (L.NPc != npc || L.mp != mp || mp < m || npc < N) ++bad;
    need(L.Scol, esz * (size_t)mp * npc);
    need(L.D, esz * (size_t)N * mp);
    if (prec == CGD_MIXED_BF16) need(L.Scol16, 2 * (size_t)mp * npc);
    if (gv != L.gv) ++bad;
    if (gv) {
      need(L.Vz, esz * (size_t)N * mp);
      need(L.Vr, esz * (size_t)N * mp);
      need(L.Vp, esz * (size_t)N * mp);
      need(L.Rp, esz * (size_t)mp);
    }
  } else if (L.NPc != 0) {
    ++bad;
  }
  // split solver: P row slices of ms rows cover m; one slot pair per member
  // and part for each exchange parity
  if (col_ok || L.splitP > 0) need(L.xw, sizeof(unsigned long long) * (2 * NN + 1));
  // the gather launch ahead of either per-member solver: one error word per
  // workgroup of kCB * 2 / NP padded rows (kCB = 512, NP <= 128: at least 8)
  if (col_ok) need(L.gerr, sizeof(int) * (((size_t)mp + 7) / 8));
  if (L.splitP > 0) need(L.gerr, sizeof(int) * (((size_t)L.splitP * L.splitMs + 7) / 8));
  if (L.splitP > 0) {
    if ((size_t)L.splitP * L.splitMs < (size_t)m || L.splitP > kMaxSplitParts) ++bad;
    const size_t np = N <= 16 ? 16 : N <= 32 ? 32 : 64, rows = (size_t)L.splitP * L.splitMs;
    need(L.xw, sizeof(unsigned long long) * (2 * NN + split_exchange_words(N, L.splitP) + 1));
    need(L.Ssplit, esz * rows * np);
    need(L.Dsplit, esz * (size_t)N * rows);
  }
  // row-block x member-group solver: its exchange words (cleared whole every
  // launch), NG * nblk workgroups covering the rows and the members
  int tnp = 0, trb = 0, tng = 0, tnb = 0;
  if (prec_tile(prec) && tile_shape(m, N, &tnp, &trb, &tng, &tnb)) {
    if (!L.tx || tnp != L.tNP || trb != L.tRB || tng != L.tNG || tnb != L.tnblk) ++bad;
    if ((size_t)trb * tnb < (size_t)m || tng * 32 < N || tnp < N) ++bad;
    need(L.tx, sizeof(unsigned long long) * tile_words(tnp, tng, tnb));
    need(L.tS, sizeof(float) * (size_t)m * tnp);
    need(L.tR, sizeof(float) * (size_t)m);
    need(L.D, sizeof(float) * (size_t)m * N);
    if (tile_part_words(tnp, tng, tnb) >= tile_words(tnp, tng, tnb)) ++bad;
  } else if (L.tx) {
    ++bad;
  }
  return bad;
}

const char* cgd_status_string(int status) {
  switch (status) {
    case CGD_OK: return "CGD_OK";
    case CGD_NOT_CONVERGED: return "CGD_NOT_CONVERGED";
    case CGD_ERR_ARG: return "CGD_ERR_ARG";
    case CGD_ERR_INDEX: return "CGD_ERR_INDEX";
    case CGD_ERR_NONPOS_R: return "CGD_ERR_NONPOS_R";
    case CGD_ERR_NONFINITE: return "CGD_ERR_NONFINITE";
    case CGD_ERR_WORKSPACE: return "CGD_ERR_WORKSPACE";
    case CGD_ERR_HIP: return "CGD_ERR_HIP";
    case CGD_ERR_UNSUPPORTED: return "CGD_ERR_UNSUPPORTED";
    case CGD_ERR_BUSY: return "CGD_ERR_BUSY";
    default: return "CGD_UNKNOWN_STATUS";
  }
}

const char* cgd_version(void) { return "0.1.0"; }

}  // extern "C"
