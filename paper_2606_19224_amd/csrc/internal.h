// Internal declarations of the CGD-EnKF HIP library (gfx950 only).
#pragma once

#include <hip/hip_runtime.h>
#include <stddef.h>
#include <stdint.h>

#include "cgd_enkf.h"

namespace cgd {

constexpr int kBlock = 256;        // threads per workgroup (4 wave64)
constexpr int kMaxGrid = 1024;     // cap on solver workgroups (sizes the partial buffers)
constexpr int kMaxResidentGrid = 1024;  // cap on resident-solver workgroups (exchange flags)
// the resident solver's flag words: arrive and done per workgroup, then the
// 64-bit start-up census word of a plain launch
constexpr int kResidentFlagWords = 2 * kMaxResidentGrid + 2;
// wait of the per-member solvers' start-up census, 100 MHz ticks (1 ms)
constexpr unsigned long long kCensusTicks = 100000;
constexpr int kStallWindow = 5;    // warm-start stall rule: window ...
constexpr double kStallFactor = 0.9;  // ... and required decrease factor

// Per-column double fields, stored field-major: col[f * N + j].
enum ColField { CF_RHO = 0, CF_RHOPREV, CF_DN, CF_AD, CF_ALPHA, CF_BETA, CF_HIST0,
                CF_NF = CF_HIST0 + kStallWindow };
// Per-column int fields: coli[f * N + j].
enum ColIField { CI_ACTIVE = 0, CI_MODE, CI_WARM, CI_FRESH, CI_ITERS, CI_STATUS, CI_FALLBACK,
                 CI_NI };
// Row-pass modes decided per column each iteration.
enum Mode { MODE_FROZEN = 0, MODE_STEP = 1, MODE_RESTART = 2, MODE_ZERO = 3 };
// Column status codes (CI_STATUS).
enum ColStatus { COL_RUNNING = 0, COL_CONVERGED = 1, COL_MAXIT = 2, COL_NONFINITE = 3 };
// Per-WG scalar partials: partS[(w * PS_NS + f) * N + j].
enum PartScalar { PS_RHO = 0, PS_A, PS_B, PS_C, PS_DN, PS_AD, PS_NS };

template <typename T>
struct CGArgs {
  int n, m, N, k, RB, nblk;
  const T* Xf;
  T* Xa;             // column solver applies the update itself
  // the rows the observations are gathered from: X_f itself (ng = n), or,
  // with a non-diagonal R, the whitened anomalies (ng = m, H = I)
  const T* Xg;
  int ng;
  const int32_t* idx;
  const T* hw;       // observation-operator weights
  const T* y;
  const T* rdiag;    // diag(R)
  const T* eps;      // may be null
  const T* z0;       // may be null
  T *S, *D, *Z, *R, *P;
  T* partG;          // nwg * N * N, per-WG S^T r, layout [j][k]
  T* partG2;         // resident solver, warm start: per-WG S^T z0
  unsigned* arrive;  // resident solver: per-WG exchange epochs (arrive, then done)
  unsigned* done;
  int* pend;         // resident solver: per-owner count of columns still moving
  int* err;          // resident solver: set when an exchange wait runs out
  unsigned long long* trace;  // diagnostic phase timestamps (workgroup 0) or null
  // per-member solvers: their gather launch writes one error word per
  // workgroup to gerr (ngerr of them) and also clears zn 32-bit words at zp
  // and *err; the solver folds gerr into *err.  Null gerr: the gather sets
  // *err directly and clears nothing.
  int* gerr;
  unsigned* zp;
  long zn;
  int ngerr;
  double* partS;     // nwg * PS_NS * N
  T* Gt;             // 2 * N * N, G = S^T p for the current row pass, layout [j][k]
  T* Gd;             // N * N, S^T d (restart), layout [j][k]
  double* partW;     // nwg * N * N, double partials of S^T z, layout [j][k]
  double* col;       // CF_NF * N
  int* coli;         // CI_NI * N
  int* ctr;          // 4 counters
  double* Wd;        // N * N, W = S^T Z / (N-1), row-major [k][j]
  double* relres;    // N
  T* z_out;
  int* iters_out;
  double* relres_out;
  double tol;
  int maxit;
  int fallback;
  int want_relres;
  int rr_period;     // mixed mode: inner steps per refinement step, 0 = automatic
  int precond;       // 1: CG on the R^{-1/2}-scaled system (diag(R) preconditioning)
  // per-member solvers: start-up census word (cleared by their gather
  // launch) for a plain launch, or null for a cooperative launch
  unsigned long long* census;
  unsigned long long census_ticks;  // its timeout in 100 MHz ticks
  // row-block x member-group solver: exchange words (partials, then reduced
  // values; zero before the launch), groups and row blocks
  unsigned long long* txp;
  unsigned long long* txr;
  int tNG, tnblk;
  T* tS;  // ... its S (m x NP, row-major) and the rows' diag(R) (m), from its gather
  T* tR;
};

// diag(R) preconditioning by scaling (cgd_precond): row i of S and D is
// multiplied by 1/sqrt(r_i), the scaled system has unit R, a warm start is
// multiplied by sqrt(r_i) and a solution divided by it.
template <typename T>
__device__ inline double precond_row_scale(const CGArgs<T>& a, int i) {
  return a.precond ? 1.0 / sqrt((double)a.rdiag[i]) : 1.0;
}
template <typename T>
__device__ inline T effective_r(const CGArgs<T>& a, int i) {
  return a.precond ? (T)1 : a.rdiag[i];
}
template <typename T>
__device__ inline T precond_z0(const CGArgs<T>& a, int i, T z) {
  return a.precond ? (T)((double)z * sqrt((double)a.rdiag[i])) : z;
}

// One problem of a batched call, as the device sees it (pointers into the
// caller's arrays and into the batch workspace).  The CG runs the column
// solver's per-member recurrence with its vectors in global memory.
template <typename T>
struct BProb {
  int n, m, N, k;
  int NP, mp, RL;  // padded N, padded rows, rows of S cached in LDS
  int gr, ur;      // rows per gather and per update work-table entry
  const T* Xf;
  T* Xa;
  const int32_t* idx;
  const T* hw;
  const T* y;
  const T* rdiag;
  const T* eps;
  T* Sp;           // S in plane layout, mp x NP
  T* Dt;           // D transposed, N x mp
  T *Vz, *Vr, *Vp; // CG vectors, N x mp each
  T* Rp;           // diag(R) padded with zeros, mp
  double* Wd;      // N * N
  double* col;     // CF_NF * N
  int* coli;       // CI_NI * N
  int* iters_out;  // N or null
};

// Workspace layout shared by the API and the launchers.
struct Layout {
  size_t S, D, Z, R, P, partG, partG2, partS, Gt, Gd, partW, col, coli, ctr, Wd, relres, flags;
  size_t Scol;     // column solver: S in plane layout (mp x NPc), 0 if not applicable
  size_t Scol16;   // mixed mode: BF16 copy of it (mp x NPc), 0 if not applicable
  size_t xw;       // published W (2 N^2 words), then the split solver's exchange slots
  size_t gerr;     // per-member solvers: their gather launch's per-workgroup error words
  size_t xwords;   // 64-bit words of xw
  size_t Ssplit, Dsplit;  // split solver: S in slices, D transposed (0 if not applicable)
  int splitP, splitMs;  // split solver: workgroups per member, rows per workgroup
  int mp, NPc;     // column solver: padded rows and padded N (0 if not applicable)
  size_t Vz, Vr, Vp, Rp;  // column solver with vectors in global memory (0 otherwise)
  int gv;
  size_t xflags, pend, err;
  int NP;  // partial/Gram stride: max(N, resident padding of N)
  // reduced mode (rNP != 0: the MFMA path, with Q = [P | Yt] at rQ and
  // (W - I)^T at rWt; otherwise the scalar path for N > 128)
  size_t rpart, rG, rB, riters, rstat, rQ, rWt, rerr;
  // non-diagonal R (mode bit 2): whitening scratch and substitute inputs
  size_t tSd, tDd, tXp, tEp, tidx, tw, ty, tr, tzt, terr;
  int rNP, rmpad, rKC, rS;
  // row-block x member-group solver (FP32): its exchange words (0 if not
  // applicable) and shape
  size_t tx, tS, tR;
  int tNP, tRB, tNG, tnblk;
  size_t total;
  int RB, nblk, nwg_max;
};

Layout make_layout(int n, int m, int N, int k, int prec, int mode);

// Launchers (return hipError_t from the launch).
template <typename T>
hipError_t launch_cg_solve(const CGArgs<T>& a, int nwg, hipStream_t s);
template <typename T>
int cg_max_coresident(int RB, int N);
hipError_t launch_zero_u32(unsigned* p, int n, hipStream_t s);
template <typename T>
int resident_np(int N);
template <typename T>
int resident_coresident(int NP, int RB);
// Column-parallel solver (cg_columns.hip): a gather launch, then one
// workgroup per member, S streamed through L2; applies the ensemble update
// itself after publishing W as flag-in-word values in wb (2 N^2 words,
// zero before the launch).
constexpr int kColumnsMaxRows = 1 << 22;  // keeps the column solver's index arithmetic in int
// Column solver geometry: padded rows mp, padded N (NPc: 16, 32, 64, or 128
// in FP32), and gv = 1 when its CG vectors live in global memory (z, r, p:
// N x mp each, diag(R) padded to mp) because they do not fit in LDS.
template <typename T>
int columns_shape(int m, int N, int mix, int* mp, int* NPc, int* gv);
template <typename T>
int columns_coresident(int m, int N, int mix);
template <typename T>
hipError_t launch_cg_columns(const CGArgs<T>& a, T* Sp, __bf16* Sh, unsigned long long* wb,
                             T* Vz, T* Vr, T* Vp, T* Rp, hipEvent_t* ev, hipStream_t s);
// Split solver (cg_columns.hip): a gather launch writing S in slices (Sg,
// P * ms * NP) and D transposed (Dg, N x P * ms), then P workgroups per
// member, each with its ms rows of S in LDS, partial sums exchanged once per
// pass through xb (split_exchange_words, zero before the launch); applies
// the update itself as the column solver does.
constexpr int kMaxSplitParts = 16;
template <typename T>
int split_shape(int m, int N, int* P, int* ms);  // 0 when no slice fits the LDS
template <typename T>
int split_coresident(int N, int P, int ms);
size_t split_exchange_words(int N, int P);       // 64-bit words of the exchange slots
template <typename T>
hipError_t launch_cg_split(const CGArgs<T>& a, int P, int ms, T* Sg, T* Dg,
                           unsigned long long* xb, unsigned long long* wb, hipEvent_t* ev,
                           hipStream_t s);  // ev[0] is recorded after the gather launch
// Bytes of S the column solver streams through L2 per member and pass (the
// rows its LDS cache does not hold).
template <typename T>
size_t columns_streamed_bytes(int m, int N);
template <typename T>
hipError_t launch_cg_resident(const CGArgs<T>& a, int NP, int RB, int nwg, hipStream_t s);
// Row-block x member-group solver (cg_tile.hip), FP32, N <= 128: members in
// groups of 32, RB observation rows per workgroup, NG * nblk workgroups,
// all co-resident.  tile_shape returns 0 when the shape is out of its range.
int tile_shape(int m, int N, int* NP, int* RB, int* NG, int* nblk);
// variant: 0 FP32, 1 the mixed mode, 2 the split-BF16 mode
int tile_coresident(int NP, int RB, int variant);
size_t tile_part_words(int NP, int NG, int nblk);  // partial words (the reduced ones follow)
size_t tile_words(int NP, int NG, int nblk);       // all exchange words, with the census word last
// Zeroes the exchange words, runs the gather, then launches the solver
// (a.txp, a.txr, a.tNG, a.tnblk, a.tS, a.tR set; a.census null for a
// cooperative launch); variant 0: FP32, 1: the mixed mode (BF16 inner CG,
// FP64 outer residual), 2: the split-BF16 mode (five BF16 products per
// S-product, FP64 final step).
hipError_t launch_cg_tile(const CGArgs<float>& a, int NP, int RB, int variant, hipStream_t s);
// Batched mode (cg_columns.hip): gather, per-member CG and update launches
// over work tables of (problem, row block), (problem, member) and (problem,
// row block) entries; a problem's row blocks are BProb::gr and BProb::ur rows.
constexpr int kBatchRowsDefault = 256;  // rows per gather / update entry unless a problem sets them
template <typename T>
int batched_shape(int m, int N, int* NP, int* mp, int* RL);  // 0 when N is out of range
template <typename T>
hipError_t launch_batched(const BProb<T>* probs, const int2* gtab, int ngather,
                          const int2* stab, int nsolve, const int2* utab, int nupdate,
                          double tol, int maxit, int precond, int* err, hipEvent_t* ev,
                          hipStream_t s);
// z_out of a diag(R)-preconditioned solve back to the original variables:
// z[i][j] /= sqrt(r[i]).
template <typename T>
hipError_t launch_unscale_rows(int m, int N, T* z, const T* rdiag, hipStream_t s);
// X_a from W (mode 0: X_f + A W, mode 1: X_f W); with `skip`, the launch
// writes nothing when bit 2 of *skip is set.
template <typename T>
hipError_t launch_update(int n, int N, const T* Xf, T* Xa, const double* Wd, int mode,
                         hipStream_t s, const int* skip = nullptr);
// Geometry of the reduced mode's MFMA path (N <= 128): N padded to NP (32,
// 64 or 128), m padded to mpad (a multiple of 32), KC rows per chunk of the
// N x 2N product and S chunks.  0 when N is out of range.
int reduced_shape(int m, int N, int* NP, int* mpad, int* KC, int* S);
// Xg (ng rows) is the array the observations are gathered from; Xf is
// updated (the same unless R is not diagonal)
template <typename T>
hipError_t launch_reduced(int n, int m, int N, int k, const T* Xf, T* Xa, const T* Xg, int ng,
                          const int32_t* idx, const T* hw, const T* y, const T* rdiag,
                          const T* eps, double tol, int maxit, void* ws, const Layout& L,
                          int* iters_out, hipStream_t s);
template <typename T>
hipError_t launch_validate(int n, int m, int N, int k, const T* Xf, const int32_t* idx,
                           const T* hw, const T* y, const T* rdiag, const T* eps, const T* z0,
                           int* flags, hipStream_t s);

// Non-diagonal R = L L^T (whiten.hip): scratch of the whitening pass and
// the substitute inputs the solvers then run on.
template <typename T>
struct TriBuffers {
  double* Sd;      // m x N, S in double
  double* Dd;      // m x N, D in double
  T* Xp;           // m x N, S~ = L^{-1} S (the observations' rows, H = I)
  T* Ep;           // m x N, D~ + S~
  int32_t* idxp;   // m, idx' = i
  T* wp;           // m, w' = 1
  T* yp;           // m, y' = 0
  T* rp;           // m, R' = I
  T* zt;           // m x N, L^T z0 (warm start) or null
  int* err;        // index error of the whitening pass (bit 1)
};
template <typename T>
hipError_t launch_tri_whiten(int n, int m, int N, int k, const T* Xf, const int32_t* idx,
                             const T* hw, const T* y, const T* eps, const T* Lf, const T* z0,
                             const TriBuffers<T>& tb, int* err, hipStream_t s);
template <typename T>
hipError_t launch_tri_back(int m, int N, const T* Lf, T* z, hipStream_t s);
template <typename T>
hipError_t launch_tri_chol(int m, const T* r, const T* o, T* Lf, int* bad, hipStream_t s);
hipError_t launch_or_u32(int* dst, const int* src, hipStream_t s);

// Validation flag bits.
enum { VF_INDEX = 1, VF_NONPOS_R = 2, VF_NONFINITE = 4 };

}  // namespace cgd
