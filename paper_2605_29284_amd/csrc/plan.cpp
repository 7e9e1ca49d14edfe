// C-ABI entry points of libkrig: plan set-up (Steps 1-4 of Section 2.2 and the
// kriging-system factorisation) and the per-call sequences (solve, scatter,
// convolution, adjoint, conditional simulation).
#include <hip/hip_runtime.h>
#include <math.h>
#include <string.h>
#include <stdlib.h>

#include <algorithm>
#include <map>
#include <tuple>
#include <mutex>
#include <new>
#include <cmath>
#include <vector>

#include "../../include/krig.h"
#include "dense.h"
#include "exact.h"
#include "interp.h"
#include "mixture.h"
#include "universal.h"
#include "fft_args.h"
#include "fft_reg.h"
#include "setup.h"

using namespace krig;

namespace {

struct DevBuf {
  void* p = nullptr;
  size_t bytes = 0;
};

}  // namespace

// Site sets with at least this many CSR entries per padded node on average (n M / (P1 P2)) take
// the scatter's own kernel before the row transforms instead of the scatter fused into them, in
// calls of fewer than SCATTER_SPLIT_MAX_B fields: with many fields the fused form has threads
// enough, and the image's write and read cost more than they save (256 fields on a 520 x 520
// padded grid: 2.38 against 2.24 ms per convolution).
constexpr int SCATTER_SPLIT_MIN_DENSITY = 1;
constexpr int SCATTER_SPLIT_MAX_B = 64;

struct krig_plan_s {
  hipStream_t st = nullptr;
  int device = 0;  // the GPU that was current at plan creation (holds every buffer)
  int dtype = KRIG_F32;
  size_t tsz = 4;  // bytes of one real dt value
  GridDev g{};
  MaternDev mt{};
  int n = 0, M = 0, P1 = 0, P2 = 0, F1 = 0, F2 = 0, H2 = 0;
  int ldP = 0;  // pitch of frequency-major spectra with P1 rows
  int ldM = 0;  // ... with m1 rows
  int ldX = 0;  // ... with 2 (m1 + L) - 1 rows
  int n1l = 0, n2l = 0;
  const FftEntry* e1 = nullptr;  // columns (length F1)
  const FftEntry* e1h = nullptr; // the length F1 / 2 whose paired column kernels serve F1, if any
  int cols_pair = 0;             // 0: the column passes' own form; k >= 1: paired, k columns per block
  int scatter_split = 0;         // 1: scatter into fimg by its own kernel, then the row transforms
  const FftEntry* e2 = nullptr;  // rows (length F2)
  int var_cols = 0, var_rows = 0;  // which compiled form of F1 / F2 (0: the default)
  // twiddles exp(-2 pi i j / F)
  double* tw1_64 = nullptr;
  double* tw2_64 = nullptr;
  float* tw1_32 = nullptr;
  float* tw2_32 = nullptr;
  // set-up products
  double* sites = nullptr;
  double* lag64 = nullptr;
  void* lagT = nullptr;
  double* filt = nullptr;  // [H2][F1] filter spectrum / (F1 F2), FP64
  int filt_setup = KRIG_FILTER_REFLECTED;  // how filt was built
  double* KN = nullptr;     // K_N as factored (jitter included when it was needed)
  double* LinvN = nullptr;
  int* d_status = nullptr;   // [0] K_N status, [1] M pivot
  int32_t* anchor = nullptr;
  double* kvec = nullptr;
  double* W = nullptr;
  double* Wt = nullptr;     // [M][n] transposed weights, columns in the gather order
  int32_t* gorder = nullptr; // [n] the gather order: sites sorted by anchor cell
  int32_t* ganchor = nullptr; // [n][2] the anchors in that order (slot s: anchor of gorder[s])
  double* Wr = nullptr;     // [n][M] residual of the weight refinement
  int32_t* node_ptr = nullptr;
  int32_t* ent_site = nullptr;
  double* ent_w = nullptr;
  CsrWork cw{};
  double* Lfac = nullptr;  // Cholesky factor of K + tau^2 I
  double* Linv = nullptr;  // its inverse
  double* LinvT = nullptr;  // and the transpose of that
  int64_t ldL = 0;  // pitch of Lfac, Linv, LinvT (n + 1 rounded up to 16: at least one zero pad column)
  double* Dinv = nullptr;
  double* work = nullptr;
  int kn_status = 0, pivot = 0;
  // per-call workspaces
  int wsB = 0;
  void* S1 = nullptr;     // cx FP64 [B][H2][ldP]   row spectra of c*
  void* S2 = nullptr;     // cx dt   [B][H2][ldM]   prediction column-pass output
  void* SG = nullptr;     // cx FP64 [B][H2][ldM]   row spectra of the upstream gradient
  void* SA = nullptr;     // cx FP64 [B][H2][ldP]   adjoint column-pass output
  void* img = nullptr;    // FP64 [B][P1][P2]       correlation image
  double* alpha = nullptr;  // [B][n]
  double* tmpv = nullptr;   // [B][ldv]  between the two triangular products
  double* fimg = nullptr;   // [min(B, 63)][P1][P2] the scattered image, when the scatter has its own kernel
  int fimgB = 0;            // fields the image holds
  bool fimg_needed = false; // a call took the scatter apart: keep the image when the workspaces grow
  int64_t ldv = 0;          // n rounded up to 4: 32-byte rows for vector loads
  void* part = nullptr;   // cx FP64 [ngroups][H2][F1]
  int part_groups = 0;
  void* XC = nullptr;     // cx FP64 [H2][ldX]
  void* mix = nullptr;    // dt [B][m1][m2]  this plan's component of a mixture prediction
  int wsB_mix = 0;
  // universal kriging
  double* uk_vx = nullptr;    // [UK_MAX][n]  M^{-1} X, one covariate per row
  double* uk_G = nullptr;     // [UK_MAX][UK_MAX + B]  X^T M^{-1} [X | z]
  double* uk_beta = nullptr;  // [B][UK_MAX]
  int wsB_uk = 0;
  // custom-lag filter
  double* filtC = nullptr;
  double* lagC64 = nullptr;
  double* phiS64 = nullptr;  // cx double [H2][F1]
  // launch shapes
  int nl_rows64 = 4;   // lines per block, FP64 row kernels
  int nl_cols64 = 4;   // columns per block, FP64-forward column kernels
  int dlag_G = 1;       // fields per block of the lag-gradient column pass
  // conditional simulation (set up on the first krig_csim call)
  int ce_clamped = 0;
  int Fs1 = 0, Fs2 = 0, Hs2 = 0;
  const FftEntry* es1 = nullptr;  // torus columns (length Fs1)
  const FftEntry* es2 = nullptr;  // torus rows (length Fs2)
  double *tws1_64 = nullptr, *tws2_64 = nullptr;
  float *tws1_32 = nullptr, *tws2_32 = nullptr;
  double* lamS = nullptr;   // sqrt(Lambda / (Fs1 Fs2)), [Hs2][Fs1]
  int csR = 0;
  void* csT = nullptr;      // cx dt [pairs][Fs2][ldP]
  void* csU = nullptr;      // dt [R][P1][P2] unconditional fields
  double* csRes = nullptr;  // [R][n]
  double* csAl = nullptr;   // [R][n]
  int wsB_adj = 0;
  // stage timing
  bool timing = false;
  int batch_refs = 0;  // recorded batches (graphs) holding pointers into the workspaces
  std::vector<hipEvent_t> ev_pool;
  // second stream of the adjoint (lag-gradient tail beside the gather and solve), with its
  // fork and join events; created with the adjoint workspaces
  hipStream_t aux = nullptr;
  hipEvent_t ev_fork = nullptr, ev_join = nullptr;
  std::vector<std::pair<hipEvent_t, hipEvent_t>> ev_pending[KRIG_STAGE_COUNT];
  std::vector<void*> allocs;
};

namespace {

std::once_flag g_once;

int hip_status(hipError_t e) { return e == hipSuccess ? KRIG_OK : KRIG_EHIP; }

hipEvent_t take_event(krig_plan p) {
  if (!p->ev_pool.empty()) {
    hipEvent_t e = p->ev_pool.back();
    p->ev_pool.pop_back();
    return e;
  }
  hipEvent_t e = nullptr;
  if (hipEventCreate(&e) != hipSuccess) return nullptr;
  return e;
}

// Brackets the launches of one stage with events when timing is on.
struct StageTimer {
  krig_plan p;
  int stage;
  hipEvent_t a = nullptr, b = nullptr;
  StageTimer(krig_plan p_, int s_) : p(p_), stage(s_) {
    if (p->timing) {
      a = take_event(p);
      b = take_event(p);
      if (a && b) (void)hipEventRecord(a, p->st);
    }
  }
  ~StageTimer() {
    if (a && b) {
      (void)hipEventRecord(b, p->st);
      p->ev_pending[stage].push_back({a, b});
    } else {
      if (a) p->ev_pool.push_back(a);
      if (b) p->ev_pool.push_back(b);
    }
  }
};

#define KRIG_TRY(expr)                         \
  do {                                         \
    hipError_t _e = (expr);                    \
    if (_e != hipSuccess) return KRIG_EHIP;    \
  } while (0)

template <typename T>
int dalloc(krig_plan p, T** out, size_t count) {
  void* q = nullptr;
  if (count == 0) count = 1;
  if (hipMalloc(&q, count * sizeof(T)) != hipSuccess) {
    *out = nullptr;
    return KRIG_ENOMEM;
  }
  p->allocs.push_back(q);
  *out = static_cast<T*>(q);
  return KRIG_OK;
}

int dalloc_bytes(krig_plan p, void** out, size_t bytes) {
  char* q = nullptr;
  int s = dalloc(p, &q, bytes);
  *out = q;
  return s;
}

void dfree(krig_plan p, void* q) {
  if (!q) return;
  auto it = std::find(p->allocs.begin(), p->allocs.end(), q);
  if (it != p->allocs.end()) p->allocs.erase(it);
  (void)hipFree(q);
}

int pick_fft(int need) {
  int sizes[64];
  const int k = fft_sizes(sizes, 64);
  int best = -1;
  for (int i = 0; i < k && i < 64; ++i)
    if (sizes[i] >= need && (best < 0 || sizes[i] < best)) best = sizes[i];
  return best;
}

int nt_of(const FftEntry* e) { return e->geo.NT; }

// largest lines (row kernels) / columns (column kernels) per block with at most 256
// threads and 64 KB of LDS
int nl_rows_for(const FftEntry* e, size_t csz) {
  int nl = std::max(1, 256 / nt_of(e));
  while (nl > 1 && rows_lds(e->geo, nl, csz) > 64 * 1024) --nl;
  return nl;
}
int nl_cols_for(const FftEntry* e, size_t csz) {
  int nl = std::max(1, 256 / nt_of(e));
  while (nl > 1 && cols_lds(e->geo, nl, csz) > 64 * 1024) --nl;
  return nl;
}
int pitch16(int rows) { return (rows + 15) / 16 * 16; }

// (cos, sin) of 2 pi j / F in x86 extended precision (64-bit significand), by the same
// exact octant reduction as trig_frac; only used to measure the rounding of the tables.
void trig_ext(long j, long F, long double* c, long double* s) {
  const long double pi = 3.14159265358979323846264338327950288L;
  long r = ((j % F) + F) % F, o = (8 * r) / F, num = 8 * r - o * F;
  const long double x = (pi / 4) * ((long double)num / (long double)F), y = pi / 4 - x;
  const long double sx = std::sin(x), cx_ = std::cos(x), sy = std::sin(y), cy = std::cos(y);
  const long double C[8] = {cx_, sy, -sx, -cy, -cx_, -sy, sx, cy};
  const long double S[8] = {sx, cy, cx_, sy, -sx, -cy, -cx_, -sy};
  *c = C[o];
  *s = S[o];
}

// Relative rounding error d = (exact - t) / t of a table entry t, as an FP32 complex pair.
template <typename T>
void rel_err(long double ec, long double es, T tc, T ts, float* d) {
  const long double hr = tc, hi = ts, er = ec - hr, ei = es - hi, den = hr * hr + hi * hi;
  d[0] = (float)((er * hr + ei * hi) / den);
  d[1] = (float)((ei * hr - er * hi) / den);
}

// Twiddle tables exp(-2 pi i j / F), j < F, in FP64 and FP32.  Each table of F complex
// entries is followed by F complex FP32 values d_j, the relative rounding error of entry
// j: a kernel that forms W^(jk) as the k-th power of entry j corrects it by (1 + k d_j).
int make_twiddles(krig_plan p, int F, double** d64, float** d32) {
  std::vector<double> h64(3 * (size_t)F);  // 2F doubles, then 2F floats
  std::vector<float> h32(4 * (size_t)F);
  float* e64 = reinterpret_cast<float*>(h64.data() + 2 * (size_t)F);
  for (int j = 0; j < F; ++j) {
    const double c = trig_frac(j, F, true), s = -trig_frac(j, F, false);
    h64[2 * j] = c;
    h64[2 * j + 1] = s;
    h32[2 * j] = (float)c;
    h32[2 * j + 1] = (float)s;
    long double ec, es;
    trig_ext(j, F, &ec, &es);
    es = -es;
    rel_err(ec, es, c, s, e64 + 2 * j);
    rel_err(ec, es, h32[2 * j], h32[2 * j + 1], h32.data() + 2 * (size_t)F + 2 * j);
  }
  int r;
  if ((r = dalloc(p, d64, h64.size())) != KRIG_OK) return r;
  if ((r = dalloc(p, d32, h32.size())) != KRIG_OK) return r;
  KRIG_TRY(hipMemcpyAsync(*d64, h64.data(), h64.size() * sizeof(double), hipMemcpyHostToDevice, p->st));
  KRIG_TRY(hipMemcpyAsync(*d32, h32.data(), h32.size() * sizeof(float), hipMemcpyHostToDevice, p->st));
  KRIG_TRY(hipStreamSynchronize(p->st));  // host vectors go out of scope
  return KRIG_OK;
}

const FftSet& set1(krig_plan p) { return p->e1->k; }
const FftSet& set2(krig_plan p) { return p->e2->k; }

// The convolution column pass (forward, filter product, inverse; FP32 output spectra for the
// prediction of FP32 plans when f32out): the column form of e1, or the paired form of e1h.
launch_cols_t conv_cols_fn(krig_plan p, bool f32out) {
  if (p->cols_pair) return f32out ? p->e1h->k.pair_conv_pred_f : p->e1h->k.pair_conv64;
  return f32out ? set1(p).conv_pred_f : set1(p).conv64;
}
int conv_cols_nl(krig_plan p) { return p->cols_pair ? p->cols_pair : p->nl_cols64; }
bool is32(krig_plan p) { return p->dtype == KRIG_F32; }
size_t csz(krig_plan p) { return 2 * p->tsz; }

// Bytes per complex value of each spectrum that passes between the transform kernels.
// FP64 plans store FP64 throughout.  FP32 plans (FP64 arithmetic in every pass) store the
// column pass's output of the prediction in FP32 (8 bytes): one rounding there moves y_hat
// by up to ~3e-6 on cancellation-heavy problems (sum |c*| / max |y_hat| ~ 1e5), ~1e-7 on the
// rest, and halves that pass's writes and the inverse rows' reads.  Everything else stays
// FP64:
//  - the row spectra of c*: one FP32 rounding there moves y_hat by up to ~3e-5 on
//    cancellation-heavy problems;
//  - the adjoint's correlation spectra: d y applies (K + tau^2 I)^{-1} to them, and one FP32
//    rounding moves d y by ~1e-4;
//  - the upstream gradient's row spectra and the lag-gradient partials: FP32 storage there was
//    harmless (~1e-7 in d y) but measured 1 us per step slower, since the conversions add to
//    the lag-gradient column pass's FP64 arithmetic, which bounds it, while its bytes do not.
enum SpecRole { SPEC_C, SPEC_PRED, SPEC_G, SPEC_CORR, SPEC_PART };
size_t spec_bytes(krig_plan p, SpecRole role) {
  if (!is32(p)) return 16;
  return role == SPEC_PRED ? 8 : 16;
}

// spectrum of the even-reflected lag quadrant (FP64), scaled by 1/(F1 F2)
int make_filter(krig_plan p, const double* lag64, double* filt_out) {
  RowsR2CArgs r{};
  r.nrows = p->F1;
  r.H2 = p->H2;
  r.out = p->phiS64;
  r.out_fs = 0;
  r.out_ld = p->F1;
  r.twF = p->tw2_64;
  r.lag = lag64;
  r.n1l = p->n1l;
  r.n2l = p->n2l;
  r.F1 = p->F1;
  r.NL = nl_rows_for(p->e2, 16);
  KRIG_TRY(p->e2->k.r2c_lag(r, 1, p->st));
  ColsArgs c{};
  c.H2 = p->H2;
  c.in = p->phiS64;
  c.in_fs = 0;
  c.in_ld = p->F1;
  c.in_off = 0;
  c.in_cnt = p->F1;
  c.out = filt_out;
  c.out_fs = 0;
  c.out_ld = p->F1;
  c.twF = p->tw1_64;
  c.twI = p->tw1_64;
  c.scale = 1.0 / ((double)p->F1 * (double)p->F2);
  c.NL = nl_cols_for(p->e1, 16);
  KRIG_TRY(p->e1->k.fwd_real64(c, 1, p->st));
  return KRIG_OK;
}

// The alternative set-up of the remark after Step 7 (no reflection, one more transform): the
// covariance between the torus centre node (F1/2, F2/2) and every torus node from plain
// coordinate differences, transformed, divided by the transform of the centre's indicator.
// Both transforms keep the real parts: the centred image is even about the centre, so its
// transform is the filter spectrum times the centre's real phase (-1)^(k1 + k2), which the
// indicator's transform holds.  Every lag up to half the torus is filled (the reflected
// construction has zeros beyond the quadrant); those lags never reach a kept output.
int make_filter_centered(krig_plan p, double* filt_out) {
  for (int pass = 0; pass < 2; ++pass) {
    RowsR2CArgs r{};
    r.nrows = p->F1;
    r.H2 = p->H2;
    r.out = p->phiS64;
    r.out_fs = 0;
    r.out_ld = p->F1;
    r.twF = p->tw2_64;
    r.F1 = p->F1;
    r.cov_sigma2 = p->mt.sigma2;
    r.cov_rho = p->mt.rho;
    r.cov_dx = p->g.dx;
    r.cov_dy = p->g.dy;
    r.cov_kind = p->mt.kind;
    r.NL = nl_rows_for(p->e2, 16);
    KRIG_TRY((pass == 0 ? p->e2->k.r2c_center : p->e2->k.r2c_delta)(r, 1, p->st));
    ColsArgs c{};
    c.H2 = p->H2;
    c.in = p->phiS64;
    c.in_fs = 0;
    c.in_ld = p->F1;
    c.in_off = 0;
    c.in_cnt = p->F1;
    c.out = pass == 0 ? filt_out : p->filtC;  // filtC: scratch for the indicator's transform
    c.out_fs = 0;
    c.out_ld = p->F1;
    c.twF = p->tw1_64;
    c.twI = p->tw1_64;
    c.scale = pass == 0 ? 1.0 / ((double)p->F1 * (double)p->F2) : 1.0;
    c.NL = nl_cols_for(p->e1, 16);
    KRIG_TRY(p->e1->k.fwd_real64(c, 1, p->st));
  }
  KRIG_TRY(div_f64(filt_out, p->filtC, (int64_t)p->H2 * p->F1, p->st));
  return KRIG_OK;
}

// forward workspaces (prediction and solves) for B fields
bool use_split(krig_plan p, int B) { return p->scatter_split && B < SCATTER_SPLIT_MAX_B; }
// whether a call of B fields takes the scatter apart now: its form says so and the image is there
// (a workspace sized for more fields than the split takes has none until such a call sizes it)
bool split_now(krig_plan p, int B) { return use_split(p, B) && p->fimg && B <= p->fimgB; }

int ensure_ws(krig_plan p, int B) {
  // with the workspaces big enough, a missing image only means the fused scatter (the same
  // bits); it is allocated unless a recorded batch holds the buffers
  if (B <= p->wsB && (!use_split(p, B) || (p->fimg && B <= p->fimgB) || p->batch_refs > 0)) return KRIG_OK;
  if (p->batch_refs > 0) return KRIG_EINVAL;  // a recorded graph uses the current buffers
  const bool img = p->scatter_split && (use_split(p, B) || p->fimg_needed);
  B = std::max(B, p->wsB);  // never shrink what earlier calls sized
  void* olds[] = {p->S1, p->S2, p->alpha, p->tmpv, p->fimg};
  KRIG_TRY(hipStreamSynchronize(p->st));
  for (void* q : olds) dfree(p, q);
  p->fimg = nullptr;
  p->fimgB = 0;
  const size_t H2 = p->H2;
  int r;
  if ((r = dalloc_bytes(p, &p->S1, spec_bytes(p, SPEC_C) * (size_t)B * H2 * p->ldP)) != KRIG_OK) return r;
  if ((r = dalloc_bytes(p, &p->S2, spec_bytes(p, SPEC_PRED) * (size_t)B * H2 * p->ldM)) != KRIG_OK) return r;
  if ((r = dalloc(p, &p->alpha, (size_t)B * p->n)) != KRIG_OK) return r;
  p->ldv = (p->n + 3) / 4 * 4;
  if ((r = dalloc(p, &p->tmpv, (size_t)B * p->ldv)) != KRIG_OK) return r;
  // the scatter's image, for the calls that take the scatter apart (fewer than SCATTER_SPLIT_MAX_B
  // fields): allocated with the first such call
  if (img) {
    p->fimgB = std::min(B, SCATTER_SPLIT_MAX_B - 1);
    if ((r = dalloc(p, &p->fimg, (size_t)p->fimgB * p->P1 * p->P2)) != KRIG_OK) return r;
  }
  p->fimg_needed = p->fimg != nullptr;
  p->wsB = B;
  return KRIG_OK;
}

// adjoint workspaces for B fields
int ensure_ws_adj(krig_plan p, int B) {
  if (!p->aux) {  // default priority, no implicit synchronisation with the null stream
    KRIG_TRY(hipStreamCreateWithFlags(&p->aux, hipStreamNonBlocking));
    KRIG_TRY(hipEventCreateWithFlags(&p->ev_fork, hipEventDisableTiming));
    KRIG_TRY(hipEventCreateWithFlags(&p->ev_join, hipEventDisableTiming));
  }
  if (B <= p->wsB_adj) return KRIG_OK;
  if (p->batch_refs > 0) return KRIG_EINVAL;
  void* olds[] = {p->SG, p->SA, p->img, p->part};
  KRIG_TRY(hipStreamSynchronize(p->st));
  for (void* q : olds) dfree(p, q);
  const size_t H2 = p->H2;
  int r;
  if ((r = dalloc_bytes(p, &p->SG, spec_bytes(p, SPEC_G) * (size_t)B * H2 * p->ldM)) != KRIG_OK) return r;
  if ((r = dalloc_bytes(p, &p->SA, spec_bytes(p, SPEC_CORR) * (size_t)B * H2 * p->ldP)) != KRIG_OK) return r;
  if ((r = dalloc_bytes(p, &p->img, 8 * (size_t)B * p->P1 * p->P2)) != KRIG_OK) return r;
  p->part_groups = B;  // worst case G = 1
  if ((r = dalloc_bytes(p, &p->part, spec_bytes(p, SPEC_PART) * (size_t)p->part_groups * H2 * p->F1)) != KRIG_OK)
    return r;
  p->wsB_adj = B;
  return KRIG_OK;
}

// mixture-component output for B fields
int ensure_ws_mix(krig_plan p, int B) {
  if (B <= p->wsB_mix) return KRIG_OK;
  if (p->batch_refs > 0) return KRIG_EINVAL;
  KRIG_TRY(hipStreamSynchronize(p->st));
  dfree(p, p->mix);
  p->mix = nullptr;
  int r;
  if ((r = dalloc_bytes(p, &p->mix, p->tsz * (size_t)B * p->g.m1 * p->g.m2)) != KRIG_OK) return r;
  p->wsB_mix = B;
  return KRIG_OK;
}

// universal-kriging workspaces for B fields
int ensure_ws_uk(krig_plan p, int B) {
  if (B <= p->wsB_uk) return KRIG_OK;
  if (p->batch_refs > 0) return KRIG_EINVAL;
  KRIG_TRY(hipStreamSynchronize(p->st));
  dfree(p, p->uk_G);
  dfree(p, p->uk_beta);
  p->uk_G = p->uk_beta = nullptr;
  int r;
  if (!p->uk_vx && (r = dalloc(p, &p->uk_vx, (size_t)UK_MAX * p->n)) != KRIG_OK) return r;
  if ((r = dalloc(p, &p->uk_G, (size_t)UK_MAX * (UK_MAX + B))) != KRIG_OK) return r;
  if ((r = dalloc(p, &p->uk_beta, (size_t)B * UK_MAX)) != KRIG_OK) return r;
  p->wsB_uk = B;
  return KRIG_OK;
}

// K_N factor and inverse factor for more than 64 neighbours (L > 4): the blocked Cholesky of
// the kriging system applied to K_N, with the same single jitter retry as the one-tile
// kernel (1e-14 sigma2 M on the diagonal) decided on the host; the outcome goes to
// d_status[0] as the one-tile kernel reports it (0 clean, 1 jitter used, -pivot failed).
int kn_factor_large(krig_plan p) {
  const int M = p->M;
  double *A = nullptr, *Dv = nullptr, *wk = nullptr;
  int r;
  if ((r = dalloc(p, &A, (size_t)M * M)) != KRIG_OK) return r;
  if ((r = dalloc(p, &Dv, (size_t)((M + 63) / 64) * 4096)) != KRIG_OK) return r;
  if ((r = dalloc(p, &wk, (size_t)64 * M)) != KRIG_OK) return r;
  int status = 0;
  for (int attempt = 0; attempt < 2; ++attempt) {
    const double jit = attempt ? 1e-14 * p->mt.sigma2 * M : 0.0;
    KRIG_TRY(kn_assemble(p->g, p->mt, p->KN, A, jit, p->st));
    KRIG_TRY(hipMemsetAsync(p->d_status + 2, 0, sizeof(int), p->st));
    KRIG_TRY(cholesky_and_inverse(A, M, M, p->LinvN, Dv, wk, p->d_status + 2, p->st));
    int piv = 0;
    KRIG_TRY(hipMemcpyAsync(&piv, p->d_status + 2, sizeof(int), hipMemcpyDeviceToHost, p->st));
    KRIG_TRY(hipStreamSynchronize(p->st));
    if (piv == 0) {
      status = attempt;
      break;
    }
    status = -piv;
  }
  KRIG_TRY(hipMemcpyAsync(p->d_status, &status, sizeof(int), hipMemcpyHostToDevice, p->st));
  KRIG_TRY(hipStreamSynchronize(p->st));
  dfree(p, A);
  dfree(p, Dv);
  dfree(p, wk);
  return KRIG_OK;
}

// Step 4: W = K_N^{-1} k for all sites (d_kvec [n][M]): the two FP64 MFMA products with the
// inverse factor, (k L_N^{-T}) L_N^{-1}, then WEIGHT_REFINE steps of iterative refinement in
// FP64, R = k - W K_N and W += (R L_N^{-T}) L_N^{-1}.  The products alone leave a residual of
// about cond(K_N) eps |k| (1e-9 for the paper-sized field, cond(K_N) ~ 3e13); refined, it meets
// the backward-stable bound ~M eps |K_N| |w| of a direct solve.  Leaves Wt rebuilt from W.
constexpr int WEIGHT_REFINE = 2;
int weights_from_kvec(krig_plan p, const double* d_kvec) {
  const int n = p->n, M = p->M;
  GemmArgs ga{};  // X L_N^{-T}
  ga.lda = M; ga.transA = 0;
  ga.B = p->LinvN; ga.ldb = M; ga.transB = 1;
  ga.ldc = M;
  ga.m_off = 0; ga.M_end = n; ga.n_off = 0; ga.N_end = M; ga.K = M;
  ga.alpha = 1.0; ga.beta = 0.0; ga.lower = 0;
  GemmArgs gb = ga;  // Y L_N^{-1}
  gb.transB = 0;
  ga.A = d_kvec; ga.C = p->Wt;
  KRIG_TRY(gemm_f64(ga, p->st));
  gb.A = p->Wt; gb.C = p->W;
  KRIG_TRY(gemm_f64(gb, p->st));
  for (int it = 0; it < WEIGHT_REFINE; ++it) {
    KRIG_TRY(hipMemcpyAsync(p->Wr, d_kvec, sizeof(double) * (size_t)n * M, hipMemcpyDeviceToDevice, p->st));
    GemmArgs gr = ga;  // R = k - W K_N
    gr.A = p->W; gr.B = p->KN; gr.transB = 0; gr.C = p->Wr; gr.alpha = -1.0; gr.beta = 1.0;
    KRIG_TRY(gemm_f64(gr, p->st));
    ga.A = p->Wr; ga.C = p->Wt;
    KRIG_TRY(gemm_f64(ga, p->st));
    GemmArgs gw = gb;  // W += (R L_N^{-T}) L_N^{-1}
    gw.A = p->Wt; gw.C = p->W; gw.beta = 1.0;
    KRIG_TRY(gemm_f64(gw, p->st));
  }
  KRIG_TRY(transpose_w(p->W, n, M, p->gorder, p->Wt, p->st));
  return KRIG_OK;
}

// The gathers' site order: sites sorted by anchor cell (row-major over the cells; ties keep site
// order), so that a wave's sites read neighbouring image windows, and the anchors in that order,
// so that a gather reads its slot's anchor without first loading the site index.  From host
// anchors [n][2].
int set_gather_order(krig_plan p, const int32_t* h_anchor) {
  std::vector<int32_t> ord(p->n);
  for (int i = 0; i < p->n; ++i) ord[i] = i;
  const int64_t m2 = p->g.m2;
  std::stable_sort(ord.begin(), ord.end(), [&](int32_t a, int32_t b) {
    return (int64_t)h_anchor[2 * a] * m2 + h_anchor[2 * a + 1] < (int64_t)h_anchor[2 * b] * m2 + h_anchor[2 * b + 1];
  });
  std::vector<int32_t> ga(2 * (size_t)p->n);
  for (int s = 0; s < p->n; ++s) {
    ga[2 * s] = h_anchor[2 * ord[s]];
    ga[2 * s + 1] = h_anchor[2 * ord[s] + 1];
  }
  KRIG_TRY(hipMemcpyAsync(p->gorder, ord.data(), sizeof(int32_t) * p->n, hipMemcpyHostToDevice, p->st));
  KRIG_TRY(hipMemcpyAsync(p->ganchor, ga.data(), sizeof(int32_t) * ga.size(), hipMemcpyHostToDevice, p->st));
  KRIG_TRY(hipStreamSynchronize(p->st));  // ord and ga are freed on return
  return KRIG_OK;
}

int do_solve(krig_plan p, int B, const double* y, double* alpha) {
  StageTimer t(p, KRIG_STAGE_SOLVE);
  KRIG_TRY(tri_apply(p->Linv, p->ldL, p->n, 0, y, p->n, p->tmpv, p->ldv, B, p->st));
  KRIG_TRY(tri_apply(p->LinvT, p->ldL, p->n, 1, p->tmpv, p->ldv, alpha, p->n, B, p->st));
  return KRIG_OK;
}

// custom lag (dt) -> filtC; returns the filter to use
int filter_for(krig_plan p, const void* d_lag, const double** out) {
  if (!d_lag) {
    *out = p->filt;
    return KRIG_OK;
  }
  int r;
  KRIG_TRY(convert_to_f64(d_lag, p->lagC64, (int64_t)p->n1l * p->n2l, p->dtype == KRIG_F32, p->st));
  if ((r = make_filter(p, p->lagC64, p->filtC)) != KRIG_OK) return r;
  *out = p->filtC;
  return KRIG_OK;
}

// Argument blocks of the prediction's three passes (Steps 5-7): scatter + forward rows of
// alpha into spec1, columns (x filter) into S2, inverse rows of S2 into yhat.
RowsR2CArgs rows_fwd_args(krig_plan p, const double* alpha, void* spec1) {
  RowsR2CArgs r{};
  r.nrows = p->P1;
  r.H2 = p->H2;
  r.out = spec1;
  r.out_fs = (int64_t)p->H2 * p->ldP;
  r.out_ld = p->ldP;
  r.twF = p->tw2_64;  // scatter + forward rows in FP64
  r.row_ptr = p->node_ptr;
  r.ent_site = p->ent_site;
  r.ent_w = p->ent_w;
  r.alpha = alpha;
  r.alpha_fs = p->n;
  r.ncols = p->P2;
  r.NL = p->nl_rows64;
  return r;
}

// The scatter and the forward row transforms (Steps 5-6 and the first pass of Step 7): fused
// into one row kernel, or, for site sets with many CSR entries per padded node, the scatter's
// own kernel (one thread per node: the fused form gives a whole row's nodes to one line of
// threads) into the plan's image, then the row transforms of that image.  Both add each node's
// entries in segment order in FP64 and transform the same values: the same bits.
int rows_fwd(krig_plan p, int B, const double* alpha, void* spec1) {
  RowsR2CArgs r = rows_fwd_args(p, alpha, spec1);
  if (!split_now(p, B)) return hip_status(set2(p).r2c_csr(r, B, p->st));
  KRIG_TRY(scatter_image(p->g, p->node_ptr, p->ent_site, p->ent_w, alpha, p->n, B, p->fimg,
                         (int64_t)p->P1 * p->P2, 0, p->st));
  r.dense = p->fimg;
  r.dense_fs = (int64_t)p->P1 * p->P2;
  r.dense_ld = p->P2;
  r.coff = 0;
  return hip_status(set2(p).r2c_dense_f64(r, B, p->st));
}

ColsArgs cols_conv_args(krig_plan p, const void* spec1, const double* filt, int B) {
  ColsArgs c{};
  c.H2 = p->H2;
  c.in = spec1;
  c.in_fs = (int64_t)p->H2 * p->ldP;
  c.in_ld = p->ldP;
  c.in_off = 0;
  c.in_cnt = p->P1;
  c.filt = filt;
  c.filt_ld = p->F1;
  c.out = p->S2;
  c.out_fs = (int64_t)p->H2 * p->ldM;
  c.out_ld = p->ldM;
  c.rows = Window{p->g.L, p->g.m1, 0, 0};
  c.twF = p->tw1_64;  // FP64 column transforms for both dtypes
  c.twI = p->tw1_64;
  c.B = B;
  c.NL = conv_cols_nl(p);
  return c;
}

RowsC2RArgs rows_inv_args(krig_plan p, void* yhat) {
  RowsC2RArgs o{};
  o.nrows = p->g.m1;
  o.H2 = p->H2;
  o.in = p->S2;
  o.in_fs = (int64_t)p->H2 * p->ldM;
  o.in_ld = p->ldM;
  o.out = yhat;
  o.out_fs = (int64_t)p->g.m1 * p->g.m2;
  o.ldo = p->g.m2;
  o.cols = Window{p->g.L, p->g.m2, 0, 0};
  o.twF = p->tw2_64;  // FP64 arithmetic; the FP32 form reads FP32 spectra and writes FP32
  o.NL = p->nl_rows64;
  return o;
}

int do_convolve(krig_plan p, int B, const double* alpha, const double* filt, void* yhat, void* spec1,
                const void* add, int64_t add_fs, int add_ld) {
  {
    StageTimer t(p, KRIG_STAGE_ROWS_FWD);
    const int r = rows_fwd(p, B, alpha, spec1);
    if (r != KRIG_OK) return r;
  }
  {
    StageTimer t(p, KRIG_STAGE_COLS_CONV);
    KRIG_TRY(conv_cols_fn(p, is32(p))(cols_conv_args(p, spec1, filt, B), B, p->st));
  }
  RowsC2RArgs o = rows_inv_args(p, yhat);
  o.add = add;
  o.add_fs = add_fs;
  o.add_ld = add_ld;
  o.add_r0 = p->g.L;
  o.add_c0 = p->g.L;
  {
    StageTimer t(p, KRIG_STAGE_ROWS_INV);
    KRIG_TRY((is32(p) ? set2(p).c2r_f32 : set2(p).c2r64)(o, B, p->st));
  }
  return KRIG_OK;
}

int validate_sites(const krig_grid* g, int n, const double* s) {
  for (int i = 0; i < n; ++i) {
    const double t = (s[2 * i] - g->x0) / g->dx;
    const double u = (s[2 * i + 1] - g->y0) / g->dy;
    if (!(t >= 0.0 && t <= (double)(g->m1 - 1) && u >= 0.0 && u <= (double)(g->m2 - 1))) return KRIG_EDOMAIN;
  }
  return KRIG_OK;
}

int matern_kind(double nu) {
  if (nu == 0.5) return 0;
  if (nu == 1.5) return 1;
  if (nu == 2.5) return 2;
  if (nu == 1.0) return 3;
  return -1;
}

void destroy_all(krig_plan p) {
  if (!p) return;
  (void)hipStreamSynchronize(p->st);
  for (auto& v : p->ev_pending)
    for (auto& pr : v) {
      (void)hipEventDestroy(pr.first);
      (void)hipEventDestroy(pr.second);
    }
  for (hipEvent_t e : p->ev_pool) (void)hipEventDestroy(e);
  if (p->aux) {
    (void)hipStreamSynchronize(p->aux);
    (void)hipStreamDestroy(p->aux);
  }
  if (p->ev_fork) (void)hipEventDestroy(p->ev_fork);
  if (p->ev_join) (void)hipEventDestroy(p->ev_join);
  for (void* q : p->allocs) (void)hipFree(q);
  p->allocs.clear();
  delete p;
}

int nl_ce_rows_for(const FftEntry* e, size_t csz) {
  int nl = std::max(1, 256 / nt_of(e));
  while (nl > 1 && ce_rows_lds(e->geo, nl, csz) > 64 * 1024) --nl;
  return nl;
}

// Circulant embedding of the padded-grid covariance (discussion section): torus
// Fs >= 2 (P - 1) from the length ladder, eigenvalues Lambda = FFT2 of the
// minimal-image covariance (FP64).  Negative eigenvalues down to -1e-6 max are
// clamped; otherwise the torus grows (up to twice the first choice); else KRIG_ECE.
int ce_setup(krig_plan p) {
  int r;
  const int f1_0 = pick_fft(2 * (p->P1 - 1)), f2_0 = pick_fft(2 * (p->P2 - 1));
  if (f1_0 < 0 || f2_0 < 0) return KRIG_EUNSUPPORTED;
  int f1 = f1_0, f2 = f2_0;
  for (;;) {
    const FftEntry* e1 = find_fft(f1);
    const FftEntry* e2 = find_fft(f2);
    if (rows_lds(e2->geo, nl_rows_for(e2, 16), 16) > 64 * 1024 ||
        cols_lds(e1->geo, nl_cols_for(e1, 16), 16) > 64 * 1024)
      return KRIG_EUNSUPPORTED;
    const int h2 = f2 / 2 + 1;
    double* lam = nullptr;
    double* spec = nullptr;
    double *t1_64 = nullptr, *t2_64 = nullptr;
    float *t1_32 = nullptr, *t2_32 = nullptr;
    if ((r = dalloc(p, &lam, (size_t)h2 * f1)) != KRIG_OK) return r;
    if ((r = dalloc(p, &spec, 2 * (size_t)h2 * f1)) != KRIG_OK) return r;
    if ((r = make_twiddles(p, f1, &t1_64, &t1_32)) != KRIG_OK) return r;
    if ((r = make_twiddles(p, f2, &t2_64, &t2_32)) != KRIG_OK) return r;
    RowsR2CArgs a{};
    a.nrows = f1;
    a.H2 = h2;
    a.out = spec;
    a.out_fs = 0;
    a.out_ld = f1;
    a.twF = t2_64;
    a.F1 = f1;
    a.cov_sigma2 = p->mt.sigma2;
    a.cov_rho = p->mt.rho;
    a.cov_dx = p->g.dx;
    a.cov_dy = p->g.dy;
    a.cov_kind = p->mt.kind;
    a.NL = nl_rows_for(e2, 16);
    KRIG_TRY(e2->k.r2c_cov(a, 1, p->st));
    ColsArgs c{};
    c.H2 = h2;
    c.in = spec;
    c.in_ld = f1;
    c.in_off = 0;
    c.in_cnt = f1;
    c.out = lam;
    c.out_ld = f1;
    c.twF = t1_64;
    c.twI = t1_64;
    c.scale = 1.0;
    c.NL = nl_cols_for(e1, 16);
    KRIG_TRY(e1->k.fwd_real64(c, 1, p->st));
    const int nb = 256;
    double* bm = nullptr;
    if ((r = dalloc(p, &bm, 3 * (size_t)nb)) != KRIG_OK) return r;
    KRIG_TRY(minmax_blocks(lam, (int64_t)h2 * f1, bm, bm + nb, (int*)(bm + 2 * nb), nb, p->st));
    std::vector<double> hb(3 * (size_t)nb);
    KRIG_TRY(hipMemcpyAsync(hb.data(), bm, hb.size() * sizeof(double), hipMemcpyDeviceToHost, p->st));
    KRIG_TRY(hipStreamSynchronize(p->st));
    double lmin = 1e300, lmax = -1e300;
    int64_t nneg = 0;
    const int* hn = reinterpret_cast<const int*>(hb.data() + 2 * nb);
    for (int i = 0; i < nb; ++i) {
      lmin = std::min(lmin, hb[i]);
      lmax = std::max(lmax, hb[nb + i]);
      nneg += hn[i];
    }
    dfree(p, bm);
    dfree(p, spec);
    if (lmin >= -1e-6 * lmax) {
      KRIG_TRY(sqrt_clamp(lam, (int64_t)h2 * f1, 1.0 / ((double)f1 * f2), p->st));
      p->lamS = lam;
      p->Fs1 = f1;
      p->Fs2 = f2;
      p->Hs2 = h2;
      p->es1 = e1;
      p->es2 = e2;
      p->tws1_64 = t1_64;
      p->tws1_32 = t1_32;
      p->tws2_64 = t2_64;
      p->tws2_32 = t2_32;
      p->ce_clamped = (int)nneg;
      return KRIG_OK;
    }
    dfree(p, lam);
    const int n1 = pick_fft(f1 + 1), n2 = pick_fft(f2 + 1);
    if (n1 < 0 || n2 < 0 || n1 > 2 * f1_0 || n2 > 2 * f2_0) return KRIG_ECE;
    f1 = n1;
    f2 = n2;
  }
}

// default launch shapes for the current row / column transform forms
void default_rows_shapes(krig_plan p) {
  p->nl_rows64 = nl_rows_for(p->e2, 16);
}
void default_cols_shapes(krig_plan p) {
  p->nl_cols64 = nl_cols_for(p->e1, 16);
  p->dlag_G = p->nl_cols64;
}

// switch the row (rows = true) or column transforms to compiled form idx of their
// length; the launch shapes of that side return to the form's defaults
int set_variant(krig_plan p, bool rows, int idx) {
  const FftEntry* v[16];
  const int F = rows ? p->F2 : p->F1;
  const int k = fft_variants(F, v, 16);
  if (idx < 0 || idx >= k || idx >= 16) return KRIG_EINVAL;
  if (rows) {
    if (rows_lds(v[idx]->geo, nl_rows_for(v[idx], 16), 16) > 64 * 1024) return KRIG_EINVAL;
    p->e2 = v[idx];
    p->var_rows = idx;
    default_rows_shapes(p);
  } else {
    if (cols_lds(v[idx]->geo, nl_cols_for(v[idx], 16), 16) > 64 * 1024) return KRIG_EINVAL;
    p->e1 = v[idx];
    p->var_cols = idx;
    default_cols_shapes(p);
  }
  return KRIG_OK;
}

// Process-wide table of autotuned launch shapes, keyed by what the kernels depend on:
// grid, neighbour order, transform lengths and dtype.
struct TuneKey {
  int m1, m2, L, F1, F2, dtype;
  bool operator<(const TuneKey& o) const {
    return std::tie(m1, m2, L, F1, F2, dtype) < std::tie(o.m1, o.m2, o.L, o.F1, o.F2, o.dtype);
  }
};
struct TuneRec {
  int var_rows, var_cols, nl_rows64, nl_cols64, dlag_G, cols_pair;
  int n, scatter_split;  // the scatter form depends on the site density: kept for plans of the same n
};
std::mutex& tune_mutex() {
  static std::mutex m;
  return m;
}
std::map<TuneKey, TuneRec>& tune_table() {
  static std::map<TuneKey, TuneRec> t;
  return t;
}
TuneKey tune_key(krig_plan p) { return TuneKey{p->g.m1, p->g.m2, p->g.L, p->F1, p->F2, p->dtype}; }

void tuned_lookup(krig_plan p) {
  TuneRec r;
  {
    std::lock_guard<std::mutex> lk(tune_mutex());
    auto it = tune_table().find(tune_key(p));
    if (it == tune_table().end()) return;
    r = it->second;
  }
  if (set_variant(p, true, r.var_rows) != KRIG_OK || set_variant(p, false, r.var_cols) != KRIG_OK) return;
  p->nl_rows64 = r.nl_rows64;
  p->nl_cols64 = r.nl_cols64;
  p->dlag_G = r.dlag_G;
  p->cols_pair = p->e1h ? r.cols_pair : 0;
  if (r.n == p->n) p->scatter_split = r.scatter_split;
}

}  // namespace

// =====================================================================================
struct krig_batch_s {
  std::vector<krig_plan> plans;
  hipGraph_t graph = nullptr;
  hipGraphExec_t exec = nullptr;
  hipStream_t own = nullptr;   // capture stream created by the batch (stream NULL)
  hipStream_t cap = nullptr;   // the capture stream
  void* qbuf = nullptr;        // persistent form: argument blocks and tile tables
};

namespace {

// The persistent form of an uneven batch.  Every pass of every problem goes into one launch
// per pass and kernel form: the two triangular products grouped by input form (vec), then
// the row, column and inverse-row transforms grouped by transform form (and, for the inverse
// rows, by dtype).  Each launch is a grid of about one resident round of blocks that walks
// the pass's (problem, tile) list.
struct QueueLaunch {
  int kind;                  // 0 triangular product, 2 rows forward, 3 columns, 4 inverse rows,
                             // 5 scatters of the problems whose scatter runs apart (direct)
  int upper = 0, vec = 0, form = 0, f32 = 0, pair = 0, dense = 0, NL = 1;
  std::vector<TriProb> direct;  // block-tile products: one launch per problem, from the host
  std::vector<std::pair<krig_plan, int>> scat;  // kind 5: (plan, B), each its own scatter launch
  const FftEntry* e = nullptr;
  size_t args_off = 0, first_off = 0, nbx_off = 0;
  int count = 0, total = 0;
};

struct QueuePlan {
  std::vector<unsigned char> host;  // the device buffer's image
  std::vector<QueueLaunch> launches;

  template <typename T>
  size_t put(const std::vector<T>& v) {
    const size_t off = (host.size() + 15) / 16 * 16;
    host.resize(off + v.size() * sizeof(T));
    if (!v.empty()) memcpy(host.data() + off, v.data(), v.size() * sizeof(T));
    return off;
  }
  template <typename T>
  void add(int kind, const std::vector<T>& args, const std::vector<int>& tiles, const std::vector<int>& nbx,
           QueueLaunch proto) {
    std::vector<int> first(tiles.size() + 1, 0);
    for (size_t i = 0; i < tiles.size(); ++i) first[i + 1] = first[i] + tiles[i];
    proto.kind = kind;
    proto.args_off = put(args);
    proto.first_off = put(first);
    proto.nbx_off = nbx.empty() ? 0 : put(nbx);
    proto.count = (int)args.size();
    proto.total = first.back();
    launches.push_back(proto);
  }
};

// Adds the launches of the problems `ids` to qp: first the solve's (products grouped by input
// vector width and tile form), then the transforms'; returns the index of the first transform
// launch.
size_t queue_problems(QueuePlan& qp, const std::vector<int>& ids, const krig_plan* plans, const int32_t* h_B,
                      const double* const* h_y, void* const* h_yhat) {
  for (int upper = 0; upper < 2; ++upper) {  // L^{-1} y -> tmpv, then L^{-T} tmpv -> alpha
    std::map<std::pair<int, int>, std::vector<TriProb>> groups;  // (vec, tile form) -> problems
    for (int i : ids) {
      const krig_plan p = plans[i];
      const int B = h_B ? h_B[i] : 1;
      const TriProb tp = upper ? tri_prob(p->LinvT, p->ldL, p->n, p->tmpv, p->ldv, p->alpha, p->n, B)
                               : tri_prob(p->Linv, p->ldL, p->n, h_y[i], p->n, p->tmpv, p->ldv, B);
      groups[{tp.vec, tp.form}].push_back(tp);
    }
    for (auto& g : groups) {
      std::vector<int> tiles;
      for (const TriProb& tp : g.second) tiles.push_back(tp.nt * tp.nfz);
      QueueLaunch ql;
      ql.upper = upper;
      ql.vec = g.first.first;
      ql.form = g.first.second;
      if (ql.form == TRI_FORM_BLOCK) ql.direct = g.second;
      qp.add(0, g.second, tiles, {}, ql);
    }
  }
  const size_t mid = qp.launches.size();
  // the scatters that run apart (dense site sets), before the row passes that read their images
  {
    QueueLaunch ql;
    ql.kind = 5;
    for (int i : ids)
      if (split_now(plans[i], h_B ? h_B[i] : 1)) ql.scat.push_back({plans[i], h_B ? h_B[i] : 1});
    if (!ql.scat.empty()) qp.launches.push_back(ql);
  }
  // transforms: scatter + forward rows (or rows of the scattered image), columns (x filter),
  // inverse rows
  std::map<std::pair<const FftEntry*, int>, std::vector<RowsR2CArgs>> rf;
  std::map<std::pair<const FftEntry*, int>, std::vector<int>> rf_t, rf_n;
  std::map<std::pair<const FftEntry*, int>, std::vector<ColsArgs>> cf;
  std::map<std::pair<const FftEntry*, int>, std::vector<int>> cf_t, cf_n;
  std::map<std::pair<const FftEntry*, int>, std::vector<RowsC2RArgs>> ri;
  std::map<std::pair<const FftEntry*, int>, std::vector<int>> ri_t, ri_n;
  for (int i : ids) {
    const krig_plan p = plans[i];
    const int B = h_B ? h_B[i] : 1;
    const int nlr = nl_rows_for(p->e2, 16), nlc = nl_cols_for(p->e1, 16);
    RowsR2CArgs r = rows_fwd_args(p, p->alpha, p->S1);
    r.NL = nlr;
    const bool split = split_now(p, B);
    if (split) {  // the rows of the image the kind-5 launch scatters (as rows_fwd)
      r.dense = p->fimg;
      r.dense_fs = (int64_t)p->P1 * p->P2;
      r.dense_ld = p->P2;
      r.coff = 0;
    }
    const int nbr = ((p->P1 + 1) / 2 + nlr - 1) / nlr;
    const auto rkey = std::make_pair(p->e2, (int)split);
    rf[rkey].push_back(r);
    rf_t[rkey].push_back(nbr * B);
    rf_n[rkey].push_back(nbr);
    ColsArgs c = cols_conv_args(p, p->S1, p->filt, B);
    const int nlq = p->cols_pair ? p->cols_pair : nlc;
    c.NL = nlq;
    const int nbc = (p->H2 + nlq - 1) / nlq;
    // the paired form is keyed by its half-length entry and flagged in the second member
    const auto ckey = std::make_pair(p->cols_pair ? p->e1h : p->e1, (int)is32(p) + (p->cols_pair ? 2 : 0));
    cf[ckey].push_back(c);
    cf_t[ckey].push_back(nbc * B);
    cf_n[ckey].push_back(nbc);
    RowsC2RArgs o = rows_inv_args(p, h_yhat[i]);
    o.NL = nlr;
    const int nbi = ((p->g.m1 + 1) / 2 + nlr - 1) / nlr;
    const auto key = std::make_pair(p->e2, (int)is32(p));
    ri[key].push_back(o);
    ri_t[key].push_back(nbi * B);
    ri_n[key].push_back(nbi);
  }
  for (auto& g : rf) {
    QueueLaunch ql;
    ql.e = g.first.first;
    ql.dense = g.first.second;
    ql.NL = g.second[0].NL;
    qp.add(2, g.second, rf_t[g.first], rf_n[g.first], ql);
  }
  for (auto& g : cf) {
    QueueLaunch ql;
    ql.e = g.first.first;
    ql.f32 = g.first.second & 1;
    ql.pair = g.first.second >> 1;
    ql.NL = g.second[0].NL;
    qp.add(3, g.second, cf_t[g.first], cf_n[g.first], ql);
  }
  for (auto& g : ri) {
    QueueLaunch ql;
    ql.e = g.first.first;
    ql.f32 = g.first.second;
    ql.NL = g.second[0].NL;
    qp.add(4, g.second, ri_t[g.first], ri_n[g.first], ql);
  }
  return mid;
}

// nblocks for the transform kernels: 0 one resident round of blocks, -d 1/d of one
int queue_launch(const QueueLaunch& ql, unsigned char* base, int nblocks, hipStream_t st) {
  if (ql.kind == 5) {
    for (const auto& sj : ql.scat) {
      const krig_plan p = sj.first;
      KRIG_TRY(scatter_image(p->g, p->node_ptr, p->ent_site, p->ent_w, p->alpha, p->n, sj.second, p->fimg,
                             (int64_t)p->P1 * p->P2, 0, st));
    }
    return KRIG_OK;
  }
  const int* first = reinterpret_cast<const int*>(base + ql.first_off);
  if (ql.kind == 0) {
    if (ql.form == TRI_FORM_BLOCK) {  // 256-thread workgroups: each problem's own launch
      for (const TriProb& tp : ql.direct) KRIG_TRY(tri_apply_prob(tp, ql.upper, st));
      return KRIG_OK;
    }
    TriQueue tq{reinterpret_cast<const TriProb*>(base + ql.args_off), first, ql.count, ql.total};
    return hip_status(tri_apply_queue(tq, ql.upper, ql.vec, ql.form, st));
  }
  QueueArgs qa{base + ql.args_off, first, reinterpret_cast<const int*>(base + ql.nbx_off), ql.count, ql.total};
  const FftSet& k = ql.e->k;
  const launch_queue_t fn = ql.kind == 2   ? (ql.dense ? k.q_r2c_dense : k.q_r2c_csr)
                            : ql.kind == 3 ? (ql.pair ? (ql.f32 ? k.q_pair_conv_pred_f : k.q_pair_conv64)
                                                      : (ql.f32 ? k.q_conv_pred_f : k.q_conv64))
                                           : (ql.f32 ? k.q_c2r_f32 : k.q_c2r64);
  return hip_status(fn(qa, ql.NL, nblocks, st));
}

// All problems' passes in order on one stream: the product of L^{-1}, that of
// L^{-T}, then the transforms.  (Splitting the problems
// into two halves staggered on two streams, one half's transforms beside the other's solve,
// measured slower: concurrent persistent grids contend for the same compute units.)
int batch_queue_record(krig_batch b, const krig_plan* plans, int count, const int32_t* h_B, const double* const* h_y,
                       void* const* h_yhat, hipStream_t st) {
  std::vector<int> ids(count);
  for (int i = 0; i < count; ++i) ids[i] = i;
  QueuePlan qp;
  queue_problems(qp, ids, plans, h_B, h_y, h_yhat);
  if (hipMalloc(&b->qbuf, qp.host.size()) != hipSuccess) return KRIG_ENOMEM;
  KRIG_TRY(hipMemcpy(b->qbuf, qp.host.data(), qp.host.size(), hipMemcpyHostToDevice));
  unsigned char* base = static_cast<unsigned char*>(b->qbuf);
  KRIG_TRY(hipStreamBeginCapture(st, hipStreamCaptureModeThreadLocal));
  int r = KRIG_OK;
  for (size_t i = 0; i < qp.launches.size() && r == KRIG_OK; ++i) r = queue_launch(qp.launches[i], base, 0, st);
  hipGraph_t g = nullptr;
  const hipError_t ee = hipStreamEndCapture(st, &g);
  if (r == KRIG_OK && ee != hipSuccess) r = KRIG_EHIP;
  if (r != KRIG_OK) {
    if (g) (void)hipGraphDestroy(g);
    return r;
  }
  b->graph = g;
  if (hipGraphInstantiate(&b->exec, b->graph, nullptr, nullptr, 0) != hipSuccess) return KRIG_EHIP;
  return KRIG_OK;
}

}  // namespace

extern "C" {

const char* krig_strerror(int s) {
  switch (s) {
    case KRIG_OK: return "ok";
    case KRIG_EINVAL: return "invalid argument";
    case KRIG_EDOMAIN: return "site outside the prediction grid";
    case KRIG_ENOTSPD: return "matrix not positive definite";
    case KRIG_ECE: return "circulant embedding not non-negative definite";
    case KRIG_ENOMEM: return "device allocation failed";
    case KRIG_EHIP: return "HIP runtime error";
    case KRIG_EUNSUPPORTED: return "unsupported parameter";
    default: return "unknown status";
  }
}

int krig_plan_create(krig_plan* out, const krig_grid* g, const krig_matern* k, int32_t n, const double* h_sites,
                     int32_t dtype, void* stream) {
  if (!out) return KRIG_EINVAL;
  *out = nullptr;
  if (!g || !k || !h_sites || n < 1) return KRIG_EINVAL;
  if (g->m1 < 2 || g->m2 < 2 || g->L < 1 || g->L > 8 || !(g->dx > 0) || !(g->dy > 0)) return KRIG_EINVAL;
  if (dtype != KRIG_F32 && dtype != KRIG_F64) return KRIG_EINVAL;
  if (!(k->sigma2 > 0) || !(k->range > 0) || !(k->tau2 >= 0)) return KRIG_EINVAL;
  const int kind = matern_kind(k->nu);
  if (kind < 0) return KRIG_EUNSUPPORTED;
  if ((int64_t)(g->m1 + 2 * g->L) * (g->m2 + 2 * g->L) > (1LL << 30)) return KRIG_EINVAL;
  int r = validate_sites(g, n, h_sites);
  if (r != KRIG_OK) return r;
  std::call_once(g_once, register_all_fft);

  krig_plan p = new (std::nothrow) krig_plan_s();
  if (!p) return KRIG_ENOMEM;
  if (hipGetDevice(&p->device) != hipSuccess) {
    delete p;
    return KRIG_EHIP;
  }
  p->st = (hipStream_t)stream;
  p->dtype = dtype;
  p->tsz = dtype == KRIG_F32 ? 4 : 8;
  p->n = n;
  p->g.m1 = g->m1;
  p->g.m2 = g->m2;
  p->g.L = g->L;
  p->g.x0 = g->x0;
  p->g.y0 = g->y0;
  p->g.dx = g->dx;
  p->g.dy = g->dy;
  p->g.P1 = g->m1 + 2 * g->L;
  p->g.P2 = g->m2 + 2 * g->L;
  p->g.M = 4 * g->L * g->L;
  p->mt.sigma2 = k->sigma2;
  p->mt.rho = k->range;
  p->mt.tau2 = k->tau2;
  p->mt.kind = kind;
  p->M = p->g.M;
  p->P1 = p->g.P1;
  p->P2 = p->g.P2;
  p->n1l = g->m1 + g->L;
  p->n2l = g->m2 + g->L;
  p->F1 = pick_fft(g->m1 + p->P1 - 1);
  p->F2 = pick_fft(g->m2 + p->P2 - 1);
  if (p->F1 < 0 || p->F2 < 0) {
    delete p;
    return KRIG_EUNSUPPORTED;
  }
  p->e1 = find_fft(p->F1);
  p->e2 = find_fft(p->F2);
  if (p->F1 % 2 == 0) {  // the paired column form: half the length on one wave per column
    const FftEntry* h = find_fft(p->F1 / 2);
    if (h && h->F == p->F1 / 2 && h->k.pair_conv64) p->e1h = h;
  }
  p->H2 = p->F2 / 2 + 1;
  p->ldP = pitch16(p->P1);
  // the scatter's form: its own kernel, one thread per padded node, where nodes hold many CSR
  // entries (n M entries over P1 P2 nodes); fused into the row kernel for sparser site sets
  p->scatter_split = (int64_t)n * p->M >= (int64_t)SCATTER_SPLIT_MIN_DENSITY * p->P1 * p->P2;
  p->ldM = pitch16(g->m1);
  p->ldX = pitch16(2 * (g->m1 + g->L) - 1);
  const bool f32 = dtype == KRIG_F32;
  // launch shapes (lines per block) within 256 threads and 64 KB of LDS
  default_rows_shapes(p);
  default_cols_shapes(p);
  tuned_lookup(p);
  if (rows_lds(p->e2->geo, p->nl_rows64, 16) > 64 * 1024 || cols_lds(p->e1->geo, p->nl_cols64, 16) > 64 * 1024) {
    delete p;
    return KRIG_EUNSUPPORTED;
  }

#define CK(x)                 \
  do {                        \
    if ((r = (x)) != KRIG_OK) { \
      destroy_all(p);         \
      return r;               \
    }                         \
  } while (0)
#define CKH(x) CK(hip_status(x))

  const int n1l = p->n1l, n2l = p->n2l, M = p->M, P1 = p->P1, P2 = p->P2;
  CK(make_twiddles(p, p->F1, &p->tw1_64, &p->tw1_32));
  CK(make_twiddles(p, p->F2, &p->tw2_64, &p->tw2_32));
  CK(dalloc(p, &p->sites, 2 * (size_t)n));
  CKH(hipMemcpyAsync(p->sites, h_sites, 2 * sizeof(double) * n, hipMemcpyHostToDevice, p->st));
  CK(dalloc(p, &p->d_status, 4));
  CKH(hipMemsetAsync(p->d_status, 0, 4 * sizeof(int), p->st));

  // Step 2: lag image and its spectrum (FP64)
  CK(dalloc(p, &p->lag64, (size_t)n1l * n2l));
  CK(dalloc_bytes(p, &p->lagT, p->tsz * (size_t)n1l * n2l));
  CK(dalloc(p, &p->lagC64, (size_t)n1l * n2l));
  CK(dalloc(p, &p->phiS64, 2 * (size_t)p->H2 * p->F1));
  CK(dalloc(p, &p->filt, (size_t)p->H2 * p->F1));
  CK(dalloc(p, &p->filtC, (size_t)p->H2 * p->F1));
  CKH(lag_image(p->g, p->mt, p->lag64, p->st));
  CKH(convert_f64(p->lag64, p->lagT, (int64_t)n1l * n2l, f32, p->st));
  CK(make_filter(p, p->lag64, p->filt));

  // Steps 1, 3, 4: K_N, k_i, A_i = K_N^{-1} k_i  (two FP64 MFMA products with L_N^{-1})
  CK(dalloc(p, &p->KN, (size_t)M * M));
  CK(dalloc(p, &p->LinvN, (size_t)M * M));
  CK(dalloc(p, &p->anchor, 2 * (size_t)n));
  CK(dalloc(p, &p->kvec, (size_t)n * M));
  CK(dalloc(p, &p->W, (size_t)n * M));
  CK(dalloc(p, &p->Wt, (size_t)n * M));
  CK(dalloc(p, &p->gorder, (size_t)n));
  CK(dalloc(p, &p->ganchor, 2 * (size_t)n));
  CK(dalloc(p, &p->Wr, (size_t)n * M));
  if (M <= 64)
    CKH(kn_factor(p->g, p->mt, p->KN, p->LinvN, p->d_status, p->st));
  else
    CK(kn_factor_large(p));
  CKH(site_kvec(p->g, p->mt, p->sites, n, p->anchor, p->kvec, p->st));
  {
    std::vector<int32_t> ha(2 * (size_t)n);
    CKH(hipMemcpyAsync(ha.data(), p->anchor, ha.size() * sizeof(int32_t), hipMemcpyDeviceToHost, p->st));
    CKH(hipStreamSynchronize(p->st));
    CK(set_gather_order(p, ha.data()));
  }
  CK(weights_from_kvec(p, p->kvec));

  // Step 5 structure
  CK(dalloc(p, &p->cw.cell_cnt, (size_t)g->m1 * g->m2));
  CK(dalloc(p, &p->cw.cell_ptr, (size_t)g->m1 * g->m2 + 1));
  CK(dalloc(p, &p->cw.cell_cur, (size_t)g->m1 * g->m2));
  CK(dalloc(p, &p->cw.cell_sites, (size_t)n));
  CK(dalloc(p, &p->cw.node_cnt, (size_t)P1 * P2));
  CK(dalloc(p, &p->cw.scan_tmp, (size_t)P1 * P2 / 1024 + 16 + (size_t)g->m1 * g->m2 / 1024));
  CK(dalloc(p, &p->node_ptr, (size_t)P1 * P2 + 1));
  CK(dalloc(p, &p->ent_site, (size_t)n * M));
  CK(dalloc(p, &p->ent_w, (size_t)n * M));
  CKH(build_csr(p->g, p->anchor, p->W, n, p->cw, p->node_ptr, p->ent_site, p->ent_w, p->st));

  // kriging system: M = K + tau^2 I, Cholesky, inverse factor
  p->ldL = (n + 16) / 16 * 16;
  CK(dalloc(p, &p->Lfac, (size_t)n * p->ldL));
  CK(dalloc(p, &p->Linv, (size_t)n * p->ldL));
  CK(dalloc(p, &p->LinvT, (size_t)n * p->ldL));
  CK(dalloc(p, &p->Dinv, (size_t)((n + 63) / 64) * 4096));
  CK(dalloc(p, &p->work, (size_t)64 * std::max(n, 64)));
  CKH(assemble_kt(p->sites, n, p->mt, p->Lfac, p->ldL, p->st));
  CKH(cholesky_and_inverse(p->Lfac, p->ldL, n, p->Linv, p->Dinv, p->work, p->d_status + 1, p->st));
  CKH(fill_f64(p->LinvT, (int64_t)n * p->ldL, 0.0, p->st));
  CKH(transpose_f64(p->Linv, p->ldL, p->LinvT, p->ldL, n, p->st));

  // dlag buffers
  CK(dalloc_bytes(p, &p->XC, 16 * (size_t)p->H2 * p->ldX));

  int hst[4] = {0, 0, 0, 0};
  CKH(hipMemcpyAsync(hst, p->d_status, sizeof(hst), hipMemcpyDeviceToHost, p->st));
  CKH(hipStreamSynchronize(p->st));
  p->kn_status = hst[0];
  p->pivot = hst[1];
  dfree(p, p->kvec);
  p->kvec = nullptr;
  if (hst[0] < 0 || hst[1] != 0) {
    destroy_all(p);
    return KRIG_ENOTSPD;
  }
  // the factor itself and its panel workspaces are not needed after set-up
  dfree(p, p->Lfac);
  dfree(p, p->Dinv);
  dfree(p, p->work);
  p->Lfac = p->Dinv = p->work = nullptr;
  *out = p;
  return KRIG_OK;
#undef CK
#undef CKH
}

int krig_plan_destroy(krig_plan p) {
  if (!p || p->batch_refs > 0) return KRIG_EINVAL;
  destroy_all(p);
  return KRIG_OK;
}

namespace {
int solve_noalloc_max_B(int n);  // with krig_solve_noalloc below
}  // namespace

int krig_plan_info(krig_plan p, int32_t what, int64_t* v) {
  if (!p || !v) return KRIG_EINVAL;
  switch (what) {
    case KRIG_INFO_N: *v = p->n; break;
    case KRIG_INFO_M: *v = p->M; break;
    case KRIG_INFO_P1: *v = p->P1; break;
    case KRIG_INFO_P2: *v = p->P2; break;
    case KRIG_INFO_F1: *v = p->F1; break;
    case KRIG_INFO_F2: *v = p->F2; break;
    case KRIG_INFO_H2: *v = p->H2; break;
    case KRIG_INFO_LDH: *v = p->ldP; break;
    case KRIG_INFO_SAVED_PER_FIELD: *v = (int64_t)p->H2 * p->ldP; break;  // complex FP64
    case KRIG_INFO_KN_STATUS: *v = p->kn_status; break;
    case KRIG_INFO_PIVOT: *v = p->pivot; break;
    case KRIG_INFO_DTYPE: *v = p->dtype; break;
    case KRIG_INFO_CE_CLAMPED: *v = p->ce_clamped; break;
    case KRIG_INFO_DLAG_GROUP: *v = p->dlag_G; break;
    case KRIG_INFO_NL_ROWS64: *v = p->nl_rows64; break;
    case KRIG_INFO_NL_COLS64: *v = p->nl_cols64; break;
    case KRIG_INFO_FFT_VARIANTS_ROWS: *v = fft_variants(p->F2, nullptr, 0); break;
    case KRIG_INFO_FFT_VARIANTS_COLS: *v = fft_variants(p->F1, nullptr, 0); break;
    case KRIG_INFO_FFT_VARIANT_ROWS: *v = p->var_rows + 1; break;
    case KRIG_INFO_FFT_VARIANT_COLS: *v = p->var_cols + 1; break;
    case KRIG_INFO_COLS_PAIR: *v = p->cols_pair + 1; break;
    case KRIG_INFO_SCATTER: *v = p->scatter_split + 1; break;
    case KRIG_INFO_FFT_R1: *v = p->e2->geo.R1; break;
    case KRIG_INFO_FFT_R2: *v = p->e2->geo.R2; break;
    case KRIG_INFO_FFT_R3: *v = p->e2->geo.R3; break;
    case KRIG_INFO_CE_F1: *v = p->Fs1; break;
    case KRIG_INFO_CE_F2: *v = p->Fs2; break;
    case KRIG_INFO_SOLVE_NOALLOC_MAX_B: *v = solve_noalloc_max_B(p->n); break;
    case KRIG_INFO_FILTER_SETUP: *v = p->filt_setup; break;
    default: return KRIG_EINVAL;
  }
  return KRIG_OK;
}

int krig_set_stream(krig_plan p, void* stream) {
  if (!p) return KRIG_EINVAL;
  p->st = (hipStream_t)stream;
  return KRIG_OK;
}

int krig_weights(krig_plan p, int32_t* d_anchor, double* d_W) {
  if (!p) return KRIG_EINVAL;
  if (d_anchor)
    KRIG_TRY(hipMemcpyAsync(d_anchor, p->anchor, 2 * sizeof(int32_t) * p->n, hipMemcpyDeviceToDevice, p->st));
  if (d_W) KRIG_TRY(hipMemcpyAsync(d_W, p->W, sizeof(double) * p->n * p->M, hipMemcpyDeviceToDevice, p->st));
  return KRIG_OK;
}

int krig_set_weights(krig_plan p, const int32_t* d_anchor, const double* d_W) {
  if (!p || !d_anchor || !d_W) return KRIG_EINVAL;
  // anchors must keep every neighbour inside the padded grid
  std::vector<int32_t> h(2 * (size_t)p->n);
  KRIG_TRY(hipMemcpyAsync(h.data(), d_anchor, h.size() * sizeof(int32_t), hipMemcpyDeviceToHost, p->st));
  KRIG_TRY(hipStreamSynchronize(p->st));
  for (int i = 0; i < p->n; ++i)
    if (h[2 * i] < 0 || h[2 * i] >= p->g.m1 || h[2 * i + 1] < 0 || h[2 * i + 1] >= p->g.m2) return KRIG_EDOMAIN;
  KRIG_TRY(hipMemcpyAsync(p->anchor, d_anchor, h.size() * sizeof(int32_t), hipMemcpyDeviceToDevice, p->st));
  KRIG_TRY(hipMemcpyAsync(p->W, d_W, sizeof(double) * p->n * p->M, hipMemcpyDeviceToDevice, p->st));
  const int r = set_gather_order(p, h.data());
  if (r != KRIG_OK) return r;
  KRIG_TRY(transpose_w(p->W, p->n, p->M, p->gorder, p->Wt, p->st));
  KRIG_TRY(build_csr(p->g, p->anchor, p->W, p->n, p->cw, p->node_ptr, p->ent_site, p->ent_w, p->st));
  return KRIG_OK;
}

int krig_set_kvec(krig_plan p, const double* d_kvec) {
  if (!p || !d_kvec) return KRIG_EINVAL;
  // Step 4 with the caller's k_i: W = K_N^{-1} k as at plan creation (the inverse-factor
  // products and their refinement); Wt is rebuilt from W
  int r = weights_from_kvec(p, d_kvec);
  if (r != KRIG_OK) return r;
  // the anchors are unchanged, so the scatter structure is too: only its weights are rewritten
  KRIG_TRY(refill_csr_weights(p->g, p->anchor, p->W, p->node_ptr, p->ent_site, p->ent_w, p->st));
  return KRIG_OK;
}

int krig_filter(krig_plan p, int32_t setup, double* d_spec) {
  if (!p || (setup != KRIG_FILTER_REFLECTED && setup != KRIG_FILTER_CENTERED)) return KRIG_EINVAL;
  if (p->batch_refs > 0) return KRIG_EINVAL;  // a recorded batch replays with the current filter
  if (setup != p->filt_setup) {
    const int r = setup == KRIG_FILTER_CENTERED ? make_filter_centered(p, p->filt) : make_filter(p, p->lag64, p->filt);
    if (r != KRIG_OK) return r;
    p->filt_setup = setup;
  }
  if (d_spec)
    KRIG_TRY(hipMemcpyAsync(d_spec, p->filt, sizeof(double) * (size_t)p->H2 * p->F1, hipMemcpyDeviceToDevice,
                            p->st));
  return KRIG_OK;
}

int krig_lag(krig_plan p, void* d_lag) {
  if (!p || !d_lag) return KRIG_EINVAL;
  KRIG_TRY(hipMemcpyAsync(d_lag, p->lagT, p->tsz * p->n1l * p->n2l, hipMemcpyDeviceToDevice, p->st));
  return KRIG_OK;
}

int krig_solve(krig_plan p, int32_t B, const double* d_y, double* d_alpha) {
  if (!p || B < 1 || B > 65535 || !d_y || !d_alpha) return KRIG_EINVAL;
  int r = ensure_ws(p, B);
  if (r != KRIG_OK) return r;
  return do_solve(p, B, d_y, d_alpha);
}

// ------------------------------------------------------------------ allocation-free solve
// Scratch of krig_solve_noalloc: the intermediate vector between the two triangular
// products (B rows of n rounded up to 4).  A
// file-scope device array, so each GPU holds one copy from module load until the process
// ends; host code reaches it only through the address hipGetSymbolAddress returns for
// the device that is current (the array's name is a host-side stand-in, not a device
// address).
static __device__ __align__(256) double scratch[KRIG_SOLVE_NOALLOC_SCRATCH_BYTES / sizeof(double)];

namespace {
constexpr int kMaxDevices = 64;
std::mutex g_scratch_mu;
double* g_scratch_ptr[kMaxDevices] = {};

// this GPU's copy of the scratch array, looked up once per device (with it current)
int scratch_for_device(int dev, double** out) {
  if (dev < 0 || dev >= kMaxDevices) return KRIG_EINVAL;
  std::lock_guard<std::mutex> lk(g_scratch_mu);
  if (!g_scratch_ptr[dev]) {
    void* ptr = nullptr;
    if (hipGetSymbolAddress(&ptr, HIP_SYMBOL(scratch)) != hipSuccess || !ptr) return KRIG_EHIP;
    g_scratch_ptr[dev] = static_cast<double*>(ptr);
  }
  *out = g_scratch_ptr[dev];
  return KRIG_OK;
}

// doubles of scratch one solve of B fields needs: the intermediate vector
size_t solve_scratch_doubles(int n, int B) { return (size_t)B * ((n + 3) / 4 * 4); }
int solve_noalloc_max_B(int n) {
  const size_t cap = KRIG_SOLVE_NOALLOC_SCRATCH_BYTES / sizeof(double);
  int lo = 0, hi = 65535;  // largest B with solve_scratch_doubles(n, B) <= cap
  while (lo < hi) {
    const int mid = (lo + hi + 1) / 2;
    if (solve_scratch_doubles(n, mid) <= cap) lo = mid; else hi = mid - 1;
  }
  return lo;
}
}  // namespace

int krig_solve_noalloc(krig_plan p, int32_t B, const double* d_y, double* d_alpha) {
  if (!p || B < 1 || B > 65535 || !d_y || !d_alpha) return KRIG_EINVAL;
  if (solve_scratch_doubles(p->n, B) * sizeof(double) > KRIG_SOLVE_NOALLOC_SCRATCH_BYTES) return KRIG_EINVAL;
  int cur = -1;
  if (hipGetDevice(&cur) != hipSuccess) return KRIG_EHIP;
  if (cur != p->device) return KRIG_EINVAL;
  double* sp = nullptr;
  int r = scratch_for_device(cur, &sp);
  if (r != KRIG_OK) return r;
  // the products of krig_solve, with the scratch in place of the plan's intermediate vector:
  // every value they read from it is written earlier in the same call (its rows up to n; the
  // row padding is loaded but masked), so nothing is cleared
  const int64_t ldv = (p->n + 3) / 4 * 4;
  double* tmpv = sp;
  KRIG_TRY(tri_apply(p->Linv, p->ldL, p->n, 0, d_y, p->n, tmpv, ldv, B, p->st));
  KRIG_TRY(tri_apply(p->LinvT, p->ldL, p->n, 1, tmpv, ldv, d_alpha, p->n, B, p->st));
  return KRIG_OK;
}

int krig_scatter(krig_plan p, int32_t B, const double* d_alpha, void* d_img) {
  if (!p || B < 1 || B > 65535 || !d_alpha || !d_img) return KRIG_EINVAL;
  KRIG_TRY(scatter_image(p->g, p->node_ptr, p->ent_site, p->ent_w, d_alpha, p->n, B, d_img,
                         (int64_t)p->P1 * p->P2, p->dtype == KRIG_F32, p->st));
  return KRIG_OK;
}

int krig_convolve(krig_plan p, int32_t B, const double* d_alpha, const void* d_lag, void* d_yhat, void* d_saved) {
  if (!p || B < 1 || B > 65535 || !d_alpha || !d_yhat) return KRIG_EINVAL;
  int r = ensure_ws(p, B);
  if (r != KRIG_OK) return r;
  const double* filt = nullptr;
  if ((r = filter_for(p, d_lag, &filt)) != KRIG_OK) return r;
  return do_convolve(p, B, d_alpha, filt, d_yhat, d_saved ? d_saved : p->S1, nullptr, 0, 0);
}

int krig_predict(krig_plan p, int32_t B, const double* d_y, const void* d_lag, void* d_yhat, double* d_alpha_out,
                 void* d_saved) {
  if (!p || B < 1 || B > 65535 || !d_y || !d_yhat) return KRIG_EINVAL;
  int r = ensure_ws(p, B);
  if (r != KRIG_OK) return r;
  double* al = d_alpha_out ? d_alpha_out : p->alpha;
  if ((r = do_solve(p, B, d_y, al)) != KRIG_OK) return r;
  const double* filt = nullptr;
  if ((r = filter_for(p, d_lag, &filt)) != KRIG_OK) return r;
  return do_convolve(p, B, al, filt, d_yhat, d_saved ? d_saved : p->S1, nullptr, 0, 0);
}

// Lag-gradient tail: inverse transform of sum_b G_b conj(C_b) from the partial spectra
// written by the adjoint's column pass (G groups), keeping lags -(n-1)..(n-1), then the
// rows and the fold of the sign images into d_dlag.  Reads part, writes XC and d_dlag.
int dlag_tail(krig_plan p, int ngroups, void* d_dlag, hipStream_t st) {
  StageTimer t(p, KRIG_STAGE_DLAG_TAIL);
  // the columns: inverse transform of the summed partial spectra, lags -(n-1)..(n-1)
  ColsArgs ci{};
  ci.H2 = p->H2;
  ci.in = p->part;
  ci.in_fs = (int64_t)p->H2 * p->F1;
  ci.in_ld = p->F1;
  ci.G = ngroups;
  ci.out = p->XC;
  ci.out_ld = p->ldX;
  ci.rows = Window{0, p->n1l, p->F1 - p->n1l + 1, p->n1l - 1};
  ci.twF = p->tw1_64;
  ci.twI = p->tw1_64;
  ci.NL = p->nl_cols64;
  KRIG_TRY(set1(p).inv_sum64(ci, 1, st));
  RowsC2RArgs oc{};
  oc.nrows = p->n1l;
  oc.H2 = p->H2;
  oc.in = p->XC;
  oc.in_fs = 0;
  oc.in_ld = p->ldX;
  oc.out = d_dlag;
  oc.out_fs = 0;
  oc.ldo = p->n2l;
  oc.cols = Window{0, p->n2l, 0, 0};
  oc.twF = p->tw2_64;
  oc.scale = 1.0 / ((double)p->F1 * p->F2);
  oc.NL = p->nl_rows64;
  KRIG_TRY((is32(p) ? set2(p).c2r_fold32 : set2(p).c2r_fold64)(oc, 1, st));
  return KRIG_OK;
}

int krig_predict_adjoint(krig_plan p, int32_t B, const void* d_g, const double* d_alpha, const void* d_saved,
                         const void* d_lag, double* d_dy, void* d_dlag) {
  if (!p || B < 1 || B > 65535 || !d_g) return KRIG_EINVAL;
  if (d_dlag && !d_saved && !d_alpha) return KRIG_EINVAL;
  int r = ensure_ws(p, B);
  if (r != KRIG_OK) return r;
  if ((r = ensure_ws_adj(p, B)) != KRIG_OK) return r;
  const double* filt = nullptr;
  if ((r = filter_for(p, d_lag, &filt)) != KRIG_OK) return r;
  // The adjoint computes in FP64 whatever the plan's dtype: d alpha is multiplied by
  // (K + tau^2 I)^{-1}, whose condition number amplifies any FP32 rounding of the
  // correlation far beyond the gradient tolerance, so the correlation spectra and image
  // stay FP64 in FP32 plans (spec_bytes).
  const void* spec1 = d_saved;
  if (d_dlag && !spec1) {
    // recompute the row spectra of c* from the coefficients
    StageTimer t(p, KRIG_STAGE_ROWS_FWD);
    if ((r = rows_fwd(p, B, d_alpha, p->S1)) != KRIG_OK) return r;
    spec1 = p->S1;
  }
  // rows of g (placed at padded offset L) -> half spectra
  RowsR2CArgs rg{};
  rg.nrows = p->g.m1;
  rg.H2 = p->H2;
  rg.out = p->SG;
  rg.out_fs = (int64_t)p->H2 * p->ldM;
  rg.out_ld = p->ldM;
  rg.twF = p->tw2_64;
  rg.dense = d_g;
  rg.dense_fs = (int64_t)p->g.m1 * p->g.m2;
  rg.dense_ld = p->g.m2;
  rg.coff = p->g.L;
  rg.ncols = p->g.m2;
  rg.NL = p->nl_rows64;
  {
    StageTimer t(p, KRIG_STAGE_ADJ_ROWS_FWD);
    KRIG_TRY((is32(p) ? set2(p).r2c_dense_f32 : set2(p).r2c_dense_f64)(rg, B, p->st));
  }
  // columns: correlation with the (even) filter, keep the P1 padded rows
  ColsArgs c{};
  c.H2 = p->H2;
  c.in = p->SG;
  c.in_fs = (int64_t)p->H2 * p->ldM;
  c.in_ld = p->ldM;
  c.in_off = p->g.L;
  c.in_cnt = p->g.m1;
  c.filt = filt;
  c.filt_ld = p->F1;
  c.out = p->SA;
  c.out_fs = (int64_t)p->H2 * p->ldP;
  c.out_ld = p->ldP;
  c.rows = Window{0, p->P1, 0, 0};
  c.twF = p->tw1_64;
  c.twI = p->tw1_64;
  c.B = B;
  int ngroups = 0;
  if (d_dlag) {
    c.in2 = spec1;
    c.in2_fs = (int64_t)p->H2 * p->ldP;
    c.in2_ld = p->ldP;
    c.in2_off = 0;
    c.in2_cnt = p->P1;
    c.part = p->part;
    c.part_fs = (int64_t)p->H2 * p->F1;
    c.part_ld = p->F1;
    c.NL = std::max(1, std::min(p->dlag_G, (int)B));  // fields (lines) per block
    ngroups = (B + c.NL - 1) / c.NL;
    StageTimer t(p, KRIG_STAGE_ADJ_COLS);
    KRIG_TRY(set1(p).conv_dlag64(c, ngroups, p->st));
  } else {
    c.NL = conv_cols_nl(p);
    StageTimer t(p, KRIG_STAGE_ADJ_COLS);
    KRIG_TRY(conv_cols_fn(p, false)(c, B, p->st));
  }
  // The lag-gradient tail does not depend on the gather and solve below (they read SA,
  // img, alpha and tmpv): with both outputs asked for, it runs on the plan's
  // second stream beside them, filling the compute units the latency-bound solve leaves
  // idle, and joins the plan's stream before this call's work ends.
  const bool fork = d_dlag && d_dy && !p->timing;
  struct Join {
    krig_plan p = nullptr;
    ~Join() {
      if (p) (void)hipStreamWaitEvent(p->st, p->ev_join, 0);
    }
  } join;
  if (fork) {
    KRIG_TRY(hipEventRecord(p->ev_fork, p->st));
    KRIG_TRY(hipStreamWaitEvent(p->aux, p->ev_fork, 0));
    const int rd = dlag_tail(p, ngroups, d_dlag, p->aux);
    KRIG_TRY(hipEventRecord(p->ev_join, p->aux));
    join.p = p;
    if (rd != KRIG_OK) return rd;
  }
  // rows back to the padded image
  RowsC2RArgs o{};
  o.nrows = p->P1;
  o.H2 = p->H2;
  o.in = p->SA;
  o.in_fs = (int64_t)p->H2 * p->ldP;
  o.in_ld = p->ldP;
  o.out = p->img;
  o.out_fs = (int64_t)p->P1 * p->P2;
  o.ldo = p->P2;
  o.cols = Window{0, p->P2, 0, 0};
  o.twF = p->tw2_64;
  o.NL = p->nl_rows64;
  {
    StageTimer t(p, KRIG_STAGE_ADJ_ROWS_INV);
    KRIG_TRY(set2(p).c2r64(o, B, p->st));
  }
  // dalpha by gathering at the neighbours, then dy = M^{-1} dalpha
  if (d_dy) {
    {
      StageTimer t(p, KRIG_STAGE_GATHER);
      KRIG_TRY(gather_sites(p->g, p->ganchor, p->Wt, p->gorder, p->n, p->img, (int64_t)p->P1 * p->P2, p->P2, B, 0, p->alpha,
                            p->n, p->st));
    }
    if ((r = do_solve(p, B, p->alpha, d_dy)) != KRIG_OK) return r;
  }
  if (d_dlag && !fork) return dlag_tail(p, ngroups, d_dlag, p->st);
  return KRIG_OK;
}

int krig_predict_universal(krig_plan p, int32_t B, const double* d_z, int32_t np, const double* d_Xs,
                           const double* d_Xg, void* d_yhat, double* d_beta, double* d_coef) {
  if (!p || B < 1 || B > 65535 - UK_MAX || np < 1 || np > UK_MAX || !d_z || !d_Xs || !d_Xg || !d_yhat)
    return KRIG_EINVAL;
  int r;
  if ((r = ensure_ws(p, std::max<int>(B, np))) != KRIG_OK) return r;
  if ((r = ensure_ws_uk(p, B)) != KRIG_OK) return r;
  const int n = p->n;
  if ((r = do_solve(p, np, d_Xs, p->uk_vx)) != KRIG_OK) return r;  // M^{-1} X
  if ((r = do_solve(p, B, d_z, p->alpha)) != KRIG_OK) return r;    // M^{-1} z
  KRIG_TRY(uk_gram(d_Xs, p->uk_vx, p->alpha, n, np, B, p->uk_G, p->st));
  KRIG_TRY(uk_solve(p->uk_G, np, B, p->uk_beta, p->st));           // eq. findbeta
  KRIG_TRY(uk_resid(p->alpha, p->uk_vx, p->uk_beta, n, np, B, p->st));  // eq. findc
  if ((r = krig_convolve(p, B, p->alpha, nullptr, d_yhat, nullptr)) != KRIG_OK) return r;
  KRIG_TRY(uk_trend(d_yhat, is32(p), d_Xg, p->uk_beta, (int64_t)p->g.m1 * p->g.m2, np, B, p->st));  // predictionf
  if (d_beta)
    KRIG_TRY(hipMemcpyAsync(d_beta, p->uk_beta, sizeof(double) * B * np, hipMemcpyDeviceToDevice, p->st));
  if (d_coef)
    KRIG_TRY(hipMemcpyAsync(d_coef, p->alpha, sizeof(double) * B * n, hipMemcpyDeviceToDevice, p->st));
  return KRIG_OK;
}

int krig_interp(krig_plan p, int32_t B, const void* d_yhat, int32_t npts, const double* d_pts, int32_t q,
                void* d_out) {
  if (!p || B < 1 || B > 65535 || npts < 0 || !d_yhat) return KRIG_EINVAL;
  if (q < 2 || q > 8 || q > p->g.m1 || q > p->g.m2) return KRIG_EINVAL;
  if (npts == 0) return KRIG_OK;
  if (!d_pts || !d_out) return KRIG_EINVAL;
  InterpArgs a{};
  a.yhat = d_yhat;
  a.yhat_fs = (int64_t)p->g.m1 * p->g.m2;
  a.m1 = p->g.m1;
  a.m2 = p->g.m2;
  a.x0 = p->g.x0;
  a.y0 = p->g.y0;
  a.dx = p->g.dx;
  a.dy = p->g.dy;
  a.pts = d_pts;
  a.npts = npts;
  a.out = d_out;
  a.out_fs = npts;
  KRIG_TRY(interp_points(a, B, q, is32(p), p->st));
  return KRIG_OK;
}

static int exact_call(krig_plan p, int32_t B, const double* d_alpha, int32_t npts, const double* d_pts, void* d_out,
                      bool f32) {
  ExactArgs a{};
  a.sites = p->sites;
  a.n = p->n;
  a.alpha = d_alpha;
  a.alpha_fs = p->n;
  a.pts = d_pts;
  a.npts = npts;
  a.g = p->g;
  a.mt = p->mt;
  a.out = d_out;
  a.out_fs = d_pts ? (int64_t)npts : (int64_t)p->g.m1 * p->g.m2;
  const hipError_t e = exact_predict(a, B, f32, p->st);
  return e == hipSuccess ? KRIG_OK : (e == hipErrorInvalidValue ? KRIG_EINVAL : KRIG_EHIP);
}

int krig_predict_exact(krig_plan p, int32_t B, const double* d_alpha, void* d_yhat) {
  if (!p || B < 1 || B > 65535 || !d_alpha || !d_yhat) return KRIG_EINVAL;
  return exact_call(p, B, d_alpha, 0, nullptr, d_yhat, is32(p));
}

int krig_exact_at(krig_plan p, int32_t B, const double* d_alpha, int32_t npts, const double* d_pts, double* d_out) {
  if (!p || B < 1 || B > 65535 || npts < 0 || !d_alpha) return KRIG_EINVAL;
  if (npts == 0) return KRIG_OK;
  if (!d_pts || !d_out) return KRIG_EINVAL;
  return exact_call(p, B, d_alpha, npts, d_pts, d_out, false);
}

int krig_kernel_at(krig_plan p, int32_t i, int32_t npts, const double* d_pts, double* d_out) {
  if (!p || i < 0 || i >= p->n || npts < 0) return KRIG_EINVAL;
  if (npts == 0) return KRIG_OK;
  if (!d_pts || !d_out) return KRIG_EINVAL;
  int32_t anc[2];  // the site's anchor, from the device copy (a small synchronous read)
  KRIG_TRY(hipMemcpyAsync(anc, p->anchor + 2 * (int64_t)i, sizeof(anc), hipMemcpyDeviceToHost, p->st));
  KRIG_TRY(hipStreamSynchronize(p->st));
  KRIG_TRY(kernel_approx_at(p->g, p->mt, anc[0], anc[1], p->W + (int64_t)i * p->M, d_pts, npts, d_out, p->st));
  return KRIG_OK;
}

int krig_plan_tune(krig_plan p, int32_t key, int64_t value) {
  if (!p || value < 1 || value > 256) return KRIG_EINVAL;
  if (p->batch_refs > 0) return KRIG_EINVAL;  // a recorded graph holds the current launches
  const int v = (int)value;
  switch (key) {
    case KRIG_TUNE_DLAG_GROUP:
      if (v * nt_of(p->e1) > 256 || cols_lds(p->e1->geo, v, 16) > 64 * 1024) return KRIG_EINVAL;
      p->dlag_G = v;
      return KRIG_OK;
    case KRIG_TUNE_NL_ROWS64:
      if (v * nt_of(p->e2) > 256 || rows_lds(p->e2->geo, v, 16) > 64 * 1024) return KRIG_EINVAL;
      p->nl_rows64 = v;
      return KRIG_OK;
    case KRIG_TUNE_NL_COLS64:
      if (v * nt_of(p->e1) > 256 || cols_lds(p->e1->geo, v, 16) > 64 * 1024) return KRIG_EINVAL;
      p->nl_cols64 = v;
      return KRIG_OK;
    case KRIG_TUNE_FFT_ROWS:
    case KRIG_TUNE_FFT_COLS: return set_variant(p, key == KRIG_TUNE_FFT_ROWS, (int)value - 1);
    case KRIG_TUNE_COLS_PAIR:
      if (v == 1) {
        p->cols_pair = 0;
        return KRIG_OK;
      }
      if (!p->e1h || v - 1 > 4 || (size_t)(v - 1) * p->e1h->k.pair_ex * 16 > 64 * 1024) return KRIG_EINVAL;
      p->cols_pair = v - 1;
      return KRIG_OK;
    case KRIG_TUNE_SCATTER:
      if (v > 2) return KRIG_EINVAL;
      p->scatter_split = v - 1;  // the next call that takes the scatter apart sizes its image
      return KRIG_OK;
    default: return KRIG_EINVAL;
  }
}

int krig_plan_autotune(krig_plan p, int32_t B, int32_t with_adjoint) {
  if (!p || B < 1 || B > 65535 || p->timing || p->batch_refs > 0) return KRIG_EINVAL;
  int r;
  if ((r = ensure_ws(p, B)) != KRIG_OK) return r;
  if (with_adjoint && (r = ensure_ws_adj(p, B)) != KRIG_OK) return r;
  const size_t npix = (size_t)B * p->g.m1 * p->g.m2;
  double *y = nullptr, *alpha = nullptr, *dy = nullptr;
  void *yhat = nullptr, *gup = nullptr, *dlag = nullptr;
  hipEvent_t e0 = nullptr, e1 = nullptr;
  auto cleanup = [&]() {
    for (void* q : {(void*)y, (void*)alpha, (void*)dy, yhat, gup, dlag}) dfree(p, q);
    if (e0) (void)hipEventDestroy(e0);
    if (e1) (void)hipEventDestroy(e1);
  };
  if ((r = dalloc(p, &y, (size_t)B * p->n)) != KRIG_OK || (r = dalloc(p, &alpha, (size_t)B * p->n)) != KRIG_OK ||
      (r = dalloc(p, &dy, (size_t)B * p->n)) != KRIG_OK || (r = dalloc_bytes(p, &yhat, p->tsz * npix)) != KRIG_OK ||
      (r = dalloc_bytes(p, &gup, p->tsz * npix)) != KRIG_OK ||
      (r = dalloc_bytes(p, &dlag, p->tsz * (size_t)p->n1l * p->n2l)) != KRIG_OK) {
    cleanup();
    return r;
  }
  if (fill_f64(y, (int64_t)B * p->n, 1.0, p->st) != hipSuccess || hipMemsetAsync(gup, 0, p->tsz * npix, p->st) != hipSuccess ||
      hipEventCreate(&e0) != hipSuccess || hipEventCreate(&e1) != hipSuccess) {
    cleanup();
    return KRIG_EHIP;
  }
  auto step = [&]() -> int {
    int q = krig_predict(p, B, y, nullptr, yhat, alpha, p->S1);
    if (q == KRIG_OK && with_adjoint) q = krig_predict_adjoint(p, B, gup, alpha, p->S1, nullptr, dy, dlag);
    return q;
  };
  // median of three windows of ten steps, after two warm-up steps
  auto measure = [&](double* ms) -> int {
    for (int i = 0; i < 2; ++i)
      if (int q = step()) return q;
    double w[3];
    for (int j = 0; j < 3; ++j) {
      if (hipEventRecord(e0, p->st) != hipSuccess) return KRIG_EHIP;
      for (int i = 0; i < 10; ++i)
        if (int q = step()) return q;
      if (hipEventRecord(e1, p->st) != hipSuccess || hipEventSynchronize(e1) != hipSuccess) return KRIG_EHIP;
      float t = 0.f;
      if (hipEventElapsedTime(&t, e0, e1) != hipSuccess) return KRIG_EHIP;
      w[j] = t / 10.0;
    }
    std::sort(w, w + 3);
    *ms = w[1];
    return KRIG_OK;
  };
  auto current = [&](int key) -> int {
    switch (key) {
      case KRIG_TUNE_FFT_ROWS: return p->var_rows + 1;
      case KRIG_TUNE_FFT_COLS: return p->var_cols + 1;
      case KRIG_TUNE_NL_ROWS64: return p->nl_rows64;
      case KRIG_TUNE_NL_COLS64: return p->nl_cols64;
      case KRIG_TUNE_COLS_PAIR: return p->cols_pair + 1;
      case KRIG_TUNE_SCATTER: return p->scatter_split + 1;
      default: return p->dlag_G;
    }
  };
  const int keys[] = {KRIG_TUNE_FFT_ROWS, KRIG_TUNE_FFT_COLS, KRIG_TUNE_NL_ROWS64, KRIG_TUNE_NL_COLS64,
                      KRIG_TUNE_COLS_PAIR, KRIG_TUNE_DLAG_GROUP, KRIG_TUNE_SCATTER};
  for (int key : keys) {
    if (key == KRIG_TUNE_DLAG_GROUP && !with_adjoint) continue;
    if (key == KRIG_TUNE_COLS_PAIR && !p->e1h) continue;
    std::vector<int> cand;
    if (key == KRIG_TUNE_FFT_ROWS || key == KRIG_TUNE_FFT_COLS) {
      const int k = fft_variants(key == KRIG_TUNE_FFT_ROWS ? p->F2 : p->F1, nullptr, 0);
      for (int v = 1; v <= k; ++v) cand.push_back(v);
    } else {
      for (int v = 1; v <= 256; v *= 2) cand.push_back(v);
      for (int v = 256; v >= 1; --v)  // the largest value the key accepts
        if (krig_plan_tune(p, key, v) == KRIG_OK) {
          if (std::find(cand.begin(), cand.end(), v) == cand.end()) cand.push_back(v);
          break;
        }
    }
    // a transform form resets its side's shapes: remember them with the form
    const int keep = current(key);
    const int s64 = p->nl_rows64, sc = p->nl_cols64, sg = p->dlag_G;
    // the current value first; another replaces it only if more than 1% faster
    double keep_ms = 1e300;
    if (krig_plan_tune(p, key, keep) == KRIG_OK && (r = measure(&keep_ms)) != KRIG_OK) {
      cleanup();
      return r;
    }
    int best = keep;
    double best_ms = keep_ms;
    for (int v : cand) {
      if (v == keep || krig_plan_tune(p, key, v) != KRIG_OK) continue;
      double ms = 0;
      if ((r = measure(&ms)) != KRIG_OK) {
        cleanup();
        return r;
      }
      if (ms < 0.99 * best_ms) {
        best_ms = ms;
        best = v;
      }
    }
    krig_plan_tune(p, key, best);
    if ((key == KRIG_TUNE_FFT_ROWS || key == KRIG_TUNE_FFT_COLS) && best == keep) {
      p->nl_rows64 = s64;
      p->nl_cols64 = sc;
      p->dlag_G = sg;
    }
  }
  if (hipStreamSynchronize(p->st) != hipSuccess) {
    cleanup();
    return KRIG_EHIP;
  }
  cleanup();
  {
    std::lock_guard<std::mutex> lk(tune_mutex());
    tune_table()[tune_key(p)] =
        TuneRec{p->var_rows, p->var_cols, p->nl_rows64, p->nl_cols64, p->dlag_G, p->cols_pair, p->n, p->scatter_split};
  }
  return KRIG_OK;
}

int krig_timing_enable(krig_plan p, int32_t on) {
  if (!p) return KRIG_EINVAL;
  p->timing = on != 0;
  return KRIG_OK;
}

int krig_timing_read(krig_plan p, int32_t stage, double* total_ms, int64_t* launches) {
  if (!p || stage < 0 || stage >= KRIG_STAGE_COUNT || !total_ms || !launches) return KRIG_EINVAL;
  double tot = 0.0;
  int64_t cnt = 0;
  for (auto& pr : p->ev_pending[stage]) {
    KRIG_TRY(hipEventSynchronize(pr.second));
    float ms = 0.f;
    KRIG_TRY(hipEventElapsedTime(&ms, pr.first, pr.second));
    tot += ms;
    ++cnt;
    p->ev_pool.push_back(pr.first);
    p->ev_pool.push_back(pr.second);
  }
  p->ev_pending[stage].clear();
  *total_ms = tot;
  *launches = cnt;
  return KRIG_OK;
}

int krig_csim(krig_plan p, int32_t R, uint64_t seed, const double* d_y, void* d_fields) {
  if (!p || R < 1 || R > 65535 || !d_y || !d_fields) return KRIG_EINVAL;
  int r;
  if (!p->lamS && (r = ce_setup(p)) != KRIG_OK) return r;
  if ((r = ensure_ws(p, R)) != KRIG_OK) return r;
  const bool f32 = is32(p);
  const int npairs = (R + 1) / 2;
  if (R > p->csR) {
    KRIG_TRY(hipStreamSynchronize(p->st));
    dfree(p, p->csT);
    dfree(p, p->csU);
    dfree(p, p->csRes);
    dfree(p, p->csAl);
    if ((r = dalloc_bytes(p, &p->csT, csz(p) * (size_t)npairs * p->Fs2 * p->ldP)) != KRIG_OK) return r;
    if ((r = dalloc_bytes(p, &p->csU, p->tsz * (size_t)2 * npairs * p->P1 * p->P2)) != KRIG_OK) return r;
    if ((r = dalloc(p, &p->csRes, (size_t)R * p->n)) != KRIG_OK) return r;
    if ((r = dalloc(p, &p->csAl, (size_t)R * p->n)) != KRIG_OK) return r;
    p->csR = R;
  }
  {
    StageTimer t(p, KRIG_STAGE_CSIM_CE);
    // pass 1: noise x sqrt(Lambda/N) and transforms over the torus columns
    ColsArgs c{};
    c.H2 = p->Fs2;
    c.filt = p->lamS;
    c.filt_ld = p->Fs1;
    c.out = p->csT;
    c.out_fs = (int64_t)p->Fs2 * p->ldP;
    c.out_ld = p->ldP;
    c.rows = Window{0, p->P1, 0, 0};
    c.key0 = (uint32_t)(seed & 0xFFFFFFFFu);
    c.key1 = (uint32_t)(seed >> 32);
    c.pair0 = 0;
    c.ncol_full = p->Fs2;
    c.twF = f32 ? (const void*)p->tws1_32 : (const void*)p->tws1_64;
    c.NL = nl_cols_for(p->es1, csz(p));
    KRIG_TRY((f32 ? p->es1->k.ce_cols32 : p->es1->k.ce_cols64)(c, npairs, p->st));
  }
  {
    StageTimer t(p, KRIG_STAGE_CSIM_ROWS);
    // pass 2: transforms over the torus rows -> two realisations per pair
    RowsCEArgs o{};
    o.nrows = p->P1;
    o.ncols = p->Fs2;
    o.in = p->csT;
    o.in_fs = (int64_t)p->Fs2 * p->ldP;
    o.in_ld = p->ldP;
    o.out = p->csU;
    o.out_fs = (int64_t)p->P1 * p->P2;
    o.ldo = p->P2;
    o.keep = p->P2;
    o.R = R;
    o.pair0 = 0;
    o.twF = f32 ? (const void*)p->tws2_32 : (const void*)p->tws2_64;
    o.NL = nl_ce_rows_for(p->es2, csz(p));
    KRIG_TRY((f32 ? p->es2->k.ce_rows32 : p->es2->k.ce_rows64)(o, npairs, p->st));
  }
  // residual of the data against the simulated data at the sites
  {
    StageTimer t(p, KRIG_STAGE_GATHER);
    KRIG_TRY(csim_residual(p->g, p->ganchor, p->Wt, p->gorder, p->n, p->csU, (int64_t)p->P1 * p->P2, p->P2, R, f32, d_y,
                           sqrt(p->mt.tau2), seed, 0, p->csRes, p->n, p->st));
  }
  if ((r = do_solve(p, R, p->csRes, p->csAl)) != KRIG_OK) return r;
  // krige the residual and add the unconditional field (last pass of the convolution)
  return do_convolve(p, R, p->csAl, p->filt, d_fields, p->S1, p->csU, (int64_t)p->P1 * p->P2, p->P2);
}


// ------------------------------------------------------------------------------ uneven batch
static int check_many(const krig_plan* plans, int32_t count, const int32_t* h_B, const double* const* h_y,
                      void* const* h_yhat) {
  if (!plans || count < 1 || !h_y || !h_yhat) return KRIG_EINVAL;
  for (int i = 0; i < count; ++i)
    if (!plans[i] || !h_y[i] || !h_yhat[i] || (h_B && (h_B[i] < 1 || h_B[i] > 65535))) return KRIG_EINVAL;
  return KRIG_OK;
}

int krig_mixture(const krig_plan* plans, int32_t C, int32_t B, const double* d_alpha, const double* d_lam_sites,
                 const double* d_lam_grid, void* d_yhat, void* stream) {
  if (!plans || C < 1 || C > MIX_MAX || B < 1 || B > 65535 || !d_alpha || !d_lam_sites || !d_lam_grid || !d_yhat)
    return KRIG_EINVAL;
  const krig_plan p0 = plans[0];
  if (!p0) return KRIG_EINVAL;
  for (int c = 0; c < C; ++c) {
    const krig_plan p = plans[c];
    if (!p || p->n != p0->n || p->dtype != p0->dtype || p->g.m1 != p0->g.m1 || p->g.m2 != p0->g.m2 ||
        p->g.x0 != p0->g.x0 || p->g.y0 != p0->g.y0 || p->g.dx != p0->g.dx || p->g.dy != p0->g.dy)
      return KRIG_EINVAL;
    for (int e = 0; e < c; ++e)
      if (plans[e] == p) return KRIG_EINVAL;  // each component needs its own workspaces
  }
  const hipStream_t st = stream ? (hipStream_t)stream : p0->st;
  const int n = p0->n;
  // Components with the same neighbour order share every transform geometry: the scaling of
  // the coefficients by lam_c(s_i) rides in each component's scatter, and one inverse-row
  // launch transforms all components' rows and adds lam_c times them in FP64 (no component
  // images, no combine pass).  Otherwise each component is predicted into its plan's
  // workspace and a combine pass adds them.
  bool fused = true;
  for (int c = 1; c < C; ++c) {
    const krig_plan p = plans[c];
    fused = fused && p->g.L == p0->g.L && p->e1 == p0->e1 && p->e2 == p0->e2 && p->P1 == p0->P1 &&
            p->P2 == p0->P2 && p->ldP == p0->ldP && p->ldM == p0->ldM && p->H2 == p0->H2;
  }
  if (fused) {
    static_assert(MIX_MAX <= MIX_COMP_MAX, "mixture components");
    MixRowsArgs m{};
    m.r = rows_inv_args(p0, d_yhat);
    m.r.in = nullptr;
    m.lam = d_lam_grid;
    m.lam_cs = (int64_t)p0->g.m1 * p0->g.m2;
    m.lam_ld = p0->g.m2;
    m.C = C;
    for (int c = 0; c < C; ++c) {
      const krig_plan p = plans[c];
      int r;
      if ((r = ensure_ws(p, B)) != KRIG_OK) return r;
      RowsR2CArgs ra = rows_fwd_args(p, d_alpha, p->S1);
      ra.alpha_scale = d_lam_sites + (size_t)c * n;
      KRIG_TRY(set2(p).r2c_csr_scaled(ra, B, st));
      KRIG_TRY(conv_cols_fn(p, is32(p))(cols_conv_args(p, p->S1, p->filt, B), B, st));
      m.in[c] = p->S2;
    }
    KRIG_TRY((is32(p0) ? set2(p0).c2r_mix_f32 : set2(p0).c2r_mix64)(m, B, st));
    return KRIG_OK;
  }
  MixArgs m{};
  m.lam = d_lam_grid;
  m.C = C;
  m.npix = (int64_t)p0->g.m1 * p0->g.m2;
  m.B = B;
  m.out = d_yhat;
  for (int c = 0; c < C; ++c) {
    const krig_plan p = plans[c];
    int r;
    if ((r = ensure_ws(p, B)) != KRIG_OK || (r = ensure_ws_mix(p, B)) != KRIG_OK) return r;
    const hipStream_t old = p->st;
    p->st = st;
    // component c: the coefficients lam_c(s_i) alpha_i through this plan's rapid predictor
    r = hip_status(mix_scale_coef(d_alpha, d_lam_sites + (size_t)c * n, n, B, p->alpha, st));
    if (r == KRIG_OK) r = krig_convolve(p, B, p->alpha, nullptr, p->mix, nullptr);
    p->st = old;
    if (r != KRIG_OK) return r;
    m.comp[c] = p->mix;
  }
  KRIG_TRY(mix_combine(m, is32(p0), st));
  return KRIG_OK;
}

int krig_predict_many(const krig_plan* plans, int32_t count, const int32_t* h_B, const double* const* h_y,
                      void* const* h_yhat, void* stream) {
  int r = check_many(plans, count, h_B, h_y, h_yhat);
  if (r != KRIG_OK) return r;
  for (int i = 0; i < count; ++i) {
    krig_plan p = plans[i];
    const hipStream_t old = p->st;
    if (stream) p->st = (hipStream_t)stream;
    r = krig_predict(p, h_B ? h_B[i] : 1, h_y[i], nullptr, h_yhat[i], nullptr, nullptr);
    p->st = old;
    if (r != KRIG_OK) return r;
  }
  return KRIG_OK;
}



static void batch_free(krig_batch b) {
  if (b->qbuf) (void)hipFree(b->qbuf);
  if (b->exec) (void)hipGraphExecDestroy(b->exec);
  if (b->graph) (void)hipGraphDestroy(b->graph);
  if (b->own) (void)hipStreamDestroy(b->own);
  for (krig_plan p : b->plans) --p->batch_refs;
  delete b;
}

int krig_batch_create(krig_batch* out, const krig_plan* plans, int32_t count, const int32_t* h_B,
                      const double* const* h_y, void* const* h_yhat, int32_t lanes, void* stream) {
  if (!out || lanes < 0 || lanes > 16) return KRIG_EINVAL;
  int r = check_many(plans, count, h_B, h_y, h_yhat);
  if (r != KRIG_OK) return r;
  for (int i = 0; i < count; ++i)
    if (plans[i]->timing) return KRIG_EINVAL;
  if (lanes == 0)  // the work-queue form runs all problems' passes at once: one plan each
    for (int i = 0; i < count; ++i)
      for (int j = 0; j < i; ++j)
        if (plans[j] == plans[i]) return KRIG_EINVAL;
  // workspaces at their final size before anything is recorded
  for (int i = 0; i < count; ++i)
    if ((r = ensure_ws(plans[i], h_B ? h_B[i] : 1)) != KRIG_OK) return r;
  krig_batch b = new krig_batch_s();
  if (!stream) {
    if (hipStreamCreateWithFlags(&b->own, hipStreamNonBlocking) != hipSuccess) {
      delete b;
      return KRIG_EHIP;
    }
    b->cap = b->own;
  } else {
    b->cap = (hipStream_t)stream;
  }
  for (int i = 0; i < count; ++i) {
    b->plans.push_back(plans[i]);
    ++plans[i]->batch_refs;
  }
  if (lanes == 0) {
    r = batch_queue_record(b, plans, count, h_B, h_y, h_yhat, b->cap);
    if (r != KRIG_OK) {
      batch_free(b);
      return r;
    }
    *out = b;
    return KRIG_OK;
  }
  // problems to branches: the problems of one plan share its workspaces, so they stay
  // on one branch (in order); plans go largest first to the least-loaded branch
  std::vector<krig_plan> uniq;
  std::vector<int> grp(count);
  for (int i = 0; i < count; ++i) {
    const auto it = std::find(uniq.begin(), uniq.end(), plans[i]);
    grp[i] = (int)(it - uniq.begin());
    if (it == uniq.end()) uniq.push_back(plans[i]);
  }
  const int ng = (int)uniq.size();
  std::vector<double> cost(ng, 0.0);
  for (int i = 0; i < count; ++i) {
    const krig_plan p = plans[i];
    const double Bi = h_B ? h_B[i] : 1;
    cost[grp[i]] += Bi * ((double)p->F1 * p->F2 * 2.0 + (double)p->n * p->n);
  }
  std::vector<int> order(ng);
  for (int g = 0; g < ng; ++g) order[g] = g;
  std::stable_sort(order.begin(), order.end(), [&](int a, int c) { return cost[a] > cost[c]; });
  const int nl = std::min<int>(lanes, ng);
  std::vector<double> load(nl, 0.0);
  std::vector<int> lane_of_grp(ng, 0), lane_of(count, 0);
  for (int g : order) {
    const int k = (int)(std::min_element(load.begin(), load.end()) - load.begin());
    lane_of_grp[g] = k;
    load[k] += cost[g];
  }
  for (int i = 0; i < count; ++i) lane_of[i] = lane_of_grp[grp[i]];
  std::vector<hipStream_t> ls(nl, nullptr);
  std::vector<hipEvent_t> ev(nl + 1, nullptr);
  std::vector<hipStream_t> old(count);
  for (int i = 0; i < count; ++i) old[i] = plans[i]->st;
  hipError_t e = hipSuccess;
  bool capturing = false;
  for (int k = 0; k < nl && e == hipSuccess; ++k) e = hipStreamCreateWithFlags(&ls[k], hipStreamNonBlocking);
  for (int k = 0; k <= nl && e == hipSuccess; ++k) e = hipEventCreateWithFlags(&ev[k], hipEventDisableTiming);
  if (e == hipSuccess) e = hipStreamBeginCapture(b->cap, hipStreamCaptureModeThreadLocal);
  if (e == hipSuccess) {
    capturing = true;
    e = hipEventRecord(ev[nl], b->cap);  // fork
    for (int k = 0; k < nl && e == hipSuccess; ++k) e = hipStreamWaitEvent(ls[k], ev[nl], 0);
  }
  r = e == hipSuccess ? KRIG_OK : KRIG_EHIP;
  for (int i = 0; i < count && r == KRIG_OK; ++i) {
    plans[i]->st = ls[lane_of[i]];
    r = krig_predict(plans[i], h_B ? h_B[i] : 1, h_y[i], nullptr, h_yhat[i], nullptr, nullptr);
    plans[i]->st = old[i];
  }
  for (int k = 0; k < nl && r == KRIG_OK; ++k) {  // join
    if (hipEventRecord(ev[k], ls[k]) != hipSuccess || hipStreamWaitEvent(b->cap, ev[k], 0) != hipSuccess) r = KRIG_EHIP;
  }
  if (capturing) {
    hipGraph_t g = nullptr;
    const hipError_t ee = hipStreamEndCapture(b->cap, &g);
    if (r == KRIG_OK && ee != hipSuccess) r = KRIG_EHIP;
    if (r == KRIG_OK) {
      b->graph = g;
      if (hipGraphInstantiate(&b->exec, b->graph, nullptr, nullptr, 0) != hipSuccess) r = KRIG_EHIP;
    } else if (g) {
      (void)hipGraphDestroy(g);
    }
  }
  for (int i = 0; i < count; ++i) plans[i]->st = old[i];
  for (auto s_ : ls)
    if (s_) (void)hipStreamDestroy(s_);
  for (auto v : ev)
    if (v) (void)hipEventDestroy(v);
  if (r != KRIG_OK) {
    batch_free(b);
    return r;
  }
  *out = b;
  return KRIG_OK;
}

int krig_batch_launch(krig_batch b, void* stream) {
  if (!b || !b->exec) return KRIG_EINVAL;
  KRIG_TRY(hipGraphLaunch(b->exec, stream ? (hipStream_t)stream : b->cap));
  return KRIG_OK;
}

int krig_batch_destroy(krig_batch b) {
  if (!b) return KRIG_EINVAL;
  batch_free(b);
  return KRIG_OK;
}

}  // extern "C"
