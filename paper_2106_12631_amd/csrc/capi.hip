// C ABI of the library (declarations and contracts in include/mg5mi.h).
#include <math.h>
#include <stdlib.h>
#include <string.h>

#include <new>

#include "mg5mi.h"
#include "internal.h"

namespace mg {
#define MG_DECL(p)                                                                          \
  int launch_sigmakin_##p##_f64(const MeArgs&, const double*, int64_t, double*, const double*, \
                                double*, double*, hipStream_t);                            \
  int launch_sigmakin_##p##_f32(const MeArgs&, const double*, int64_t, double*, const double*, \
                                double*, double*, hipStream_t);
MG_DECL(eemumu)
MG_DECL(ggtt)
MG_DECL(ggttg)
MG_DECL(ggttgg)
#undef MG_DECL
#define MG_DECL(p)                                                                              \
  int launch_sigmakin_##p##_mfma_f32(const MeArgs&, const double*, int64_t, double*, const double*, \
                                     double*, hipStream_t);                                     \
  int launch_sigmakin_##p##_mfma_bf16(const MeArgs&, const double*, int64_t, double*,              \
                                      const double*, double*, hipStream_t);
MG_DECL(eemumu)
MG_DECL(ggtt)
MG_DECL(ggttg)
MG_DECL(ggttgg)
#undef MG_DECL

typedef int (*skm_fn)(const MeArgs&, const double*, int64_t, double*, const double*, double*,
                      hipStream_t);
static const skm_fn SKM[4][2] = {
    {launch_sigmakin_eemumu_mfma_f32, launch_sigmakin_eemumu_mfma_bf16},
    {launch_sigmakin_ggtt_mfma_f32, launch_sigmakin_ggtt_mfma_bf16},
    {launch_sigmakin_ggttg_mfma_f32, launch_sigmakin_ggttg_mfma_bf16},
    {launch_sigmakin_ggttgg_mfma_f32, launch_sigmakin_ggttgg_mfma_bf16},
};

typedef int (*sk_fn)(const MeArgs&, const double*, int64_t, double*, const double*, double*,
                     double*, hipStream_t);
static const sk_fn SK[4][2] = {
    {launch_sigmakin_eemumu_f64, launch_sigmakin_eemumu_f32},
    {launch_sigmakin_ggtt_f64, launch_sigmakin_ggtt_f32},
    {launch_sigmakin_ggttg_f64, launch_sigmakin_ggttg_f32},
    {launch_sigmakin_ggttgg_f64, launch_sigmakin_ggttgg_f32},
};

#define MG_DECL(p)                                                                          \
  int launch_sigmakin_##p##_guard(const MeArgs&, const double*, int64_t, double*, const double*, \
                                  double*, hipStream_t);
MG_DECL(eemumu)
MG_DECL(ggtt)
MG_DECL(ggttg)
MG_DECL(ggttgg)
#undef MG_DECL
static const skm_fn GUARD[4] = {launch_sigmakin_eemumu_guard, launch_sigmakin_ggtt_guard,
                                launch_sigmakin_ggttg_guard, launch_sigmakin_ggttgg_guard};

// prec: 0 FP64, 1 FP32 amplitudes + VALU colour sum, 2 mixed (BF16-split MFMA
// colour sum for 24 colour flows, FP32 MFMA otherwise), 3 mixed with FP32 MFMA;
// the reduced-precision forms are followed by the precision guard (FP64 for
// the ill-conditioned events) when a.guard_kappa > 0
int launch_sigmakin(int proc, int prec, const MeArgs& a, const double* mom, int64_t nevt,
                    double* me, const double* wgt, double* evtw, hipStream_t s) {
  if (proc < 0 || proc > 3 || prec < 0 || prec > 3) return -1;
  int rc;
  if (prec == 0) return SK[proc][0](a, mom, nevt, me, wgt, evtw, nullptr, s);
  if (prec == 1) {
    rc = SK[proc][1](a, mom, nevt, me, wgt, evtw, nullptr, s);
  } else {
    const int bf16 = (prec == 2 && proc == MG_GGTTGG) ? 1 : 0;
    rc = SKM[proc][bf16](a, mom, nevt, me, wgt, evtw, s);
  }
  if (rc) return rc;
  return GUARD[proc](a, mom, nevt, me, wgt, evtw, s);
}

int launch_sigmakin_hel(int proc, int prec, const MeArgs& a, const double* mom, int64_t nevt,
                        double* mehel, hipStream_t s) {
  if (proc < 0 || proc > 3 || prec < 0 || prec > 1) return -1;
  return SK[proc][prec](a, mom, nevt, nullptr, nullptr, nullptr, mehel, s);
}

int launch_grad_eemumu(int, const MeArgs&, const RamboArgs&, const double*, int64_t, const double*,
                       double*, double*, double*, hipStream_t);
int launch_grad_ggtt(int, const MeArgs&, const RamboArgs&, const double*, int64_t, const double*,
                     double*, double*, double*, hipStream_t);
int launch_grad_ggttg(int, const MeArgs&, const RamboArgs&, const double*, int64_t, const double*,
                      double*, double*, double*, hipStream_t);

__global__ void __launch_bounds__(256) count_nonfinite_kernel(const double* __restrict__ x,
                                                              int64_t n,
                                                              unsigned long long* count) {
  __shared__ int part[256];
  int local = 0;
  for (int64_t i = (int64_t)blockIdx.x * 256 + threadIdx.x; i < n; i += (int64_t)gridDim.x * 256)
    local += isfinite(x[i]) ? 0 : 1;
  part[threadIdx.x] = local;
  __syncthreads();
  for (int st = 128; st > 0; st >>= 1) {
    if ((int)threadIdx.x < st) part[threadIdx.x] += part[threadIdx.x + st];
    __syncthreads();
  }
  if (threadIdx.x == 0 && part[0]) atomicAdd(count, (unsigned long long)part[0]);
}

int launch_count_nonfinite(const double* x, int64_t n, int64_t* d_count, hipStream_t s) {
  int64_t blocks = (n + 255) / 256;
  if (blocks > 4096) blocks = 4096;
  if (blocks < 1) blocks = 1;
  count_nonfinite_kernel<<<(unsigned)blocks, 256, 0, s>>>(x, n, (unsigned long long*)d_count);
  return 0;
}

}  // namespace mg

using namespace mg;

struct ProcInfo {
  int npar, ncol, ndiag, iden;
};

static const ProcInfo PROC_INFO[4] = {
    {4, 1, 2, 4},      // e+ e- -> mu+ mu-
    {4, 2, 3, 256},    // g g -> t t~
    {5, 6, 16, 256},   // g g -> t t~ g
    {6, 24, 123, 512}, // g g -> t t~ g g
};

struct mg_handle {
  int proc;
  int prec;
  mg_params_t prm;
  RamboArgs rambo;
  MeArgs me;
  int nhel_good;
};

static bool aligned8(const void* p) { return ((uintptr_t)p & 7u) == 0; }

static int hip_status() {
  const hipError_t e = hipGetLastError();
  return e == hipSuccess ? MG_OK : MG_EHIP;
}

static void derive(mg_handle* h) {
  const mg_params_t& p = h->prm;
  const double pi = 3.14159265358979323846;
  const double alpha = 1.0 / p.alpha_inv;
  const double e = sqrt(4.0 * pi * alpha);
  const double gs = sqrt(4.0 * pi * p.alphas);
  const double mz2 = p.mZ * p.mZ;
  const double mw2 = mz2 / 2.0 + sqrt(mz2 * mz2 / 4.0 - pi * alpha * mz2 / (sqrt(2.0) * p.gfermi));
  const double sw2 = 1.0 - mw2 / mz2;
  const double swcw = sqrt(sw2 * (1.0 - sw2));
  const double Q = -1.0, T3 = -0.5;  // charged leptons
  Couplings<double> c;
  c.gs = gs;
  c.gs2 = gs * gs;
  c.cqed = -e * Q;
  c.czl = -(e / swcw) * (T3 - Q * sw2);
  c.czr = -(e / swcw) * (-Q * sw2);
  c.mt = p.mt;
  c.wt = p.wt;
  c.wtt = (p.flags & MG_FLAG_TCHANNEL_ZERO_WIDTH) ? 0.0 : p.wt;
  c.mz = p.mZ;
  c.wz = p.wZ;
  h->me.c64 = c;
  Couplings<float> f;
  f.gs = (float)c.gs;
  f.gs2 = (float)c.gs2;
  f.cqed = (float)c.cqed;
  f.czl = (float)c.czl;
  f.czr = (float)c.czr;
  f.mt = c.mt;
  f.wt = c.wt;
  f.wtt = c.wtt;
  f.mz = c.mz;
  f.wz = c.wz;
  h->me.c32 = f;
  h->me.inv_iden = 1.0 / PROC_INFO[h->proc].iden;
  h->me.guard_kappa =
      (h->prec != MG_FP64 && !(p.flags & MG_FLAG_NO_PRECISION_GUARD)) ? MG_PRECISION_GUARD_KAPPA : 0.0;

  const int nf = PROC_INFO[h->proc].npar - 2;
  RamboArgs& r = h->rambo;
  r.sqrts = p.sqrts;
  const double s = p.sqrts * p.sqrts;
  double fact1 = 1.0, fact2 = 1.0;
  for (int k = 2; k <= nf - 1; ++k) fact1 *= k;
  for (int k = 2; k <= nf - 2; ++k) fact2 *= k;
  r.w0 = pow(pi / 2.0, nf - 1) * pow(s, nf - 2) / (fact1 * fact2);
  if (p.flags & MG_FLAG_WEIGHT_2PI) r.w0 *= pow(2.0 * pi, 4 - 3 * nf);
  double msum = 0.0;
  for (int i = 0; i < 4; ++i) r.m2[i] = 0.0;
  if (h->proc != MG_EEMUMU) {
    r.m2[0] = r.m2[1] = p.mt * p.mt;
    msum = 2.0 * p.mt;
  }
  r.massive = msum > 0.0;
  r.xi0 = sqrt(1.0 - (msum / p.sqrts) * (msum / p.sqrts));
}

// Helicity filtering (Sec. II): the helicities whose contribution is
// exactly zero in FP64 on a small sample of events are dropped (reading:
// only exact zeros, never small ones).
static int filter_helicities(mg_handle* h) {
  const int npar = PROC_INFO[h->proc].npar;
  const int nhel = 1 << npar;
  const int64_t n = 64;
  double *mom = nullptr, *wgt = nullptr, *mehel = nullptr;
  const size_t mom_bytes = sizeof(double) * (size_t)npar * 4 * ((n + NEPPM - 1) / NEPPM) * NEPPM;
  if (hipMalloc(&mom, mom_bytes) != hipSuccess || hipMalloc(&wgt, sizeof(double) * n) != hipSuccess ||
      hipMalloc(&mehel, sizeof(double) * n * nhel) != hipSuccess) {
    (void)hipFree(mom);
    (void)hipFree(wgt);
    (void)hipFree(mehel);
    (void)hipGetLastError();
    return MG_ENOMEM;
  }
  int rc = MG_OK;
  double* host = (double*)malloc(sizeof(double) * n * nhel);
  if (!host) rc = MG_ENOMEM;
  if (rc == MG_OK && launch_sample(npar - 2, 0x5EEDull, 0, n, h->rambo, nullptr, mom, wgt, 0))
    rc = MG_ENOTSUP;
  if (rc == MG_OK && launch_sigmakin_hel(h->proc, 0, h->me, mom, n, mehel, 0)) rc = MG_ENOTSUP;
  if (rc == MG_OK) rc = hip_status();
  if (rc == MG_OK && hipMemcpy(host, mehel, sizeof(double) * n * nhel, hipMemcpyDeviceToHost) != hipSuccess)
    rc = MG_EHIP;
  if (rc == MG_OK) {
    h->me.hel.n = 0;
    for (int ih = 0; ih < nhel; ++ih) {
      bool keep = false;
      for (int64_t i = 0; i < n; ++i) keep |= host[ih * n + i] != 0.0;
      if (keep) h->me.hel.code[h->me.hel.n++] = (uint8_t)ih;
    }
    h->nhel_good = h->me.hel.n;
  }
  free(host);
  (void)hipFree(mom);
  (void)hipFree(wgt);
  (void)hipFree(mehel);
  return rc;
}

extern "C" {

int mg_create(int proc, int prec, const mg_params_t* prm, mg_handle_t** out) {
  if (!out || proc < 0 || proc > 3 || prec < 0 || prec > 3) return MG_EINVAL;
  *out = nullptr;
  mg_params_t p = {1500.0, 132.5, 1.16639e-5, 91.188, 2.441, 173.0, 1.49, 0.118, 0};
  if (prm) p = *prm;
  if (!(p.sqrts > 0) || !(p.alpha_inv > 0) || !(p.gfermi > 0) || !(p.mZ > 0) || p.wZ < 0 ||
      p.mt < 0 || p.wt < 0 || !(p.alphas > 0) ||
      (p.flags & ~(MG_FLAG_TCHANNEL_ZERO_WIDTH | MG_FLAG_WEIGHT_2PI | MG_FLAG_NO_PRECISION_GUARD)) != 0)
    return MG_EINVAL;
  if (proc != MG_EEMUMU && 2.0 * p.mt >= p.sqrts) return MG_ENOPHASE;
  mg_handle* h = new (std::nothrow) mg_handle();
  if (!h) return MG_ENOMEM;
  h->proc = proc;
  h->prec = prec;
  h->prm = p;
  derive(h);
  const int rc = filter_helicities(h);
  if (rc != MG_OK) {
    delete h;
    return rc;
  }
  *out = h;
  return MG_OK;
}

int mg_destroy(mg_handle_t* h) {
  delete h;
  return MG_OK;
}

int mg_layout(const mg_handle_t* h, mg_layout_t* o) {
  if (!h || !o) return MG_EINVAL;
  const ProcInfo& pi = PROC_INFO[h->proc];
  o->npar = pi.npar;
  o->nparf = pi.npar - 2;
  o->nrnd = 4 * (pi.npar - 2);
  o->nhel = 1 << pi.npar;
  o->nhel_good = h->nhel_good;
  o->ncol = pi.ncol;
  o->ndiag = pi.ndiag;
  o->neppM = NEPPM;
  o->neppR = NEPPR;
  o->iden = pi.iden;
  return MG_OK;
}

int mg_rng(const mg_handle_t* h, uint64_t seed, int64_t evt_offset, int64_t nevt, double* rnd,
           void* stream) {
  if (!h || nevt < 0 || evt_offset < 0 || (nevt > 0 && !rnd)) return MG_EINVAL;
  if (!aligned8(rnd)) return MG_EALIGN;
  if (nevt == 0) return MG_OK;
  if (launch_rng(4 * (PROC_INFO[h->proc].npar - 2), seed, evt_offset, nevt, rnd, (hipStream_t)stream))
    return MG_ENOTSUP;
  return hip_status();
}

int mg_rambo(const mg_handle_t* h, const double* rnd, int64_t nevt, double* mom, double* wgt,
             void* stream) {
  if (!h || nevt < 0 || (nevt > 0 && (!rnd || !mom || !wgt))) return MG_EINVAL;
  if (!aligned8(rnd) || !aligned8(mom) || !aligned8(wgt)) return MG_EALIGN;
  if (nevt == 0) return MG_OK;
  if (launch_rambo(PROC_INFO[h->proc].npar - 2, rnd, nevt, h->rambo, mom, wgt, (hipStream_t)stream))
    return MG_ENOTSUP;
  return hip_status();
}

int mg_sample(const mg_handle_t* h, uint64_t seed, int64_t evt_offset, int64_t nevt,
              double* rnd_or_null, double* mom, double* wgt, void* stream) {
  if (!h || nevt < 0 || evt_offset < 0 || (nevt > 0 && (!mom || !wgt))) return MG_EINVAL;
  if (!aligned8(rnd_or_null) || !aligned8(mom) || !aligned8(wgt)) return MG_EALIGN;
  if (nevt == 0) return MG_OK;
  if (launch_sample(PROC_INFO[h->proc].npar - 2, seed, evt_offset, nevt, h->rambo, rnd_or_null, mom,
                    wgt, (hipStream_t)stream))
    return MG_ENOTSUP;
  return hip_status();
}

int mg_sigmakin(const mg_handle_t* h, const double* mom, int64_t nevt, double* me,
                const double* wgt_or_null, double* evtw_or_null, void* stream) {
  if (!h || nevt < 0 || (nevt > 0 && (!mom || !me))) return MG_EINVAL;
  if ((wgt_or_null == nullptr) != (evtw_or_null == nullptr)) return MG_EINVAL;
  if (!aligned8(mom) || !aligned8(me) || !aligned8(wgt_or_null) || !aligned8(evtw_or_null))
    return MG_EALIGN;
  if (nevt == 0) return MG_OK;
  if (launch_sigmakin(h->proc, h->prec, h->me, mom, nevt, me, wgt_or_null, evtw_or_null,
                      (hipStream_t)stream))
    return MG_ENOTSUP;
  return hip_status();
}

int mg_sigmakin_hel(const mg_handle_t* h, const double* mom, int64_t nevt, double* mehel,
                    void* stream) {
  if (!h || nevt < 0 || (nevt > 0 && (!mom || !mehel))) return MG_EINVAL;
  if (!aligned8(mom) || !aligned8(mehel)) return MG_EALIGN;
  if (nevt == 0) return MG_OK;
  const int prec = h->prec == MG_FP64 ? 0 : 1;
  if (launch_sigmakin_hel(h->proc, prec, h->me, mom, nevt, mehel, (hipStream_t)stream))
    return MG_ENOTSUP;
  return hip_status();
}

int mg_adjoint(const mg_handle_t* h, const double* rnd, int64_t nevt, const double* gbar_or_null,
               double* grad_rnd, double* grad_logw_or_null, double* f_or_null, void* stream) {
  if (!h || nevt < 0 || (nevt > 0 && (!rnd || !grad_rnd))) return MG_EINVAL;
  if (!aligned8(rnd) || !aligned8(gbar_or_null) || !aligned8(grad_rnd) ||
      !aligned8(grad_logw_or_null) || !aligned8(f_or_null))
    return MG_EALIGN;
  if (h->proc == MG_GGTTGG) return MG_ENOTSUP;
  if (nevt == 0) return MG_OK;
  const int prec = h->prec == MG_FP64 ? 0 : 1;
  hipStream_t s = (hipStream_t)stream;
  int rc = 0;
  switch (h->proc) {
    case MG_EEMUMU:
      rc = launch_grad_eemumu(prec, h->me, h->rambo, rnd, nevt, gbar_or_null, grad_rnd,
                              grad_logw_or_null, f_or_null, s);
      break;
    case MG_GGTT:
      rc = launch_grad_ggtt(prec, h->me, h->rambo, rnd, nevt, gbar_or_null, grad_rnd,
                            grad_logw_or_null, f_or_null, s);
      break;
    case MG_GGTTG:
      rc = launch_grad_ggttg(prec, h->me, h->rambo, rnd, nevt, gbar_or_null, grad_rnd,
                             grad_logw_or_null, f_or_null, s);
      break;
  }
  if (rc) return MG_ENOTSUP;
  return hip_status();
}

int mg_unweight_noalloc(const double* f, int64_t n, double fmax, uint64_t seed,
                        int64_t evt_offset, int64_t* idx_out, int64_t* count_out, void* stream) {
  if (n < 0 || evt_offset < 0 || !count_out || (n > 0 && (!f || !idx_out)) || !(fmax >= 0.0))
    return MG_EINVAL;
  if (n > MG_UNWEIGHT_NOALLOC_MAX_EVENTS) return MG_ERANGE;
  if (!aligned8(f) || !aligned8(idx_out) || !aligned8(count_out)) return MG_EALIGN;
  int64_t* ws = unweight_scratch();
  if (!ws) return MG_EHIP;
  if (launch_unweight(f, n, fmax, seed, evt_offset, idx_out, count_out, ws, (hipStream_t)stream))
    return MG_EINVAL;
  return hip_status();
}

int mg_count_nonfinite(const double* x, int64_t n, int64_t* d_count, void* stream) {
  if (n < 0 || !d_count || (n > 0 && !x)) return MG_EINVAL;
  if (!aligned8(x) || !aligned8(d_count)) return MG_EALIGN;
  if (n == 0) return MG_OK;
  launch_count_nonfinite(x, n, d_count, (hipStream_t)stream);
  return hip_status();
}

int64_t mg_xsec_stats_workspace_bytes(int64_t n) {
  return xsec_blocks(n < 0 ? 0 : n) * 4 * (int64_t)sizeof(double);
}

int mg_xsec_stats(const double* f, int64_t n, double* stats, void* workspace, void* stream) {
  if (n < 0 || !stats || !workspace || (n > 0 && !f)) return MG_EINVAL;
  if (!aligned8(f) || !aligned8(stats) || !aligned8(workspace)) return MG_EALIGN;
  launch_xsec_stats(f, n, stats, (double*)workspace, (hipStream_t)stream);
  return hip_status();
}

int mg_xsec(const mg_handle_t* h, const double* st, int64_t n, double* sigma_pb,
            double* error_pb) {
  if (!h || !st || !sigma_pb || !error_pb || n < 2) return MG_EINVAL;
  const int nfinal = PROC_INFO[h->proc].npar - 2;
  const double s = h->prm.sqrts * h->prm.sqrts;
  const double hbarc2_pb = 0.3893793721e9;
  const double twopi = (h->prm.flags & MG_FLAG_WEIGHT_2PI) ? 1.0 : pow(2.0 * M_PI, 4 - 3 * nfinal);
  const double scale = hbarc2_pb * twopi / (2.0 * s);
  const double mean = st[0] / (double)n;
  double var = st[1] / (double)n - mean * mean;
  if (var < 0.0) var = 0.0;
  *sigma_pb = scale * mean;
  *error_pb = scale * sqrt(var / (double)(n - 1));
  return MG_OK;
}

int64_t mg_unweight_workspace_bytes(int64_t n) {
  return n <= 0 ? 8 : unweight_blocks(n) * (int64_t)sizeof(int64_t);
}

int mg_unweight(const double* f, int64_t n, double fmax, uint64_t seed, int64_t evt_offset,
                int64_t* idx_out, int64_t* count_out, void* workspace, void* stream) {
  if (n < 0 || evt_offset < 0 || !count_out || (n > 0 && (!f || !idx_out || !workspace)) ||
      !(fmax >= 0.0))
    return MG_EINVAL;
  if (!aligned8(f) || !aligned8(idx_out) || !aligned8(count_out) || !aligned8(workspace))
    return MG_EALIGN;
  if (launch_unweight(f, n, fmax, seed, evt_offset, idx_out, count_out, (int64_t*)workspace,
                      (hipStream_t)stream))
    return MG_EINVAL;
  return hip_status();
}

const char* mg_strerror(int code) {
  switch (code) {
    case MG_OK: return "success";
    case MG_EINVAL: return "invalid argument";
    case MG_ENOTSUP: return "not supported for this process or precision";
    case MG_ENOPHASE: return "no phase space: sum of masses >= sqrt(s)";
    case MG_EHIP: return "HIP runtime or kernel launch error";
    case MG_EALIGN: return "buffer not 8-byte aligned";
    case MG_ENOMEM: return "allocation failed";
    case MG_ERANGE: return "size exceeds the fixed scratch of the allocation-free entry point";
  }
  return "unknown error";
}

}  // extern "C"
