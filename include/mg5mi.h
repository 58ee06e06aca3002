/* mg5mi.h -- C ABI of the per-event |M|^2 library for AMD MI355X (gfx950).
 *
 * The library evaluates, for baskets of independent events, the three
 * components of the workflow in Sec. IV.a/IV.b of arxiv 2106.12631: a
 * random-number generator, the RAMBO phase-space sampler and the
 * matrix-element engine (SIGMAKIN: helicity amplitudes, colour-flow
 * amplitudes, colour sum, helicity sum; Sec. II).  Every call works on one
 * "iteration" of events held in caller-owned device arrays of fixed
 * dimension (Sec. IV.b).
 *
 * Ownership and threading
 *   - Every buffer pointer is a DEVICE pointer owned by the caller; the
 *     library never allocates, frees or keeps caller memory.  Pointers must
 *     be 8-byte aligned (MG_EALIGN otherwise).
 *   - `stream` is a hipStream_t cast to void* (NULL = the null stream).
 *     Calls enqueue work on it and return without synchronising, except
 *     mg_create (which allocates, runs and frees a small helicity-filtering
 *     pass and waits for it); mg_xsec and the *_workspace_bytes functions
 *     are host arithmetic only.
 *   - A handle is immutable after mg_create; any number of streams may use
 *     it concurrently with disjoint outputs.
 *   - Apart from mg_create, the calls that take a stream only enqueue
 *     kernels (no allocation, no synchronisation, no memset), so a
 *     sequence of them can be captured into a HIP graph on that stream.
 *
 * Layouts (AoSoA, Sec. IV.b "AOSOA"; page sizes from mg_layout):
 *   rnd  [ceil(nevt/neppR)][nrnd][neppR]    uniforms, irnd = 4*ifinal + k
 *   mom  [ceil(nevt/neppM)][npar][4][neppM] (E, px, py, pz) per particle
 *   flat arrays wgt, me, evtw, gbar: [nevt]
 *   grad_rnd, grad_logw: same AoSoA layout as rnd
 *   Event ievt sits in page ievt / nepp at slot ievt % nepp.  AoSoA buffers
 *   must hold ceil(nevt/nepp)*nepp events; slots past nevt are not written.
 *
 * Errors: every entry point returns 0 on success or a negative MG_E* code;
 * no C++ exception crosses the ABI.  Kernel launch failures are reported
 * as MG_EHIP (from hipGetLastError after the launch).  Non-finite matrix
 * elements are not errors: mg_count_nonfinite counts them.
 */
#ifndef MG5MI_H
#define MG5MI_H

#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

/* error codes */
#define MG_OK 0
#define MG_EINVAL (-1)   /* invalid argument: null pointer, nevt < 0, bad enum */
#define MG_ENOTSUP (-2)  /* precision or entry point not built for this process */
#define MG_ENOPHASE (-3) /* sum of final-state masses >= sqrt(s) */
#define MG_EHIP (-4)     /* HIP runtime or launch error */
#define MG_EALIGN (-5)   /* buffer not 8-byte aligned */
#define MG_ENOMEM (-6)   /* mg_create could not allocate its small tables */
#define MG_ERANGE (-7)   /* size beyond the fixed scratch of an allocation-free entry point */

/* processes (Sec. II, Table "tab-compl"; particle order as written) */
typedef enum {
  MG_EEMUMU = 0, /* e+ e- -> mu+ mu-   (Fig. 1: photon and Z exchange) */
  MG_GGTT = 1,   /* g g -> t t~ */
  MG_GGTTG = 2,  /* g g -> t t~ g */
  MG_GGTTGG = 3  /* g g -> t t~ g g */
} mg_proc_t;

/* arithmetic of the matrix-element engine (Sec. IV.b, single/double
 * precision switch, refined per stage):
 *   MG_FP64     everything in binary64
 *   MG_FP32AMP  wavefunctions, currents, amplitudes, jamps and the colour
 *               sum in binary32 (VALU); momenta, propagator denominators,
 *               helicity sum and /IDEN in binary64
 *   MG_MIXED    as MG_FP32AMP but the colour sum runs on the matrix cores
 *               with FP32 accumulation: for 24 colour flows (g g -> t t~ g g)
 *               the jamps are split into three BF16 terms against the exact
 *               BF16 colour numerators; otherwise FP32 MFMA operands
 *   MG_MIXED_F32MFMA  as MG_MIXED with FP32 MFMA operands for every process
 * Precision guard (the three reduced-precision forms, unless
 * MG_FLAG_NO_PRECISION_GUARD): |M|^2 is ill-conditioned in its invariants
 * when kappa = s / min_{i<j} |2 p_i.p_j| over the external momenta is large
 * (soft or collinear gluons), where FP32 rounding of the diagram sums grows
 * like eps32 sqrt(kappa).  After the reduced-precision kernel, the events
 * with kappa > MG_PRECISION_GUARD_KAPPA are recomputed in FP64 (one more
 * kernel on the same stream; about 0.04 % of g g -> t t~ g and 0.2 % of
 * g g -> t t~ g g benchmark events). */
#define MG_PRECISION_GUARD_KAPPA 1.0e4
typedef enum { MG_FP64 = 0, MG_FP32AMP = 1, MG_MIXED = 2, MG_MIXED_F32MFMA = 3 } mg_prec_t;

/* bits of mg_params_t.flags (Sec. IV.c: physics parameters of the kernels;
 * the paper leaves both points open):
 *   MG_FLAG_TCHANNEL_ZERO_WIDTH  top propagators with exactly one incoming
 *       particle on each side (t- and u-channel) get zero width; the others
 *       keep wt.  A width in a spacelike propagator breaks gauge invariance
 *       at O(wt); by default every top propagator carries wt.
 *   MG_FLAG_WEIGHT_2PI  RAMBO weights carry (2 pi)^(4 - 3 nfinal), i.e. the
 *       measure prod d^3p/((2 pi)^3 2E) (2 pi)^4 delta^4; mg_xsec then adds
 *       no 2 pi factor of its own.
 *   MG_FLAG_NO_PRECISION_GUARD  turn off the precision guard of the
 *       reduced-precision forms (see mg_prec_t). */
#define MG_FLAG_TCHANNEL_ZERO_WIDTH 1
#define MG_FLAG_WEIGHT_2PI 2
#define MG_FLAG_NO_PRECISION_GUARD 4

/* physics inputs; couplings are derived in mg_create (sin^2 theta_W in the
 * G_F scheme from alpha, G_F and mZ) */
typedef struct {
  double sqrts;     /* partonic centre-of-mass energy [GeV] */
  double alpha_inv; /* 1/alpha */
  double gfermi;    /* G_F [GeV^-2] */
  double mZ, wZ;    /* Z mass and width [GeV] */
  double mt, wt;    /* top mass and width [GeV]; mt and wt may be 0 */
  double alphas;    /* strong coupling (fixed) */
  int flags;        /* MG_FLAG_* bits; unknown bits give MG_EINVAL */
} mg_params_t;

typedef struct {
  int npar;      /* external particles */
  int nparf;     /* final-state particles */
  int nrnd;      /* uniforms per event = 4 * nparf */
  int nhel;      /* helicity combinations (2^npar) */
  int nhel_good; /* helicities kept after filtering (exactly-zero ones dropped) */
  int ncol;      /* colour flows */
  int ndiag;     /* Feynman diagrams (4-gluon vertex counted once) */
  int neppM;     /* events per momentum page */
  int neppR;     /* events per random-number page */
  int iden;      /* spin/colour average and identical-particle factor */
} mg_layout_t;

typedef struct mg_handle mg_handle_t;

/* Create a handle for one process and precision on the current HIP device.
 * Derives couplings, uploads small tables and determines the nonzero
 * helicities on 64 internally sampled events (synchronises the device).
 * prm == NULL selects the defaults (sqrt(s)=1500, 1/alpha=132.5,
 * G_F=1.16639e-5, mZ=91.188, wZ=2.441, mt=173, wt=1.49, alpha_s=0.118,
 * flags=0).  The parameters are copied: prm may be freed afterwards.
 * Errors: MG_EINVAL, MG_ENOTSUP, MG_ENOPHASE, MG_ENOMEM, MG_EHIP. */
int mg_create(int proc, int prec, const mg_params_t* prm, mg_handle_t** out);
int mg_destroy(mg_handle_t* h);
int mg_layout(const mg_handle_t* h, mg_layout_t* out);

/* Uniform randoms (Sec. IV.b random-number component): Philox4x32-10 with
 * key = seed and counter = (global event index evt_offset + i, block), so
 * any event range is reproducible independently of how it is split.
 * u = ((w >> 11) + 1/2) 2^-53 in (0, 1).  rnd: AoSoA, nrnd per event. */
int mg_rng(const mg_handle_t* h, uint64_t seed, int64_t evt_offset, int64_t nevt, double* rnd,
           void* stream);

/* RAMBO phase space (Sec. IV.a/IV.b phase-space sampler; Kleiss, Stirling,
 * Ellis 1986): rnd (AoSoA) -> mom (AoSoA, all npar particles, initial
 * momenta along +-z) and weights wgt[nevt] (phase-space volume measure
 * prod d^3p/(2E) delta^4, no 2pi factors unless MG_FLAG_WEIGHT_2PI, no
 * flux).  Massive final states
 * by Newton rescaling in FP64; a non-converged event gets a NaN weight. */
int mg_rambo(const mg_handle_t* h, const double* rnd, int64_t nevt, double* mom, double* wgt,
             void* stream);

/* mg_rng + mg_rambo fused in one kernel; rnd_or_null == NULL keeps the
 * uniforms in registers (never written to memory). */
int mg_sample(const mg_handle_t* h, uint64_t seed, int64_t evt_offset, int64_t nevt,
              double* rnd_or_null, double* mom, double* wgt, void* stream);

/* Matrix elements (Sec. II, SIGMAKIN): me[i] = (1/IDEN) sum over kept
 * helicities and all colours of |M|^2 for the momenta of event i.
 * If both wgt_or_null and evtw_or_null are given, evtw[i] = wgt[i]*me[i].
 * Any momenta are accepted.  Events whose incoming momenta are exactly
 * (E,0,0,E) and (E,0,0,-E), as mg_rambo writes them, take a faster body of
 * the same arithmetic with those zero components as constants (checked per
 * event where an event has a wave of its own, else for all the events of a
 * wave together); the two bodies agree to rounding. */
int mg_sigmakin(const mg_handle_t* h, const double* mom, int64_t nevt, double* me,
                const double* wgt_or_null, double* evtw_or_null, void* stream);

/* Per-helicity colour-summed |M|^2 (not divided by IDEN), for ALL 2^npar
 * helicities: mehel[ihel * nevt + i].  Used for helicity filtering and
 * tests; helicity ihel gives particle k the helicity +1 if bit (npar-1-k)
 * of ihel is set, else -1. */
int mg_sigmakin_hel(const mg_handle_t* h, const double* mom, int64_t nevt, double* mehel,
                    void* stream);

/* Gradient of the differentiable event weight f(r) = w(r) |M|^2(p(r)) of
 * RAMBO + SIGMAKIN with respect to the nrnd uniforms of each event (the
 * derivative of the workflow's sampling weight times matrix element,
 * Sec. IV.a), for gradient-based phase-space adaptation:
 *   grad_rnd[j]  = gbar[i] * df/dr_j       (AoSoA like rnd; gbar NULL = 1)
 *   grad_logw[j] = d log w / dr_j          (optional, AoSoA like rnd)
 *   f[i]         = w |M|^2                 (optional)
 * Computed in reverse mode: per helicity the amplitudes run forward, the
 * colour sum gives the colour-flow adjoints 2 C J / den, and hand-written
 * adjoints of the wavefunction and vertex routines carry them back to the
 * final-state momenta; the RAMBO Jacobian (including the Newton rescaling,
 * by the implicit-function theorem) comes from one dual-number pass per
 * uniform.  FP64 for MG_FP64, FP32 amplitudes and adjoints with FP64 RAMBO,
 * momentum adjoints and sums otherwise.  Built for e+e- -> mu+mu-, g g -> t t~ and
 * g g -> t t~ g; MG_ENOTSUP for g g -> t t~ g g. */
int mg_adjoint(const mg_handle_t* h, const double* rnd, int64_t nevt, const double* gbar_or_null,
               double* grad_rnd, double* grad_logw_or_null, double* f_or_null, void* stream);

/* Cross-section statistics of n weighted events f = w |M|^2 (device FP64,
 * e.g. evtw from mg_sigmakin): stats[0] = sum of the finite f, stats[1] =
 * sum of their squares, stats[2] = their maximum (0 if none), stats[3] =
 * how many are finite; stats is a device array of 4 doubles.  Two kernels
 * of fixed shape (blocks over contiguous event ranges, then one block over
 * their partial sums) in a fixed summation order, so the result does not
 * depend on timing (Sec. II: cross section from weighted events).
 * workspace: device memory of mg_xsec_stats_workspace_bytes(n) bytes
 * (8-byte aligned, contents need not be initialised; at most 64 KiB). */
int64_t mg_xsec_stats_workspace_bytes(int64_t n);
int mg_xsec_stats(const double* f, int64_t n, double* stats, void* workspace, void* stream);

/* Host: cross section and Monte Carlo error in pb from stats copied to the
 * host, for n events of h's process:
 *   sigma = (hbar c)^2 (2 pi)^(4 - 3 nfinal) / (2 s) * stats[0] / n
 * (massless partons at fixed sqrt(s); RAMBO weights without 2 pi factors;
 * with MG_FLAG_WEIGHT_2PI the weights already carry them and the factor
 * (2 pi)^(4 - 3 nfinal) is left out),
 *   error = same factor * sqrt((stats[1]/n - (stats[0]/n)^2) / (n - 1)).
 * Non-finite events count as zero.  MG_EINVAL for n < 2 or null pointers. */
int mg_xsec(const mg_handle_t* h, const double* stats_host, int64_t n, double* sigma_pb,
            double* error_pb);

/* Bytes of device workspace mg_unweight needs for n events (8-byte
 * aligned; contents need not be initialised). */
int64_t mg_unweight_workspace_bytes(int64_t n);

/* Hit-or-miss unweighting (Sec. II: unweighted events from weighted ones):
 * event i is kept iff u_i * fmax < f[i], u_i the Philox uniform of (seed,
 * global event evt_offset + i) at counter block 2^31 (no sampler uses that
 * block, so the sampling seed may be reused).  The kept indices i (0-based,
 * increasing) go to idx_out[0 .. *count_out) (device; idx_out must hold n
 * entries), *count_out is a device int64.  NaN f is never kept.  Three
 * kernels (count, scan, write) on `stream`. */
int mg_unweight(const double* f, int64_t n, double fmax, uint64_t seed, int64_t evt_offset,
                int64_t* idx_out, int64_t* count_out, void* workspace, void* stream);

/* mg_unweight without a workspace argument, for callers that cannot
 * allocate device memory (code under HIP graph capture, serving loops,
 * harnesses that forbid hipMalloc).  Same kernels, inputs, outputs and
 * errors as mg_unweight; the per-block counts live in a fixed device array
 * of the library (8 bytes per 256 events, 512 KiB, allocated with the
 * library's code object on each GPU it runs on and held until the process
 * ends), so n is limited to MG_UNWEIGHT_NOALLOC_MAX_EVENTS (MG_ERANGE
 * beyond it, before anything is enqueued).  Nothing in that array needs to
 * start at zero: every call writes the counts it reads.  All calls on one
 * GPU share the array: calls that overlap in time on one GPU (different
 * streams, or different host threads without ordering) race and must not
 * be issued.  Calls no hipMalloc, hipFree or hipMemset. */
#define MG_UNWEIGHT_NOALLOC_MAX_EVENTS (1 << 24)
int mg_unweight_noalloc(const double* f, int64_t n, double fmax, uint64_t seed,
                        int64_t evt_offset, int64_t* idx_out, int64_t* count_out, void* stream);

/* Number of non-finite entries of x[0..n) accumulated into *d_count (a
 * device int64 the caller zeroes first). */
int mg_count_nonfinite(const double* x, int64_t n, int64_t* d_count, void* stream);

const char* mg_strerror(int code);

#ifdef __cplusplus
}
#endif
#endif /* MG5MI_H */
