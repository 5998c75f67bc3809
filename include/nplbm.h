/*
 * nplbm.h -- C ABI of the MI355X (gfx950) implementation of the N-phase
 * phase-field lattice Boltzmann model of Yuan, Liang, Chai & Shi
 * (arXiv:1904.12553).
 *
 * One domain = one 2-D D2Q9 lattice holding (N-1) Cahn-Hilliard
 * distributions h^i_k (eq:N24), one Navier-Stokes distribution g_k (eq:24)
 * and the previous-step phi_i, u needed by the source term (eq:N27).
 * nplbm_step advances all of them by one time step per call-count, fully on
 * the GPU; the host only sees parameters going in and macroscopic fields
 * (c_i, u, p) coming out.
 *
 * Conventions shared by every call:
 *   - lattice units: dx = dt = 1, c_s^2 = 1/3 (Sec. 3.1);
 *   - a field array is row-major with x fastest: element (x, y) of field f
 *     is at f[(f * ny + y) * nx + x];
 *   - host pointers are caller-owned and only read/written during the call;
 *   - every call returns NPLBM_OK (0) or a negative error code, and sets a
 *     thread-local message readable with nplbm_last_error();
 *   - calls on one domain must not overlap (a domain is not thread-safe);
 *     calls on different domains may run from different threads.
 */
#ifndef NPLBM_H
#define NPLBM_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

#define NPLBM_MAX_PHASES 8

enum {
  NPLBM_OK = 0,
  NPLBM_EINVAL = -1,   /* a parameter or argument is out of range        */
  NPLBM_ENOTSPD = -2,  /* eq:N14 has no SPD solution lambda for this sigma */
  NPLBM_ENOMEM = -3,   /* device or host allocation failed / too small   */
  NPLBM_EDEVICE = -4,  /* a HIP runtime call failed                       */
  NPLBM_ETOOBIG = -5,  /* request larger than the whole serving budget    */
  NPLBM_ESTATE = -6,   /* call not valid in the object's current state    */
  NPLBM_ENOTFOUND = -7 /* unknown ticket                                  */
};

/*
 * Physical and numerical parameters of one domain (the problem statement of
 * Sec. 2: N constant-density, constant-viscosity phases with pairwise
 * surface tensions; eq:N13c/eq:N30 mobility; eq:N36 energy scale).
 *
 *   N               number of phases, 2..NPLBM_MAX_PHASES
 *   nx, ny          lattice size, each >= 4
 *   wall_y          0: periodic in y; 1: halfway bounce-back walls below
 *                   row 0 and above row ny-1 (Sec. 4.2). x is periodic.
 *   precision       32 or 64: storage type of the state and arithmetic
 *                   type of the stencils and CH collisions; the NS
 *                   collision is evaluated in FP64 arithmetic in both
 *                   (FP32 rounding there biases the momentum of moving
 *                   droplets).  FP32 stores deviations from the rest state.
 *   grad_scheme     first derivatives of phi_i and C_i: 0 = isotropic
 *                   central stencil of eq:N31a; 1 = isotropic mixed
 *                   stencil of eq:N40 (Sec. 4.4) with its two-hop term
 *                   -zeta(x + 2 c_i) (printed with a + sign, which would make
 *                   it twice the gradient).  The Laplacian is eq:N31b in
 *                   both.  Other values: NPLBM_EINVAL.
 *   force_form      total-force distribution of the NS equation: 0 = G_k of
 *                   eq:N20_1 (the J~ u / (tau_g - 1/2) term in its second
 *                   moment); 1 = the alternative of Remark 1 (Sec. 3.1): G_k
 *                   without that term and F = -div(J~ u) + F_s + G, component
 *                   a of the divergence being sum_b d_b (J~_b u_a) by the
 *                   eq:N31a stencil, with J~ of the current step and u of
 *                   the previous step (the stored u of eq:N27).  Built with
 *                   grad_scheme 0 only; other values or combinations:
 *                   NPLBM_EINVAL.
 *   sigma           N*N row-major pairwise tensions sigma_kl > 0, symmetric;
 *                   the diagonal is ignored
 *   rho, mu         N densities rho~_k > 0 and dynamic viscosities mu~_k > 0
 *   mobility        N-1 Cahn-Hilliard mobilities m_i > 0 (eq:N13c)
 *   tau_phi         N-1 Cahn-Hilliard relaxation times tau_i > 1/2 (eq:N24)
 *   interface_width W > 0; the interface scale is eta = W / (2 sqrt 2), so
 *                   the equilibrium profile is 1/2 + 1/2 tanh(2 x / W)
 *   gx, gy          body-force acceleration, G = rho (gx, gy) (Sec. 2)
 *   gz              z component of the body-force acceleration (3-D only)
 *   nz              0 or 1: a 2-D domain on the D2Q9 lattice; >= 4: a 3-D
 *                   domain of nx x ny x nz nodes on the D3Q15 lattice of
 *                   Sec. 3.1 (x and y periodic; N <= 5, grad_scheme 0,
 *                   force_form 0 and wall_y 0 are required, else
 *                   NPLBM_EINVAL).  Fields of a 3-D domain are
 *                   f[((f * nz + z) * ny + y) * nx + x] and u has three
 *                   components.
 *   wall_z          3-D only: 0 periodic in z; 1 halfway bounce-back walls
 *                   below plane 0 and above plane nz-1
 *
 * Derived on the host (Sec. 2 and eq:N36): beta^2 = 3 sqrt(2) sigma_min eta,
 * lambda_ij from eq:N14-N16, eta_i = m_i / (c_s^2 (tau_i - 1/2)) (eq:N30);
 * the NS relaxation time varies per node, tau_g = 1/2 + mu / (rho c_s^2)
 * with mu = sum_k mu~_k c_k (eq:N21_1).
 */
typedef struct nplbm_params {
  int32_t N, nx, ny;
  int32_t wall_y;
  int32_t precision;
  int32_t grad_scheme;
  int32_t force_form;
  const double *sigma;
  const double *rho;
  const double *mu;
  const double *mobility;
  const double *tau_phi;
  double interface_width;
  double gx, gy;
  double gz;
  int32_t nz;
  int32_t wall_z;
} nplbm_params;

typedef struct nplbm_domain nplbm_domain;

/* Message of the last error raised on this thread ("" if none). */
const char *nplbm_last_error(void);

/*
 * Host-only validation of a parameter set (no GPU needed).  Checks the
 * ranges above and solves eq:N14 for lambda; returns NPLBM_EINVAL or
 * NPLBM_ENOTSPD on failure.  On success, if non-NULL: lambda_out receives
 * the (N-1)x(N-1) row-major mixing matrix, beta2_out receives beta^2 and
 * K_out receives beta^2 / eta^2.
 */
int nplbm_validate(const nplbm_params *p, double *lambda_out, double *beta2_out,
                   double *K_out);

/* Host-only: bytes of device memory nplbm_create needs for these
 * parameters (0 if they are invalid). */
size_t nplbm_footprint(const nplbm_params *p);

/*
 * Create a domain on the current HIP device.
 *   stream        hipStream_t (as void*) every kernel of this domain runs
 *                 on; NULL = the null stream.  All later calls enqueue on it.
 *   device_mem    optional caller-owned device buffer of at least
 *                 nplbm_footprint(p) bytes, 256-byte aligned; the domain
 *                 keeps using it until nplbm_destroy and never frees it.
 *                 NULL = the library allocates (and frees) its own memory.
 *   device_bytes  size of device_mem (ignored when device_mem is NULL)
 * The state is undefined until nplbm_set_fields.  Errors: NPLBM_EINVAL,
 * NPLBM_ENOTSPD, NPLBM_ENOMEM (device_bytes too small or allocation
 * failed), NPLBM_EDEVICE.
 */
int nplbm_create(const nplbm_params *p, void *stream, void *device_mem,
                 size_t device_bytes, nplbm_domain **out);

/*
 * Initial state from host volume fractions c (N fields, values with
 * |sum_k c_k - 1| <= 1e-9 at every node) and velocity u (2 fields, or NULL
 * for rest): phi_i = (rho~_i c_i - rho~_N c_N - (rho~_i - rho~_N)/2) /
 * ((rho~_i + rho~_N)/2) (eq:N12 inverted), p = 0, g = g^eq (eq:25),
 * h = h^eq (eq:N25), previous (phi, u) = current so that the first source
 * term of eq:N26 is zero.  Resets the time to 0.  Synchronous.
 */
int nplbm_set_fields(nplbm_domain *d, const double *c, const double *u);

/*
 * Advance nsteps >= 0 time steps: for every node, stream (pull),
 * phi_i by eq:N28, closure eq:N18, C_i by eq:N18 with the eq:N31b Laplacian,
 * gradients by eq:N31a, F and J~, u by eq:N22_1, p by eq:N23, NS collision
 * eq:24 with eq:25 and eq:N20_1, CH collisions eq:N24 with eq:N25-N27.
 * Asynchronous: returns once the work is enqueued on the domain's stream.
 */
int nplbm_step(nplbm_domain *d, int64_t nsteps);

/* Macroscopic fields of the current state (the moments above, no
 * collision), converted to FP64, copied to host arrays of N, 2 and 1
 * fields.  Synchronous. */
int nplbm_get_c(nplbm_domain *d, double *c);
int nplbm_get_u(nplbm_domain *d, double *u);
int nplbm_get_p(nplbm_domain *d, double *p);

/*
 * Conservation diagnostics of the current state, reduced on the GPU in
 * FP64 (any output may be NULL): mass_out[k] = sum_x c_k (N values),
 * *max_sum_dev = max_x |sum_k c_k - 1|, *nonfinite = number of nodes with a
 * non-finite c_k.  Synchronous.
 */
int nplbm_diagnostics(nplbm_domain *d, double *mass_out, double *max_sum_dev,
                      int64_t *nonfinite);

/*
 * For callers that cannot allocate device memory or synchronise (code under
 * HIP graph capture, tight serving loops, harnesses that forbid hipMalloc):
 * the conservation diagnostics of nplbm_diagnostics, written to device
 * memory and allocating nothing.
 *   out_dev  caller-owned device buffer of N + 2 doubles: sum_x c_k for
 *            k = 0..N-1, then max_x |sum_k c_k - 1|, then the number of
 *            nodes with a non-finite c_k (as a double).
 * Asynchronous on the domain's stream; enqueues kernels only (the FP64
 * read-back into the domain's own read-back planes, then the reduction) and
 * reads the state current at enqueue time.  The reduction's partial records
 * live in a static device array of the library (1024 x 10 doubles + 16, about
 * 82 KB, held on each GPU it runs on until the process ends) instead of the
 * domain's allocation: every call on one GPU shares it, so calls that
 * overlap on one GPU (other streams or threads) race.  Results equal
 * nplbm_diagnostics' bitwise (same kernels, same block count).  Errors:
 * NPLBM_EINVAL (NULL argument, the domain belongs to another device than
 * the current one, or a reduction larger than the static array, which the
 * 1024-block cap rules out), NPLBM_ESTATE, NPLBM_EDEVICE.
 */
int nplbm_diagnostics_noalloc(nplbm_domain *d, double *out_dev);

/*
 * Laplace pressure jump of a droplet centred at (xc, yc) (Sec. 4.1): the
 * mean of p over nodes with distance <= r_in minus the mean over nodes with
 * distance >= r_out (plain Euclidean distance), reduced in FP64 on the GPU.
 * Synchronous.
 */
int nplbm_laplace(nplbm_domain *d, double xc, double yc, double r_in,
                  double r_out, double *dp);

/*
 * The same for a 3-D domain and a spherical droplet centred at
 * (xc, yc, zc) (Sec. 4.1's test with the jump 2 sigma / R of a sphere).
 * NPLBM_EINVAL on a 2-D domain.  Synchronous.
 */
int nplbm_laplace3(nplbm_domain *d, double xc, double yc, double zc, double r_in,
                   double r_out, double *dp);

/* Number of steps taken since nplbm_set_fields, or -1 for NULL. */
int64_t nplbm_time(const nplbm_domain *d);

/* Wait for all work enqueued on the domain's stream. */
int nplbm_sync(nplbm_domain *d);

/* Release the domain (NULL is accepted). */
void nplbm_destroy(nplbm_domain *d);

/*
 * Raw state in the library's storage order, for checkpoint / resume:
 * nplbm_state_bytes gives the size; get copies device -> host, set copies
 * host -> device and restores the time step.  Resuming from a saved state
 * is bitwise identical to an uninterrupted run.  Synchronous.
 */
size_t nplbm_state_bytes(const nplbm_domain *d);
int nplbm_get_state(nplbm_domain *d, void *host, int64_t *time_out);
int nplbm_set_state(nplbm_domain *d, const void *host, int64_t time);

/*
 * Measurement helper: copy nbytes bytes between two device buffers with a
 * plain vectorised copy kernel on the given stream (asynchronous).  Used to
 * calibrate HBM traffic counters and measure copy bandwidth.
 */
int nplbm_device_copy(void *dst, const void *src, size_t nbytes, void *stream);

/* ---------------------------------------------------------------------
 * Serving: continuous batching of many small domains on one GPU.
 *
 * A server owns a device-memory budget and a set of resident domains.
 * nplbm_submit queues a request (parameters, initial fields, number of
 * steps); nplbm_server_pump admits queued requests whose footprint fits the
 * free budget and the slot limit, initialises them, then runs one quantum:
 * `quantum` steps of every resident domain packed into the same kernel
 * launches (captured once per resident set as a HIP graph); domains that
 * reach their step count retire, their c, u, p are read back and their
 * memory is released.  Results are bitwise identical to running the same
 * request alone with nplbm_create / nplbm_step.
 * --------------------------------------------------------------------- */
typedef struct nplbm_server nplbm_server;

/* hbm_budget: bytes of device memory the server may hold for domains;
 * max_slots: maximum resident domains; quantum: steps per pump (>= 1). */
int nplbm_server_create(size_t hbm_budget, int32_t max_slots, int32_t quantum,
                        void *stream, nplbm_server **out);

/* Queue a request.  c (N fields) and u (2 fields or NULL) are copied before
 * return.  *ticket receives an id.  Errors: NPLBM_EINVAL, NPLBM_ENOTSPD,
 * NPLBM_ETOOBIG (footprint above the whole budget).  Thread-safe. */
int nplbm_submit(nplbm_server *s, const nplbm_params *p, const double *c,
                 const double *u, int64_t nsteps, uint64_t *ticket);

/* Admit what fits, run one quantum, retire finished requests.
 * *active_out (may be NULL) = resident domains after the pump. */
int nplbm_server_pump(nplbm_server *s, int32_t *active_out);

/* *state: 0 queued, 1 resident, 2 done, 3 failed. Thread-safe. */
int nplbm_poll(nplbm_server *s, uint64_t ticket, int32_t *state);

/* Results of a finished request (host arrays of N, 2 and 1 fields, any may
 * be NULL) and its timing: seconds from submit to admission and from submit
 * to completion.  The request is forgotten afterwards.  A failed request
 * (state 3: its admission or read-back raised an error) is forgotten too,
 * and the call returns that error with its message.  NPLBM_ESTATE (the
 * ticket stays valid) while the request is queued or resident;
 * NPLBM_ENOTFOUND for an unknown or already collected ticket. */
int nplbm_result(nplbm_server *s, uint64_t ticket, double *c, double *u,
                 double *p, double *admit_s, double *done_s);

/* Aggregate statistics since creation (any output may be NULL):
 *   p50_s, p99_s  median and 99th percentile of the time from nplbm_submit
 *                 to completion over every request completed so far
 *                 (linear interpolation between order statistics; 0 if
 *                 none);
 *   mlups         node updates done / (last completion - first submission)
 *                 / 1e6: aggregate throughput of the whole stream;
 *   node_updates  node updates done, busy_s seconds spent inside
 *                 nplbm_server_pump, completed requests finished.
 * Thread-safe. */
int nplbm_server_stats(nplbm_server *s, double *p50_s, double *p99_s, double *mlups,
                       double *node_updates, double *busy_s, int64_t *completed);

void nplbm_server_destroy(nplbm_server *s);

#ifdef __cplusplus
}
#endif

#endif /* NPLBM_H */
