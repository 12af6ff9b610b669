/*
 * dgd.h -- C interface of the MI355X library for the ADER discontinuous
 * Galerkin update of 3D seismic waves in the continuum-damage (CDM) rheology
 * (Niu, Gabriel, Wolf, Ulrich, Lyakhovsky, Igel: "A Discontinuous Galerkin
 * Method for Simulating 3D Seismic Wave Propagation in Nonlinear Rock
 * Models", JGR Solid Earth).
 *
 * Conventions used by every call
 * ------------------------------
 * State vector (Section 2.1, Eq. nonlinear hyper pdes), tensor shear strains:
 *     p = 0..9 : eps_xx, eps_yy, eps_zz, eps_xy, eps_yz, eps_zx, v_x, v_y, v_z, alpha
 * Polynomial degree N (the paper's p, Section 2.2); L = (N+1)(N+2)(N+3)/6
 * modes per quantity (Eq. modal dg space).  Modes are the orthonormal Dubiner
 * basis on the reference tetrahedron {xi >= 0, xi1+xi2+xi3 <= 1}:
 *     phi_ijk = sqrt((2i+1)(2i+2j+2)(2i+2j+2k+3)) P_i^(0,0)(a) ((1-b)/2)^i
 *               P_j^(2i+1,0)(b) ((1-c)/2)^(i+j) P_k^(2i+2j+2,0)(c),
 *     a = 2 xi1/(1-xi2-xi3) - 1, b = 2 xi2/(1-xi3) - 1, c = 2 xi3 - 1,
 * ordered by total degree i+j+k, then lexicographically by (i, j, k).
 * Modal state arrays are row-major [element][quantity][mode] in FP64.
 * Tetrahedra (v0, v1, v2, v3) must be positively oriented
 * (det[x1-x0, x2-x0, x3-x0] > 0).  Face f of a tetrahedron is the face
 * opposite local vertex 3-f: f0 = (v0,v2,v1), f1 = (v0,v1,v3),
 * f2 = (v0,v3,v2), f3 = (v1,v2,v3).
 * Volume quadrature: (N+1)^3 collapsed Gauss-Jacobi points.  Both sides of an
 * interior face evaluate the flux at the same physical points: the
 * (N+1)^2-point collapsed face rule laid on the face with its vertices
 * ordered by (periodically identified) global vertex number.
 *
 * Ownership: host arrays passed in are copied and never kept.  Device
 * pointers (on_device != 0) are borrowed for the duration of the call.  The
 * library owns all of its device buffers.  Every kernel runs on the stream
 * given to dgd_create (e.g. PyTorch's current stream); calls return once the
 * work is queued, except where a call says it synchronises.
 *
 * Errors: every call returns a dgd_status; on failure dgd_last_error() gives
 * a message.  A call made before its prerequisites returns DGD_ESTATE.
 */
#ifndef DGD_H
#define DGD_H

#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef struct dgd_handle dgd_handle;

typedef enum {
  DGD_OK = 0,
  DGD_EINVAL = -1,    /* bad argument, shape, mesh or tag */
  DGD_ENOMEM = -2,    /* device or host allocation failed */
  DGD_EDEVICE = -3,   /* HIP runtime error */
  DGD_ESTATE = -4,    /* call out of order (e.g. step before set_state) */
  DGD_ENUMERIC = -5   /* NaN or Inf found in the state */
} dgd_status;

typedef enum {
  DGD_FP64 = 0,       /* every contraction and pointwise law in FP64 */
  DGD_FP32 = 1,       /* FP32 state and arithmetic; alpha kept and updated in FP64 */
  DGD_BF16 = 2        /* as FP32, reference-matrix contractions with BF16 MFMA
                         inputs (FP32 accumulation) */
} dgd_precision;

typedef enum {
  DGD_FACE_INTERIOR = -1,  /* interior or periodic face */
  DGD_BC_FREE = 1,         /* free surface (Appendix A.3, Eq. freeSurface-flux) */
  DGD_BC_ABSORB = 2        /* absorbing (Appendix A.3, Eq. absorbing-flux) */
} dgd_face_tag;

typedef enum { DGD_STF_RICKER = 0, DGD_STF_GAUSSIAN = 1 } dgd_stf_kind;

/* Create a solver of polynomial degree N (1..4; the paper's p of Section 2.2,
 * Eq. modal dg space) in the given precision (dgd_precision).  Builds the
 * reference data of Appendix A on the host: the orthonormal modal basis, the
 * (N+1)^3 volume, (N+1)^2 face and N+1 Gauss-Legendre time quadratures
 * (reading: the paper names the weights but not the rules), the stiffness
 * matrices K^e of Eq. CKIter, the nodal evaluation and projection of Eq. 3rd
 * term and the face trace / lift matrices of Eq. 2nd term.
 * hip_stream: a hipStream_t (NULL = the null stream); every later call queues
 * its kernels there.  Selects the HIP device current at the time of the call.
 * *out receives the handle (NULL on failure).  EINVAL for N outside 1..4 or
 * an unknown precision; ENOMEM / EDEVICE if the reference data cannot be
 * placed on the device. */
dgd_status dgd_create(int N, int precision, void* hip_stream, dgd_handle** out);
/* Waits for the stream and frees every device buffer of the handle (NULL is
 * accepted). */
dgd_status dgd_destroy(dgd_handle* h);
/* Message of the last failed call on h (owned by the handle, valid until the
 * next call on it). */
const char* dgd_last_error(const dgd_handle* h);

/* Number of modes L = (N+1)(N+2)(N+3)/6 (Eq. modal dg space), volume points
 * Q = (N+1)^3, face points Ns = (N+1)^2 and time points Nt = N+1 (the
 * quadratures of Eq. 2nd term / 3rd term and Eq. time-integrated).  Any
 * output pointer may be NULL. */
dgd_status dgd_sizes(const dgd_handle* h, int* L, int* Q, int* Ns, int* Nt);

/* Mesh (Section 2.2: conforming tetrahedral elements with affine maps
 * x = x_0 + J xi; Appendix A.2: neighbour traces across each face).
 * xyz: nv*3 vertex coordinates; tets: ne*4 vertex ids; face_tag: ne*4 tags
 * (dgd_face_tag) in the face numbering above; periodic_map: nv ids (vertex v
 * is identified with vertex periodic_map[v]) or NULL.  Host arrays, copied.
 * Interior faces are matched by their identified vertex triples; each must
 * have exactly one partner.  Computes J^-1, |J|, face normals and |S_f|/|J|
 * in FP64 on the host; allocates the state.  EINVAL on an inverted
 * tetrahedron, an unmatched face, a bad tag or a bad id; the state, material,
 * sources and receivers must be set again afterwards.  Drops a checkpointed
 * run. */
dgd_status dgd_set_mesh(dgd_handle* h, int64_t nv, const double* xyz, int64_t ne,
                        const int64_t* tets, const int8_t* face_tag,
                        const int64_t* periodic_map);

/* Per-element CDM parameters of Eq. cdb-model (host arrays of ne, copied):
 * density rho, Lame lambda0, mu0, third modulus gamma_r, threshold xi0,
 * damage coefficient C_d.  Selects the CDM law for every later step.  EINVAL
 * if rho, mu0 <= 0, or if the clamp alpha_max already set by dgd_set_params
 * makes an effective modulus non-positive (see dgd_set_params).  Drops a
 * checkpointed run kept for dgd_backward. */
dgd_status dgd_set_material(dgd_handle* h, const double* rho, const double* lambda0,
                            const double* mu0, const double* gamma_r,
                            const double* xi0, const double* Cd);

/* Per-element parameters of the internal-variable rheology (Eq. ivm-model,
 * Murnaghan terms off), which then replaces the CDM law in every step:
 *   sigma = (1 - alpha)(lambda0 I1 delta + 2 mu0 eps),
 *   r_alpha = [lambda0 I1^2/2 + mu0 I2 - gamma_b (alpha/(1 - alpha))^2]
 *             / (gamma_b tau_b),
 * alpha clamped to [0, alpha_max] where used; boundary moduli of Eq.
 * effective-ivm.  Host arrays of ne: density rho, Lame lambda0, mu0, storage
 * energy scale gamma_b (Pa), damage time scale tau_b (s).  A later
 * dgd_set_material returns to the CDM law.  The adjoint and dgd_energy are
 * those of the CDM law and return EINVAL under this one.  EINVAL if rho, mu0,
 * gamma_b or tau_b <= 0, or if alpha_max (dgd_set_params) is not below 1.
 * Drops a checkpointed run. */
dgd_status dgd_set_material_ivm(dgd_handle* h, const double* rho, const double* lambda0,
                                const double* mu0, const double* gamma_b, const double* tau_b);

/* Global time step dt (fixed for the run and for its adjoint; the paper uses
 * global time stepping, Section 5.1, and states no CFL rule: the workloads
 * take dt = 0.5 * 2 r_in / ((2N+1) c_p,max)) and the clamp alpha_max applied
 * to alpha wherever it is used (stress, damage rate, tangent, boundary
 * moduli, diagnostics; the stored alpha is never modified).  The paper bounds
 * alpha by 1 (Section 2.1) but gives no clamp; alpha_max is that reading.
 * EINVAL unless dt > 0 and alpha_max >= 0, and, once a material is set, if
 * alpha_max leaves a non-positive effective modulus: under the CDM law
 * mu0 + a xi0 gamma_r - a gamma_r xi/2 > 0 and lambda0 + 2 mu0 + 2 a xi0
 * gamma_r - 4 a gamma_r xi/3 > 0 are required for every element, all
 * a in [0, alpha_max] and xi in [-sqrt 3, sqrt 3] (Eq. effective-cdb);
 * under the IVM law alpha_max < 1 (Eq. ivm-model is singular at alpha = 1).
 * Drops a checkpointed run kept for dgd_backward. */
dgd_status dgd_set_params(dgd_handle* h, double dt, double alpha_max);

/* Physical coordinates x = x_0 + J xi_q of the volume quadrature points of
 * elements [e0, e0+count) (the nodes of the paper's nodal evaluation, Eq. 3rd
 * term, read as the quadrature points), written to the host array
 * [count][Q][3].  Needs the mesh (ESTATE); EINVAL for a range outside
 * [0, ne). */
dgd_status dgd_get_quadrature_points(dgd_handle* h, int64_t e0, int64_t count, double* xyz);

/* Initial condition: L2 projection onto the modes (U_l = sum_q w_q phi_l(xi_q)
 * u(x_q), the projection step of Eq. 3rd term with the orthonormal basis of
 * Eq. modal dg space) of point values vals [count][Q][10] (host, copied;
 * quantity fastest) at the points of dgd_get_quadrature_points, for elements
 * [e0, e0+count); done in FP64 on the device, so large meshes are filled in
 * slices.  Marks the state as set and resets the time to 0.  Synchronises.
 * ESTATE before the mesh; EINVAL for an empty or out-of-range slice. */
dgd_status dgd_set_state_from_points(dgd_handle* h, int64_t e0, int64_t count,
                                     const double* vals);

/* Modal state U (Eq. modal dg space: u = sum_l U_l phi_l per element and
 * quantity) as [ne][10][L] FP64, host (on_device = 0, copied) or device
 * memory (on_device = 1, borrowed for the call) in the layout of the
 * conventions above.  The library converts to its working precision (alpha
 * stays FP64).  set_state resets the time to 0 unless dgd_set_time is called
 * after it; both synchronise.  ESTATE before the mesh (get_state: before a
 * state is set). */
dgd_status dgd_set_state(dgd_handle* h, const double* dofs, int on_device);
dgd_status dgd_get_state(dgd_handle* h, double* dofs, int on_device);  /* synchronises */
/* Point values u(x_q) = sum_l U_l phi_l(xi_q) of the current state at the
 * volume quadrature points (the nodal values of Eq. 3rd term) of elements
 * [e0, e0+count), evaluated in FP64 on the device: vals [count][Q][10],
 * host (on_device = 0) or device memory (on_device = 1, borrowed).
 * Synchronises.  ESTATE before a state is set; EINVAL for a bad range. */
dgd_status dgd_get_point_values(dgd_handle* h, int64_t e0, int64_t count, double* vals,
                                int on_device);

/* Simulation time t_n, which positions the source time functions (R24
 * reading below); advanced by dt per step. */
dgd_status dgd_set_time(dgd_handle* h, double t);
dgd_status dgd_get_time(const dgd_handle* h, double* t);

/* Predictor of the step (Appendix A.1).  DGD_PREDICT_CK (the default): the
 * linearised Cauchy-Kovalevskaya recursion at the cell-averaged Jacobian
 * (Eqs. CKIter, CKIter-ref-matrix, CKIter-ref-source) and its Taylor sums.
 * DGD_PREDICT_PICARD: the discrete Picard iteration the paper's Section 5.1
 * names as the replacement that keeps high order for nonlinear rheologies.
 * Reading (the paper gives no formulas): the element-local evolution that
 * the recursion differentiates, dU/dt = R(U) = -sum_e K^e P G^e(U) + P r(U)
 * in strong form with the pointwise flux and damage rate of the current
 * iterate (no linearisation), is solved on the N+1 Gauss-Legendre time points
 * by `iterations` Picard sweeps of the collocation equations
 * U_z = U^n + dt sum_j Om_zj R(U_j), Om_zj = int_0^tau_z l_j, from U_z = U^n
 * (iterations = 0 means N + 1).  The corrector is unchanged.  The discrete
 * adjoint is that of the Cauchy-Kovalevskaya predictor: its calls return
 * EINVAL under this one.  EINVAL for another kind or iterations < 0.  Drops
 * a checkpointed run. */
typedef enum { DGD_PREDICT_CK = 0, DGD_PREDICT_PICARD = 1 } dgd_predictor;
dgd_status dgd_set_predictor(dgd_handle* h, int kind, int iterations);

/* Clustered local time stepping.  The paper steps every element with one
 * global step and names local time stepping as the missing piece for its
 * nonlinear runs (Section 5.1); it gives no scheme.  Reading (rate-2
 * clusters): element e steps with dt0 2^cluster[e] (cluster 0..7, face
 * neighbours at most one cluster apart, EINVAL otherwise).  A step of cluster
 * c over [t, t + dt_c] predicts its elements at t (Cauchy-Kovalevskaya, the
 * derivatives kept), lets cluster c-1 take its two steps inside, then
 * corrects: faces to clusters >= c take the flux at the cluster's time
 * points with the neighbour's Taylor expansion evaluated there; faces to
 * cluster c-1 take the flux integrals that cluster computed over its two
 * steps; volume and source terms and the update are those of the global
 * step.  Every face flux is computed once, by the finer side, so the wave
 * quantities are conserved across cluster boundaries; one cluster is the
 * global step.  A point source adds its time integral over its element's
 * step after that element's update.
 * dgd_set_clusters: cluster per element (host, ne, copied) and dt0 (> 0);
 * NULL removes the clusters.  ESTATE before the mesh.  Drops a checkpointed
 * run.
 * dgd_make_clusters: proposes clusters from each element's admissible step
 * cfl 2 r_in / ((2N+1) c_p) (intact moduli): dt0 = the smallest, cluster =
 * floor(log2(dt_e / dt0)) capped at max_clusters - 1 and lowered until face
 * neighbours are at most one apart; writes cluster[ne] and *dt0 (host).
 * ESTATE before mesh and material; EINVAL for cfl <= 0 or max_clusters
 * outside 1..8.
 * dgd_step_lts: advances nmacro macro steps of dt0 2^(C-1) (C clusters), the
 * receivers sampled at the end of each.  Synchronises (DGD_ENUMERIC like
 * dgd_synchronize).  ESTATE without clusters or before mesh, material,
 * params and state; EINVAL with the Picard predictor. */
dgd_status dgd_set_clusters(dgd_handle* h, const int32_t* cluster, double dt0);
dgd_status dgd_make_clusters(dgd_handle* h, double cfl, int max_clusters, int32_t* cluster,
                             double* dt0);
dgd_status dgd_step_lts(dgd_handle* h, int64_t nmacro);

/* Point moment-tensor sources.  The paper drives its Gorkha runs with a
 * kinematic finite-fault source (Section 4.1) without printing how it enters
 * the discrete system; the reading used here is the equivalent body force
 * -div(M(t) delta(x - x_s)) in the momentum equation of Eq. nonlinear hyper
 * pdes.  xyz: n*3 positions; M6: n*6 moment tensors (xx,yy,zz,xy,yz,zx) in
 * N m; the moment function is the integral of the moment-rate wavelet
 * (stf_kind DGD_STF_RICKER: Ricker of peak frequency stf_param;
 * DGD_STF_GAUSSIAN: unit Gaussian of width stf_param) started at t_onset.
 * Each step adds the exact time integral of that force, tested with the
 * modes, to the velocity modes of the element holding x_s (the
 * lowest-numbered element whose closed tetrahedron contains it), after the
 * DG update.  Host arrays, copied.  EINVAL for a point outside the mesh, a
 * non-positive stf_param or an unknown stf_kind; ESTATE before mesh and
 * material.  n = 0 removes all sources.  Drops a checkpointed run. */
dgd_status dgd_set_point_sources(dgd_handle* h, int n, const double* xyz,
                                 const double* M6, const double* t_onset,
                                 const double* stf_param, int stf_kind);

/* Receivers: the paper shows velocity seismograms at stations (Section 4)
 * without defining the sampling; here u(x_r) = sum_l U_l phi_l(xi_r) of
 * (v_x, v_y, v_z) is taken from U^{n+1} at the end of every step.  xyz:
 * nrec*3 host positions (copied).  nrec = 0 removes them.  Clears recorded
 * seismograms.  EINVAL for a point outside the mesh; ESTATE before the mesh.
 * Drops a checkpointed run. */
dgd_status dgd_set_receivers(dgd_handle* h, int nrec, const double* xyz);

/* Advance nsteps global time steps t_n -> t_n + dt of the ADER-DG scheme
 * (Appendix A): the linearised Cauchy-Kovalevskaya predictor (A.1, Eqs.
 * CKIter, CKIter-ref-matrix, CKIter-ref-source, taylor_expansion), the
 * volume and damage-source integrals (A.2, Eqs. 3rd term, rhs term), the
 * local Lax-Friedrichs face fluxes (Eq. rusanov-flux, 2nd term) or boundary
 * fluxes (A.3, Eqs. freeSurface-flux, absorbing-flux) and the update of Eq.
 * time-integrated; then point sources and receivers.  Queues the work on the
 * stream.  Returns DGD_ENUMERIC if a step left a non-finite value (the check
 * reads a device flag every check_interval steps, default 64); ESTATE before
 * mesh, material, params and state; EINVAL for nsteps < 0. */
dgd_status dgd_step(dgd_handle* h, int64_t nsteps);
/* How often (in steps, >= 1) dgd_step synchronises to read the non-finite
 * flag; EINVAL for every < 1. */
dgd_status dgd_set_check_interval(dgd_handle* h, int64_t every);
/* Waits for the stream; DGD_ENUMERIC if a step flagged a non-finite value. */
dgd_status dgd_synchronize(dgd_handle* h);

/* Seismograms (the receiver samples above) recorded since the last
 * dgd_set_receivers / dgd_clear_seismograms: out [nrecorded][nrec][3] FP64
 * host, step-major; *nrecorded (may be NULL) receives the number of steps.
 * out may be NULL only when nothing is recorded.  Synchronises. */
dgd_status dgd_get_seismograms(dgd_handle* h, double* out, int64_t* nrecorded);
/* Number of recorded steps (no synchronisation); forget the recorded
 * seismograms (the receivers stay). */
dgd_status dgd_num_seismogram_steps(const dgd_handle* h, int64_t* n);
dgd_status dgd_clear_seismograms(dgd_handle* h);

/* FP64 diagnostics computed on the device from the current state.
 * dgd_energy: the paper plots energies and damage (Section 3) but prints no
 * formula; the reading is the total energy
 *   sum_m |J_m| sum_q w_q (rho |v|^2/2 + W(eps, alpha))
 * with W = lambda0 I1^2/2 + (mu0 + a xi0 gamma_r) I2 - a gamma_r I1 sqrt(I2),
 * the energy whose strain derivative is the stress of Eq. cdb-model (a the
 * clamped alpha).  CDM law only (EINVAL under the IVM law).
 * dgd_wavespeed_change: the shear-wave-speed reduction mapped in Section 4.2,
 * read as the damage-only part per element from the effective shear modulus
 * of Eq. effective-cdb at zero strain: sqrt(max(mu0 + abar xi0 gamma_r, 0)/mu0)
 * - 1 (abar: clamped cell mean of alpha), and sqrt(1 - abar) - 1 under the
 * IVM law (Eq. effective-ivm).  Output: host array of ne.  Both synchronise;
 * ESTATE before state, material and params. */
dgd_status dgd_energy(dgd_handle* h, double* E);
dgd_status dgd_wavespeed_change(dgd_handle* h, double* dcs_over_cs /* ne */);

/* dgd_energy for callers that cannot allocate device memory (code under HIP
 * graph capture, tight serving or monitoring loops, harnesses that forbid
 * hipMalloc): the same energy, computed by the same kernels, but the
 * per-element partial sums live in a static device buffer of the library
 * (2^20 doubles, 8 MiB, held by every GPU the library runs on until the
 * process ends), and the result is written to E, a device pointer to one
 * double (borrowed).  Queued on the solver's stream without synchronising;
 * allocates and frees nothing.  EINVAL for a mesh of more than 2^20
 * elements (use dgd_energy), under the IVM law, or for a NULL pointer;
 * ESTATE before state, material and params.  All calls on one GPU share the
 * buffer: calls that overlap in time on one GPU (other streams or host
 * threads) race and must be serialised by the caller. */
dgd_status dgd_energy_noalloc(dgd_handle* h, double* E /* device, 1 double */);

/* Instrumentation (no passage of the paper: it measures the method).
 * Per-kernel timing with HIP events recorded on the solver's stream around
 * every launch while profiling is on.  dgd_get_kernel_times synchronises,
 * returns the summed milliseconds and launch counts of the kernel classes
 * {0: predictor (Cauchy-Kovalevskaya, time points), 1: face fluxes,
 *  2: sources, 3: receivers, 4: adjoint's predictor recomputation,
 *  5: adjoint faces and their lift, 6: adjoint volume + predictor,
 *  7: adjoint receivers, 8: lift of the face fluxes + update,
 *  9: volume and source integrals}
 * since the last call, and resets them. */
#define DGD_NUM_KERNEL_CLASSES 10
dgd_status dgd_set_profiling(dgd_handle* h, int on);
dgd_status dgd_get_kernel_times(dgd_handle* h, double* ms /* 10 */, int64_t* launches /* 10 */);

/* Intermediate results of the last dgd_step call for testing: the time-point
 * states U(t_n + tau_z dt) of its last step (the Taylor sums of Eq.
 * taylor_expansion at the Gauss-Legendre points tau_z), [ne][Nt][10][L] FP64
 * host.  Synchronises; ESTATE before a state is set. */
dgd_status dgd_get_time_point_states(dgd_handle* h, double* out);

/* ---------------------------------------------------------------------------
 * Discrete adjoint (gradients of a seismogram misfit).
 *
 * The paper computes forward seismograms only; these calls differentiate the
 * discrete step defined by the calls above (Appendix A.1-A.3 with the CDM law
 * of Eq. cdb-model) exactly, with respect to the state and to the per-element
 * shear modulus mu0 and damage coefficient C_d of Eq. cdb-model (gamma_r,
 * lambda0, rho and dt held fixed).  Conventions at the non-smooth points of
 * the step: d clamp(alpha)/d alpha = 1 on the closed interval
 * [0, alpha_max]; the damage rate and the sqrt(I2) terms have zero
 * derivative where they are switched off (xi <= xi0, sqrt(I2) <= 1e-15); at a
 * tie of the two sides' Lax-Friedrichs speeds (Eq. rusanov-flux) each side
 * takes half of the derivative.  Point sources do not depend on the state or
 * on mu0, C_d.  The adjoint arithmetic is FP64 on DGD_FP64 handles and FP32
 * on the others: a DGD_BF16 handle runs its forward (and replayed) steps in
 * its split-BF16 form and differentiates them with the FP32 adjoint of the
 * step, taken at the states of that trajectory (its FP32 operators are
 * packed on the first adjoint call).  CDM law only.
 *
 * dgd_adjoint_step: one reverse step on the device, asynchronous on the
 * solver's stream.  state_n: U^n, device [ne][10][L] FP64 (borrowed).
 * lam: device [ne][10][L] FP64, in: the cotangent lambda^{n+1} of U^{n+1},
 * out: lambda^n = (dU^{n+1}/dU^n)^T (lambda^{n+1} + R^T dJ_dseis_n).
 * dJ_dseis_n: device [nrec][3] FP64 cotangent of the receiver samples taken
 * from U^{n+1}, or NULL.  grad_mu0, grad_cd: device [ne] FP64 to which the
 * step's (dU^{n+1}/dmu0_e)^T (...) and (dU^{n+1}/dC_d,e)^T (...) are ADDED,
 * or NULL.  Does not change the solver's state or time.  Device buffers of
 * the adjoint are allocated on the first call and kept.  ESTATE before mesh,
 * material and params.
 *
 * dgd_adjoint_step_host: the same product at the solver's current state for
 * tests, with host arrays: lam_next, lam_out [ne][10][L]; grad_mu0, grad_cd
 * [ne] overwritten with this step's contribution (either may be NULL); no
 * receiver term.  Synchronises.
 *
 * dgd_forward_checkpointed: runs nsteps steps from the current state like
 * dgd_step (seismograms recorded as usual), keeping a device copy of the
 * state every `every` steps (ceil(nsteps/every) copies) for dgd_backward.
 * Synchronises (and reports DGD_ENUMERIC like dgd_synchronize).
 *
 * dgd_backward: gradients of a scalar misfit J(seismograms) of the last
 * checkpointed run, given dl_dseis = dJ/dseismograms [nsteps][nrec][3] FP64
 * host (the seismograms that run recorded, in recording order; may be NULL
 * without receivers).  Each segment of `every` steps is recomputed from its
 * checkpoint and then reversed.  Outputs (host, overwritten):
 * grad_mu0[ne], grad_cd[ne], and if grad_u0 is not NULL dJ/dU^0 as
 * [ne][10][L].  The current state, time and seismograms are left as the
 * forward run left them.  The checkpoints are kept until the next
 * dgd_forward_checkpointed, dgd_release_tape or any call that changes the
 * problem (dgd_set_mesh, dgd_set_material, dgd_set_material_ivm,
 * dgd_set_params, dgd_set_point_sources, dgd_set_receivers); without them
 * dgd_backward returns DGD_ESTATE.  Synchronises.
 *
 * dgd_tape_id: identifies the kept checkpointed run (a counter that grows
 * with each dgd_forward_checkpointed), 0 when there is none, so that a caller
 * can check that dgd_backward differentiates the run it means.
 */
dgd_status dgd_adjoint_step(dgd_handle* h, const double* state_n, double* lam,
                            const double* dJ_dseis_n, double* grad_mu0, double* grad_cd);
dgd_status dgd_adjoint_step_host(dgd_handle* h, const double* lam_next, double* lam_out,
                                 double* grad_mu0, double* grad_cd);
dgd_status dgd_forward_checkpointed(dgd_handle* h, int64_t nsteps, int64_t every);
dgd_status dgd_backward(dgd_handle* h, const double* dl_dseis, double* grad_mu0, double* grad_cd,
                        double* grad_u0);
dgd_status dgd_tape_id(const dgd_handle* h, int64_t* id);
dgd_status dgd_release_tape(dgd_handle* h);

#ifdef __cplusplus
}
#endif
#endif /* DGD_H */
