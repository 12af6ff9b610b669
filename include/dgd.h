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

/* Create a solver of polynomial degree N (1..4) in the given precision.
 * hip_stream: a hipStream_t (NULL = the null stream).  Selects the current
 * HIP device at the time of the call. */
dgd_status dgd_create(int N, int precision, void* hip_stream, dgd_handle** out);
dgd_status dgd_destroy(dgd_handle* h);
const char* dgd_last_error(const dgd_handle* h);

/* Number of modes L, volume points Q, face points Ns and time points Nt. */
dgd_status dgd_sizes(const dgd_handle* h, int* L, int* Q, int* Ns, int* Nt);

/* Mesh (Section 2.2: tetrahedral elements, affine maps).
 * xyz: nv*3 vertex coordinates; tets: ne*4 vertex ids; face_tag: ne*4 tags
 * (dgd_face_tag) in the face numbering above; periodic_map: nv ids (vertex v
 * is identified with vertex periodic_map[v]) or NULL.  Interior faces are
 * matched by their identified vertex triples; each must have exactly one
 * partner.  EINVAL on an inverted tetrahedron, an unmatched face or a bad id. */
dgd_status dgd_set_mesh(dgd_handle* h, int64_t nv, const double* xyz, int64_t ne,
                        const int64_t* tets, const int8_t* face_tag,
                        const int64_t* periodic_map);

/* Per-element CDM parameters of Eq. cdb-model (host arrays of ne):
 * density rho, Lame lambda0, mu0, third modulus gamma_r, threshold xi0,
 * damage coefficient C_d.  EINVAL if rho, mu0 <= 0. */
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
 * gamma_b or tau_b <= 0. */
dgd_status dgd_set_material_ivm(dgd_handle* h, const double* rho, const double* lambda0,
                                const double* mu0, const double* gamma_b, const double* tau_b);

/* Global time step dt (fixed for the run) and the clamp alpha_max applied to
 * alpha wherever it is used (the stored alpha is never modified). */
dgd_status dgd_set_params(dgd_handle* h, double dt, double alpha_max);

/* Physical coordinates of the volume quadrature points of elements
 * [e0, e0+count), host array [count][Q][3].  Needs the mesh. */
dgd_status dgd_get_quadrature_points(dgd_handle* h, int64_t e0, int64_t count, double* xyz);

/* L2 projection onto the modes of point values vals [count][Q][10] (host)
 * for elements [e0, e0+count), done on the device (large meshes are filled
 * in slices).  Marks the state as set and resets the time to 0. */
dgd_status dgd_set_state_from_points(dgd_handle* h, int64_t e0, int64_t count,
                                     const double* vals);

/* Modal state [ne][10][L] FP64, host (on_device = 0) or device memory.
 * set_state resets the time to 0 unless dgd_set_time is called after it. */
dgd_status dgd_set_state(dgd_handle* h, const double* dofs, int on_device);
dgd_status dgd_get_state(dgd_handle* h, double* dofs, int on_device);  /* synchronises */
dgd_status dgd_set_time(dgd_handle* h, double t);
dgd_status dgd_get_time(const dgd_handle* h, double* t);

/* Point moment-tensor sources.  M6: n*6 moment tensors (xx,yy,zz,xy,yz,zx)
 * in N m; the moment function is the integral of the moment-rate wavelet
 * (Ricker of peak frequency stf_param, or unit Gaussian of width stf_param)
 * started at t_onset.  Each step adds the exact time integral of the force
 * -div(M delta(x - x_s)) to the velocity modes of the element holding x_s
 * (the lowest-numbered element whose closed tetrahedron contains it).
 * EINVAL for a point outside the mesh.  n = 0 removes all sources. */
dgd_status dgd_set_point_sources(dgd_handle* h, int n, const double* xyz,
                                 const double* M6, const double* t_onset,
                                 const double* stf_param, int stf_kind);

/* Receivers sampling (v_x, v_y, v_z) at the end of every step.  nrec = 0
 * removes them.  Clears recorded seismograms. */
dgd_status dgd_set_receivers(dgd_handle* h, int nrec, const double* xyz);

/* Advance nsteps global time steps (Appendix A: prediction + correction).
 * Queues the work on the stream; returns DGD_ENUMERIC if a previous step
 * left a non-finite value (the check reads a device flag every
 * check_interval steps, default 64, see dgd_set_check_interval). */
dgd_status dgd_step(dgd_handle* h, int64_t nsteps);
dgd_status dgd_set_check_interval(dgd_handle* h, int64_t every);
dgd_status dgd_synchronize(dgd_handle* h);   /* waits; DGD_ENUMERIC if flagged */

/* Seismograms recorded since the last dgd_set_receivers / dgd_clear_seismograms:
 * out [nrecorded][nrec][3] FP64 host; *nrecorded may be NULL.  Synchronises. */
dgd_status dgd_get_seismograms(dgd_handle* h, double* out, int64_t* nrecorded);
dgd_status dgd_num_seismogram_steps(const dgd_handle* h, int64_t* n);
dgd_status dgd_clear_seismograms(dgd_handle* h);

/* FP64 diagnostics computed on the device from the current state:
 * total energy  sum_m |J| sum_q w_q (rho |v|^2/2 + W(eps, alpha)) with the
 * CDM energy W whose strain derivative is the stress of Eq. cdb-model, and
 * the damage-only shear-wave-speed change per element
 * sqrt(max(mu0 + abar xi0 gamma_r, 0)/mu0) - 1 (abar: clamped cell mean of
 * alpha), sqrt(1 - abar) - 1 under the IVM law.  Both synchronise. */
dgd_status dgd_energy(dgd_handle* h, double* E);
dgd_status dgd_wavespeed_change(dgd_handle* h, double* dcs_over_cs /* ne */);

/* Per-kernel timing with HIP events recorded on the solver's stream around
 * every launch while profiling is on.  dgd_get_kernel_times synchronises,
 * returns the summed milliseconds and launch counts of the kernel classes
 * {0: predictor + volume, 1: face fluxes, 2: sources, 3: receivers,
 *  4: adjoint's predictor recomputation, 5: adjoint faces and their lift, 6: adjoint
 *  volume + predictor, 7: adjoint receivers, 8: lift of the face fluxes +
 *  update}
 * since the last call, and resets them. */
#define DGD_NUM_KERNEL_CLASSES 9
dgd_status dgd_set_profiling(dgd_handle* h, int on);
dgd_status dgd_get_kernel_times(dgd_handle* h, double* ms /* 9 */, int64_t* launches /* 9 */);

/* Intermediate results of the last dgd_step call for testing: the time-point
 * states U(t_n + tau_z dt) of its last step, [ne][Nt][10][L] FP64 host.
 * Synchronises. */
dgd_status dgd_get_time_point_states(dgd_handle* h, double* out);

/* ---------------------------------------------------------------------------
 * Discrete adjoint (gradients of a seismogram misfit).
 *
 * The paper computes forward seismograms only; these calls differentiate the
 * discrete step defined by the calls above (Appendix A.1-A.3 with the CDM law
 * of Eq. cdb-model) exactly, with respect to the state and to the per-element
 * shear modulus mu0 and damage coefficient C_d of Eq. cdb-model.  Conventions
 * at the non-smooth points of the step: d clamp(alpha)/d alpha = 1 on the
 * closed interval [0, alpha_max]; the damage rate and the sqrt(I2) terms have
 * zero derivative where they are switched off (xi <= xi0, sqrt(I2) <= 1e-15);
 * at a tie of the two sides' Lax-Friedrichs speeds (Eq. rusanov-flux) each
 * side takes half of the derivative.  Point sources do not depend on the
 * state or on mu0, C_d.  Runs in FP64 or FP32 (DGD_BF16 handles return
 * DGD_EINVAL); the adjoint arithmetic has the handle's precision.
 *
 * dgd_adjoint_step: one step's vector-Jacobian product at the current state
 * U^n (left unchanged):  lam_out = (dU^{n+1}/dU^n)^T lam_next,
 * grad_mu0[e] = lam_next . dU^{n+1}/dmu0_e, grad_cd[e] likewise (both may be
 * NULL).  lam_next, lam_out: [ne][10][L] FP64 host; gradients: [ne] FP64
 * host.  Synchronises.
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
 * forward run left them; the checkpoints are kept until the next
 * dgd_forward_checkpointed or dgd_release_tape.  Synchronises.
 */
dgd_status dgd_adjoint_step(dgd_handle* h, const double* lam_next, double* lam_out,
                            double* grad_mu0, double* grad_cd);
dgd_status dgd_forward_checkpointed(dgd_handle* h, int64_t nsteps, int64_t every);
dgd_status dgd_backward(dgd_handle* h, const double* dl_dseis, double* grad_mu0, double* grad_cd,
                        double* grad_u0);
dgd_status dgd_release_tape(dgd_handle* h);

#ifdef __cplusplus
}
#endif
#endif /* DGD_H */
