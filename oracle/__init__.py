"""FP64 CPU oracle for the ADER-DG update of the continuum-damage (CDM) rheology.

TEST INFRASTRUCTURE ONLY.  This package is the plain, slow, obviously correct
reference that the GPU library is checked against.  Only ``tests/``,
``__graft_entry__.smoke()`` and the ``cpu_baseline`` leg of ``bench.py`` may
import it; the product path (``paper_2502_09714_amd``) never does, and this
package never imports the product path.  The two share no code: the oracle has
its own basis, quadrature, reference matrices, connectivity, constitutive law,
fluxes and time stepping.  Only the seeded input generators in ``workloads``
serve both.

Everything follows the paper (Niu et al., "A Discontinuous Galerkin Method for
Simulating 3D Seismic Wave Propagation in Nonlinear Rock Models", JGR Solid
Earth), Section 2 and Appendix A, in its order and notation, computed with
PyTorch CPU float64 tensors.  Each function cites the passage it follows.
Parity pins (tests/test_oracle_*.py) tie every function to something other
than itself: exact integrals, closed forms, printed matrices, invariants.

Module map
  basis        Dubiner orthonormal basis on the reference tetrahedron
  quadrature   collapsed-coordinate Gauss-Jacobi rules (volume, face, time)
  refmat       reference matrices M, K^e, projection, traces, lift
  mesh         geometry, connectivity and neighbour point matching
  cdm          CDM stress, damage rate, flux, Jacobian, LLF constant
  ivm          the same for the internal-variable law (Eq. ivm-model)
  boundary     free-surface and absorbing boundary fluxes
  step         predictor (linearised Cauchy-Kovalevskaya) + corrector
  sources      point moment-tensor sources and receivers
  diagnostics  energy and shear-wave-speed change
  adjoint      gradients of a step and of a seismogram misfit (autograd)
"""
