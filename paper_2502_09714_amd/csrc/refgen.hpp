// Host-side generator of the reference-element data (FP64).
//
// Quadrature: collapsed (Stroud conical product) Gauss-Jacobi rules with N+1
// points per direction -- nodes by Newton iteration on the three-term Jacobi
// recurrence, weights 2^(a+1) / ((1 - t^2) P_n'(t)^2) for weight (1-t)^a.
// Basis: orthonormal Dubiner polynomials evaluated through collapsed
// coordinates with the Jacobi recurrence, gradients by the chain rule.
// Matrices (paper, Appendix A):
//   V[q][l]    = phi_l(xi_q)                       nodal evaluation
//   Pw[l][q]   = w_q phi_l(xi_q)                   L2 projection (mass = I)
//   Sw[e][l][q]= w_q dphi_l/dxi_e(xi_q)            volume stiffness (Eq. 3rd term)
//   K[e][k][l] = int phi_k dphi_l/dxi_e            Cauchy-Kovalevskaya (Eq. CKIter-ref-matrix)
//   F[f][s][i][l] = phi_l(xi^f(eta_i permuted by s)) face traces, s = permutation of
//                   the face vertices that puts the rule on the face in global order
//   beta[i], tau[z], gamma[z]                      face and time weights
//   KP[e][k][q] = sum_l K[e][k][l] Pw[l][q]        strong-form derivative of a projected field
//   Om[z][j]   = int_0^tau_z l_j(s) ds             time integration of the Lagrange
//                                                  polynomials of the time points
#pragma once
#include <vector>

namespace dgd {

struct RefData {
  int N = 0, L = 0, Q = 0, Ns = 0, Nt = 0;
  std::vector<double> xq;     // Q*3 reference points
  std::vector<double> wq;     // Q
  std::vector<double> eta;    // Ns*2 face rule points
  std::vector<double> beta;   // Ns (sum 1)
  std::vector<double> tau;    // Nt on [0,1]
  std::vector<double> gamma;  // Nt (sum 1)
  std::vector<double> V;      // Q*L
  std::vector<double> Pw;     // L*Q
  std::vector<double> Sw;     // 3*L*Q
  std::vector<double> K;      // 3*L*L
  std::vector<double> KP;     // 3*L*Q
  std::vector<double> Om;     // Nt*Nt
  std::vector<double> F;      // 4*6*Ns*L
  std::vector<int> deg;       // L total degrees
};

// Permutations of three face slots, index s -> perm[s][j] = slot receiving the
// j-th smallest global vertex.
extern const int kPerm3[6][3];
extern const int kFaceVerts[4][3];

int n_modes(int N);
void gauss_jacobi(int n, double alpha, std::vector<double>& t, std::vector<double>& w);
void basis_eval(int N, const double xi[3], double* phi, double* dphi /* 3*L or null */);
RefData build_reference(int N);

}  // namespace dgd
