"""FP64 CPU oracle -- TEST INFRASTRUCTURE ONLY.

Plain, slow, obviously correct reference implementations of what the GPU
library computes, written from the paper's definitions:

  fci.py     determinant-basis Hamiltonian and exact (dense) diagonalization
             (the Hamiltonian of real orbitals in second quantization; the
             eigenproblem of the time-independent DMRG equation at full M);
  fock.py    brute-force Jordan-Wigner Fock-space matrices for tiny systems
             (an independent construction used only to pin fci.py);
  mpsvec.py  MPS -> FCI vector, the product-basis maps P_i of the one-site and
             two-site mixed-canonical forms, and the dense explicit effective
             Hamiltonian P^T H P (definition of the site problem, Sec. II A);
  tda.py     the Tamm-Dancoff eigenproblem as Rayleigh-Ritz of H in the MPS
             tangent space with the reference removed (Sec. II C-D);
  firstorder.py  first-order MPS wavefunctions in the mixed gauge (Sec. II B)
             and the TDA sigma P_i^T H Psi1 (Sec. III D, eqs. sigv1, sigv2).
  response.py    frequency-dependent linear response in the tangent space
             (Sec. II B, eqs. realresp, imagresp);
  transition.py  one-particle transition densities of the TDA roots (Sec. VI A);
  rpa.py     DMRG-RPA: the second-order matrix W of the non-redundant
             mixed-canonical parameterization (Sec. II C-D, eq. bmatrix) and
             the RPA roots (eqs. dmrgrpa, reducedrpa).

Only tests/, the smoke check in __graft_entry__.py and the cpu_baseline leg
of bench.py may import this package.  The GPU library never does, and this
package never imports the GPU library.
"""
