"""CPU FP64 oracle for the SPME-integrated stochastic Lanczos MBD energy.

TEST INFRASTRUCTURE ONLY. Only the test suite, the smoke check and the
benchmark's CPU-baseline leg may import this package. The GPU library never
imports, links or calls it, and it shares no code with the GPU path.

Everything here is plain PyTorch on the CPU in float64 (PyTorch serves as an
array library with FFT, eigensolvers and automatic differentiation). Atomic
units throughout: bohr, bohr^3, Hartree. The "energy convention" is used for
dipole fields: the field of dipoles d is E = T d with the dipole-dipole energy
d_i^T T_ij d_j, which is the sign that makes the Hamiltonian (eq. ham) and the
generalized-field form of the Lanczos vector l_k (eq. lk3) agree.

Modules:
  params   - parameter rules: Ewald tau from the real cutoff, damping range, grid size
  probes   - SplitMix64 counter generator and normalized Rademacher probes (eq. dds)
  tensors  - dipole tensors: bare, erfc-screened, Fermi-damped, pair field sums
  exact    - converged Ewald sum: dense T^pbc and C, matrix-free exact matvec
  spme     - smooth particle-mesh Ewald reciprocal field (eqs. scaledfractional, spme, dipolarr)
  method   - the SPME-Lanczos matvec l = Omega y + g * E*(g * y) (eqs. lk3, ewalddip)
  lanczos  - Lanczos recurrence, Gauss quadrature and Hutchinson trace (Algorithms 1-2)
  dense    - exact energy from the full spectrum (eqs. plasmonic, plasmonic2)
  replica  - truncated replica sum over periodic images (eq. replica)
  scs      - range-separated self-consistent screening of the polarizabilities (Review section)
  block_lanczos - block Lanczos quadrature over blocks of b probes
"""
