"""FP64 CPU oracle for the differentiable PME of charges and dipoles.

TEST INFRASTRUCTURE ONLY.  Nothing in the product package imports, calls or
links anything here; only the tests, the smoke check of the entry module and
the CPU-baseline leg of the benchmark do.  The oracle shares no code with the
HIP path: it evaluates the spline weights from the truncated-power formula
(the HIP path uses per-interval polynomial tables built by the Cox-de Boor
recursion), it transforms with full complex DFT matrices (the HIP path uses
its own real-to-complex Stockham FFT), and it sums directly over the stencil
with numpy scatter/gather.

Modules
-------
bspline   centered cardinal B-spline M_p and its derivatives (Sec. 2.3.2)
pme       the particle-mesh method on a given mesh (Secs. 2.3.1-2.3.5):
          density, influence function, potential, energy, gradients and the
          Hessian-vector product
ewald     explicit Ewald summation for charges and point dipoles (the
          conventional baseline the paper validates against, Sec. 2.3 and 3)
quad      the quadrupole channel the paper names as its next extension
          (Sec. 4): density, self terms, PME and Ewald energies and gradients
pol       the Thole-damped polarizable teacher: real-space pair sum, its
          gradients and Hessian rows, and the self-consistent dipoles
dip       the learned dipole head on local features (Sec. 2.2) and its
          training through PME (Sec. 2.4)
heads     the charge head (Sec. 2.2) and training on conservative forces
          (Sec. 2.4), second order through the features and both networks
"""
