"""CPU FP64 oracle for the voxel hex8 SIMP state solve, sensitivity, filters and
density-to-SDF transfer (Jezek et al., "Sequential topology optimization: SIMP
initialization for level-set boundary refinement").

TEST INFRASTRUCTURE ONLY.  This package is the plain, slow, obviously-correct
reference that the GPU path is checked against.  Only the test-suite, the smoke
check and the CPU-baseline leg of the benchmark may import it.  The product
path (the HIP library and its Python binding) never imports, links or calls
anything here, and this package imports nothing from the product.

Everything is NumPy/SciPy in float64, one step per paper passage:

  grid      numbering, boundary conditions and loads,
            the paper's own BC variants                 (Sec. 2.1.1, Eq. 2;
                                                          Secs. 4.2-4.3)
  element   unit-modulus hex8 stiffness k_e^0           (Sec. 2.1.2, Eq. 3)
  fem       assembled K, masked operator, direct solve,
            Jacobi-PCG, compliance and sensitivity       (Eqs. 1-3)
  filters   density filter, its adjoint, sensitivity
            filter                                       (Sec. 2.1.3, Eq. 4)
  sdf       nodal LSQ map, marching tetrahedra, closest
            point, unsigned/signed distance, ersatz
            volume fraction                              (Secs. 3.2-3.4,
                                                          Eqs. 25-30)
  simp      optimality-criteria update with bisection on
            the volume multiplier, and the SIMP loop     (Sec. 2.1, SIMP
                                                          set-up of Sec. 4)
  levelset  Hamilton-Jacobi evolution with the CFL step
            and reinitialisation with the smeared sign,
            first-order Godunov upwind on the node grid  (Secs. 2.2.7-2.2.8,
                                                          Eqs. 21-24)
  shape     relaxed shape derivative (nodal vector) and
            the Hilbertian extension A_H vbar = g        (Secs. 2.2.5-2.2.6,
                                                          Eqs. 15-20)
"""
