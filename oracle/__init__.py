"""FP64 CPU oracle for the COLA particle-mesh step (Koda et al. 2015, Sec. 2).

TEST INFRASTRUCTURE ONLY.  Nothing in the product path (the HIP library and
its Python binding) imports, links or calls this package.  Only the tests,
the smoke check and the CPU-baseline leg of the benchmark use it.

It is a plain, slow, obviously-correct implementation written from the paper:
NumPy/SciPy in float64, CIC by ``np.bincount``, FFTs by ``scipy.fft``.  It
shares no code with the GPU path.  Each function cites the passage it follows.

Modules
  cosmology  growth factors, Hubble rate, COLA kick/drift factors (Sec. 2.1-2.2)
  ic         Gaussian field -> 2LPT displacements (Sec. 2.1, 2LPT growing mode)
  pm         CIC deposit, Poisson/gradient, CIC readout (Sec. 2.2-2.3)
  cola       residual kick/drift integrator (eqs. cola-drift, cola-kick)
  velocity   full particle velocities at the position time, redshift-space
             displacements (Sec. 2.1-2.2, Sec. 4.4)
  pk         matter power-spectrum estimator (Sec. 3.3)
  cic_fp32   float32 same-order replay of the deterministic CIC deposit
  adjoint    reverse-mode derivative of the step and of the 2LPT map
  philox     Philox4x32-10 counter-based generator (Salmon et al. 2011)
  fof        friends-of-friends groups, b = 0.2 of the mean separation (Sec. 3.1)
"""
