"""FP64 CPU oracle for the MUSER imaging hot path (test infrastructure only).

This package is the slow, plain reference that the GPU path is checked against.  It is
test infrastructure: only the test suite, the package smoke check and the benchmark's
CPU-baseline leg may import it.  It shares no code with the HIP library or its Python
binding and imports neither.

Parity status per function (see each module header for the pins):
  gcf.pswf / gcf.kernel_table / gcf.correction   pinned (scipy prolate functions, eigen-equation)
  imager.prep / weights / grid / b0 / dirty_*    pinned (direct DFT, closed forms, Alg. 1 pillbox case)
  clean.hogbom / clean.replay                    pinned (closed forms, CLEAN identity)
  clean.fit_clean_beam / clean.restore           pinned (exact Gaussian beam, empty model)
  adjoint.predict / adjoint.adjoint              pinned (dot-product identity, brute-force transpose)
  gmm.histogram / gmm.em_fit / gmm.levels        pinned (exact binning, closed-form moments, monotone EM, known mixture)
  centering.correlate / peak_offset / disk_offset / phase_correct
                                                 pinned (direct-sum correlation, whole-pixel shifts, point-source phase)
  steer.steer / steer.replay / steer.convolve_window
                                                 pinned (trim 1 = Hogbom, point-source and flat-source closed
                                                 forms, two-tap alpha, CLEAN identity, direct-sum convolution)
  wproj.exact_dirty / plan / kernel_table / dirty_image_w
                                                 pinned (2-D DFT at w = 0, spheroidal product at w = 0, symmetries,
                                                 phase rule, exact w-term image of a point source)
"""
