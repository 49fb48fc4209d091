"""FP64 CPU oracle for the per-frame signal-separation path.

TEST INFRASTRUCTURE ONLY.  Nothing in the product imports this package: only
the test suite, the smoke check in ``__graft_entry__`` and the CPU-baseline leg
of ``bench.py`` may import or call it.  It shares no code with the HIP path;
the only inputs both sides share come from the ``synth`` package.

The oracle is plain and slow on purpose: NumPy over explicit per-bin and
per-pixel arrays, float64 throughout, following the paper's definitions in the
order the paper states them (Kieffer et al., "Application of signal separation
to diffraction image compression and serial crystallography", 2024):

* ``geometry``  -- pixel scattering angles, radial bins and the CSR
  pixel-to-bin matrix with optional bounding-box pixel splitting (Sec. 2.2,
  "Azimuthal averaging");
* ``correct``   -- Jungfrau raw words to corrected signal (Sec. 1.2); the
  formula is the reading stated in that module (the paper defers it to the
  LImA2 reference) and is **parity unpinned** against the paper, pinned only
  by its own definition and by the detector forward model;
* ``stats``     -- per-bin weighted moments (eqs. avg, varA, varB, omega,
  omegaomega, Vp, VVp, weighted_avg, std2, sem2), the Poisson model (eqs.
  poisson, varianceP, sem), iterative sigma-clipping (eq. clip, Sec. 2.4) and
  the Chauvenet cut-off (eq. chauvenet);
* ``classify``  -- per-pixel background lookup, sparsification (Sec. 3),
  densification, noise free and with regenerated noise (Sec. 3.2), the peak
  finder and the peak-count veto (Sec. 4);
* ``rng``       -- the counter-based generator (Philox4x32-10) and the
  Box-Muller normals of the noisy densification, pinned by the generator's
  published known-answer vectors.

Readings where the paper is silent are stated in each function's docstring.
Parity unpinned by the paper (pinned only by stated definitions): the raw-word
correction, the bounding-box splitting rule, the per-pixel background
interpolation, the peak-record definition, and the noise convention of the
noisy densification (generator, truncation).
"""

from . import geometry, correct, stats, classify, rng  # noqa: F401
