"""Plain FP64 CPU oracle of the power-spectrum and bispectrum multipole estimators.

TEST INFRASTRUCTURE ONLY.  Only ``tests/``, ``__graft_entry__.smoke()`` and the
``cpu_baseline`` leg of ``bench.py`` may import or run anything in this package.
The GPU library never calls it and shares no code, table or constant generator
with it; both sides only consume the seeded inputs of ``synthcat``.

Every function follows the plain definition of what the paper's estimators
compute (sections "Lossless Symmetry Reduction of Existing Estimators",
"Modified high-order multipoles", "A New Compressed TripoSH Bispectrum
Estimator" and "Bispectrum Shot Noise ..."), in FP64, without the m >= 0
symmetry reduction, the half-spectrum layout or any blocking: it sums over all
2l+1 values of m with complex FFTs, so the GPU path's symmetry shortcuts are
*tested* against it rather than assumed.

Readings of points the paper leaves open are fixed in the module docstrings of
``mesh``, ``spectra``, ``bispectrum`` and ``shotnoise``.

Pins: ``tests/test_oracle_*.py`` check every function here against values the
paper prints, closed forms, identities and brute-force sums (see each test's
docstring).  Functions without such a pin say "parity unpinned" in their
docstring.

Parity unpinned (partially): the l > 0 analytic shot-noise assembly
(``shotnoise.scoccimarro_shot`` and ``shotnoise.triposh_shot`` for l = 2).  Its
ingredients are pinned (g_l, the ring lemma, the alias sums, Q_l/H_l as shell
means) and its l = 0 case is pinned statistically on Poisson catalogs, but no
printed value or closed form fixes the l = 2 combination itself.
"""

from . import catalog, mesh, ylm, spectra, bispectrum, shotnoise, pipeline  # noqa: F401
