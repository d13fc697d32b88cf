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

The l > 0 analytic shot-noise assembly (``shotnoise.scoccimarro_shot_terms``,
``shotnoise.triposh_shot_terms``) is pinned term by term against the exact
closure sums of ``shotnoise_exact`` (the FFT method of the section validating
the analytic noise, extended to every coincidence case), which are themselves
pinned by a brute-force particle enumeration of each case
(``tests/test_oracle_shot_exact.py``); the agreement holds within the stated
thin-shell tolerances, and planted assembly mistakes fail them.
"""

from . import catalog, mesh, ylm, spectra, bispectrum, shotnoise, shotnoise_exact, pipeline  # noqa: F401
