"""Write the FP64 oracle's outputs for full-size benchmark catalogs.

Calls only ``oracle`` (and ``synthcat`` for the seeded inputs); nothing here
reads the GPU library.  The GPU tests regenerate the same catalogs from the same
seeds, check their SHA-256 against the one stored here, and compare the
library's outputs with these values element by element.

    python tests/golden/make_oracle_fixtures.py c2|c3|c4min [--out DIR]

* c2: 256^3 TSC + interlacing, 5e6 + 2.5e7 (seeds 2000 / 2001), 20 bins of 0.01:
  P_0, P_2, P_4, P_22, P_42, P_44, P_4b, P_6b, P_8b, mode counts, k_eff
  (eqs. Hand17, Pllp, Plnew).
* c3: 256^3, 2e6 + 2e7 (seeds 3000 / 3001), 20 bins: Scoccimarro B_0 and B_2
  (configurations, N_T, raw, shot; eq. bi_sco with the analytic noise) and
  TripoSH BB_202 (raw, shot; eq. new_bispec).
* c4min: the smallest mock of the 64-mock batch (N_g from the log-uniform draw of
  seed 4999, 10 N_g randoms, seeds 4126 / 4127): P_0, P_2, P_4 and B_0.
The oracle takes about 10-20 minutes per case on one core.
"""

from __future__ import annotations

import argparse
import hashlib
import json
import os
import sys
import time

HERE = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(os.path.dirname(HERE))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)

import numpy as np  # noqa: E402

import synthcat  # noqa: E402
from oracle.pipeline import MeshConfig, measure_bk, measure_pk  # noqa: E402


def catalog_digest(g: np.ndarray, r: np.ndarray) -> str:
    h = hashlib.sha256()
    h.update(np.ascontiguousarray(g).tobytes())
    h.update(np.ascontiguousarray(r).tobytes())
    return h.hexdigest()


def case_catalog(case: str):
    if case in ("c2", "c3"):
        config = int(case[1])
        spec = synthcat.config_spec(config)
        g = synthcat.lognormal_catalog(spec.ngal, spec.boxsize, 1000 * config)
        r = synthcat.random_catalog(spec.nran, 1000 * config + 1)
        return spec, g, r
    if case == "c4min":
        spec = synthcat.config_spec(4)
        sizes = synthcat.mock_sizes_c4(64)
        k = int(np.argmin(sizes))
        ng = int(sizes[k])
        g = synthcat.lognormal_catalog(ng, spec.boxsize, 4000 + 2 * k)
        r = synthcat.random_catalog(10 * ng, 4000 + 2 * k + 1)
        return spec, g, r
    raise ValueError(case)


def _floats(a):
    return [float(x) for x in np.asarray(a, dtype=np.float64).ravel()]


def run(case: str) -> dict:
    spec, g, r = case_catalog(case)
    obs = synthcat.observer_position()
    cfg = MeshConfig(spec.boxsize, spec.nmesh, spec.assign, spec.interlace, obs)
    out = {"case": case, "ngal": int(g.shape[1]), "nran": int(r.shape[1]),
           "catalog_sha256": catalog_digest(g, r), "nmesh": spec.nmesh, "boxsize": spec.boxsize,
           "dk": spec.dk, "nbins": spec.nbins}
    t0 = time.time()
    if case in ("c2", "c4min"):
        pk = measure_pk(g, None, r, None, cfg, 0.0, spec.dk, spec.nbins, ells=(0, 2, 4),
                        modified=(case == "c2"))
        out["nmodes"] = [int(x) for x in pk["nmodes"]]
        out["k_eff"] = _floats(pk["k_eff"])
        keys = ("P0", "P2", "P4", "P22", "P42", "P44", "P4b", "P6b", "P8b") if case == "c2" else ("P0", "P2", "P4")
        out["pk"] = {k: _floats(pk[k]) for k in keys}
    if case in ("c3", "c4min"):
        sco = (0, 2) if case == "c3" else (0,)
        tri = (2,) if case == "c3" else ()
        bk = measure_bk(g, None, r, None, cfg, spec.dk, spec.nbins, ells=(0, 2) if case == "c3" else (0,),
                        scoccimarro=sco, triposh=tri)
        out["nmodes"] = [int(x) for x in bk["nmodes"]]
        for l in sco:
            out[f"B{l}"] = {"configs": [[int(v) for v in c] for c in bk[f"B{l}_configs"]],
                            "ntri": [int(x) for x in bk[f"B{l}_ntri"]],
                            "raw": _floats(bk[f"B{l}_raw"]), "shot": _floats(bk[f"B{l}_shot"])}
        for l in tri:
            key = f"BB{l}0{l}"
            out[key] = {"pairs": [[int(v) for v in p] for p in bk[f"{key}_pairs"]],
                        "raw": _floats(bk[f"{key}_raw"]), "shot": _floats(bk[f"{key}_shot"])}
    out["oracle_seconds"] = round(time.time() - t0, 1)
    return out


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("case", choices=("c2", "c3", "c4min"))
    ap.add_argument("--out", default=HERE)
    a = ap.parse_args()
    res = run(a.case)
    path = os.path.join(a.out, f"oracle_{a.case}.json")
    with open(path, "w") as f:
        json.dump(res, f, separators=(",", ":"))
        f.write("\n")
    print(f"wrote {path} ({res['oracle_seconds']} s of oracle)")


if __name__ == "__main__":
    main()
