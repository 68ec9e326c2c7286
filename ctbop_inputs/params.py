"""Potential parameters as a flat float64 vector.

This module is data marshalling only: it reads a JSON parameter file and lays
its numbers out in the flat order that every consumer (the HIP library's C
ABI and the CPU oracle) documents for itself.  It does no arithmetic of the
method.

Flat layout (56 doubles).  Species index t: 0 = Si, 1 = C; base = 26 * t.

    base+0  A        base+1  B        base+2  lam1     base+3  lam2
    base+4  R        base+5  S        base+6  sigma
    base+7  .. base+13   channel 1: gamma, c, d, h, n, g, alpha
    base+14 .. base+20   channel 2: gamma, c, d, h, n, g, alpha
    base+21 chi      base+22 J        base+23 gamma_coul
    base+24 E0       base+25 mass
    52  B_mix_SiC    53  ke           54  rc_coul      55  p
"""
from __future__ import annotations

import json
import os

import numpy as np

N_PER_SPECIES = 26
N_PARAMS = 56
SPECIES = ("Si", "C")
_CH_KEYS = ("gamma", "c", "d", "h", "n", "g", "alpha")
_SP_KEYS = ("A", "B", "lam1", "lam2", "R", "S", "sigma")
_Q_KEYS = ("chi", "J", "gamma_coul", "E0", "mass")
_G_KEYS = ("B_mix_SiC", "ke", "rc_coul", "p")

DEFAULT_FILE = os.path.join(os.path.dirname(__file__), "sic_standin.json")


def names() -> list[str]:
    """Human-readable name of every flat slot, in layout order."""
    out = []
    for sp in SPECIES:
        out += [f"{sp}.{k}" for k in _SP_KEYS]
        for ch in ("ch1", "ch2"):
            out += [f"{sp}.{ch}.{k}" for k in _CH_KEYS]
        out += [f"{sp}.{k}" for k in _Q_KEYS]
    out += list(_G_KEYS)
    assert len(out) == N_PARAMS
    return out


def index(name: str) -> int:
    return names().index(name)


def flatten(doc: dict) -> np.ndarray:
    vals = []
    for sp in SPECIES:
        s = doc["per_species"][sp]
        vals += [float(s[k]) for k in _SP_KEYS]
        for ch in ("ch1", "ch2"):
            vals += [float(s[ch][k]) for k in _CH_KEYS]
        vals += [float(s[k]) for k in _Q_KEYS]
    vals += [float(doc["global"][k]) for k in _G_KEYS]
    arr = np.asarray(vals, dtype=np.float64)
    assert arr.shape == (N_PARAMS,)
    return arr


def load(path: str | None = None) -> np.ndarray:
    """Flat parameter vector from a JSON file (default: the Si-C stand-in)."""
    with open(path or DEFAULT_FILE) as f:
        return flatten(json.load(f))


def with_values(theta: np.ndarray, **kw) -> np.ndarray:
    """Copy of `theta` with named slots replaced, e.g. with_values(t, **{"C.ch1.alpha": 1.5})."""
    out = np.array(theta, dtype=np.float64, copy=True)
    nm = names()
    for k, v in kw.items():
        out[nm.index(k)] = float(v)
    return out


def variant_all_paths(theta: np.ndarray | None = None) -> np.ndarray:
    """Test-only set that switches on the terms the base set leaves at zero or
    at their neutral value: alpha != 0, g1 != g2, n1 != n2, E0 != 0."""
    t = load() if theta is None else np.array(theta, copy=True)
    upd = {}
    for sp, e0 in (("Si", -1.3), ("C", -2.1)):
        upd[f"{sp}.ch1.alpha"] = 1.5
        upd[f"{sp}.ch2.alpha"] = 0.8
        upd[f"{sp}.ch1.g"] = 1.3
        upd[f"{sp}.ch2.g"] = 0.9
        upd[f"{sp}.E0"] = e0
    upd["Si.ch1.n"] = 0.70
    upd["C.ch2.n"] = 0.80
    return with_values(t, **upd)
