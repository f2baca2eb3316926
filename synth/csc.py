"""Inputs of the charge-self-consistent term: on-site hardness U per atom (eV)
and a shift set for charge runs.  Values are stand-ins keyed by the valence
charge of each atom (Si 4, O 6, H 1); the paper gives no parameters."""
from __future__ import annotations

import numpy as np

HUBBARD_U = {4.0: 6.7, 6.0: 13.5, 1.0: 11.4}


def hubbard_u(system) -> np.ndarray:
    return np.array([HUBBARD_U[float(z)] for z in system.valence], dtype=np.float64)
