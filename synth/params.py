"""Primary parameter vector of the Segment Linking chain (configuration input).

These are the free constants of the method as this project reads the paper:
the 0.8 GeV threshold and the 3.8 T field are the paper's (Sec. 2); the
resolutions are those of the synthetic detector; the remaining window widths
and chi2 limits are this project's choices (the paper prints no cut value).
Both the HIP library and the CPU oracle take this vector as input and derive
their FP32 constants from it independently.  Order matches the C enums.
"""
import numpy as np

from .events import B_FIELD, SIGMA_U, SIGMA_V

NAMES = ("bfield", "ptmin", "z0max", "sigu", "sigv", "nsig", "epsk", "epsa", "d0max",
         "xrphi", "xrz", "w", "map_dphi", "map_dl")

DEFAULTS = dict(
    bfield=B_FIELD,     # T
    ptmin=0.8,          # GeV, stub/segment/triplet threshold (Sec. 2)
    z0max=15.0,         # cm, 3 sigma of the luminous region
    sigu=SIGMA_U,       # cm, precise-axis resolution
    sigv=SIGMA_V,       # cm, coarse-axis resolution
    nsig=3.0,           # window half-width in resolution units
    epsk=0.05,          # relative curvature margin above kappa_max
    epsa=0.05,          # curvature-agreement slack in units of kappa_max
    d0max=2.0,          # cm, impact parameter allowed by the beam-line cut
    xrphi=13.82,        # chi2 (2 dof) at p = 1e-3
    xrz=16.27,          # chi2 (3 dof) at p = 1e-3
    w=1.0,              # window scale
    map_dphi=0.02,      # rad, azimuthal margin of the module map
    map_dl=1.0,         # cm, length margin of the module map
)


def make(**over) -> np.ndarray:
    d = dict(DEFAULTS)
    for k, v in over.items():
        if k not in d:
            raise KeyError(k)
        d[k] = v
    return np.array([d[n] for n in NAMES], dtype=np.float64)
