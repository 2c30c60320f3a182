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


# pixel objects (pLS, pT3, pT5, cross-cleaning): the synthetic pixel
# detector's resolutions and this project's window, cleaning distance and
# chi2 limits at p = 1e-3 (the paper prints none)
PIX_NAMES = ("sig_rphi", "sig_z", "wlink", "dr2", "x5p", "x5z", "x3p", "x3z")
PIX_DEFAULTS = dict(
    sig_rphi=0.0010,    # cm, pixel hit resolution across the track
    sig_z=0.0020,       # cm, along z
    wlink=0.05,         # sine of the largest angle between a pLS and an object it links to
    dr2=1e-3,           # squared eta-phi distance of duplicates in cross-cleaning
    x5p=22.46,          # pT5 r-phi chi2 (6 dof)
    x5z=24.32,          # pT5 r-z chi2 (7 dof)
    x3p=18.47,          # pT3 r-phi chi2 (4 dof)
    x3z=20.52,          # pT3 r-z chi2 (5 dof)
)


def make_pixel(**over) -> np.ndarray:
    d = dict(PIX_DEFAULTS)
    for k, v in over.items():
        if k not in d:
            raise KeyError(k)
        d[k] = v
    return np.array([d[n] for n in PIX_NAMES], dtype=np.float64)
