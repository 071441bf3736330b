"""Case presets: the tiny parity plan, the prostate-shaped and head-and-neck-
shaped cases, and small seeded cases for the parity tests.

Attenuation is 0.05 per cm (0.005 per mm).  The lateral cut ``thr`` is the
one calibration knob: it sets how far the Gaussian profile is kept and so the
number of non-zeros.  Its values below were chosen to land the non-zero
counts near the stated problem sizes (about 1e6, 1e8 and 4e8).
"""
from __future__ import annotations

from . import CaseSpec, Shape

MU_PER_MM = 0.005


def _tiny() -> CaseSpec:
    # 36 beams at 10 deg, 10x10 beamlets at 6 mm, 32^3 voxels at 4 mm.
    h = 4.0
    return CaseSpec(
        name="tiny36",
        grid=(32, 32, 32), h=h,
        n_beams=36, n_rows=10, n_cols=10, pitch=6.0,
        sigma_vox=1.0, mu_per_mm=MU_PER_MM, thr=0.28,
        shapes=[
            Shape("target", "ellipsoid", (0.0, 0.0, 0.0), T=60.0, alpha=1.0, beta=1.0,
                  semi=(6 * h, 6 * h, 6 * h)),
            Shape("oar", "cyl_z", (9 * h, 0.0, 0.0), T=20.0, alpha=0.0, beta=0.5,
                  radius=3 * h, half_len=1e9),
        ],
        gamma=0.1, circular=1, max_leaf_step=2, seed=0,
    )


def _prostate() -> CaseSpec:
    # 180 beams at 2 deg, 40x40 beamlets at 5 mm, 128x128x64 voxels at 2.5 mm.
    return CaseSpec(
        name="prostate180",
        grid=(128, 128, 64), h=2.5,
        n_beams=180, n_rows=40, n_cols=40, pitch=5.0,
        sigma_vox=1.5, mu_per_mm=MU_PER_MM, thr=0.8,
        shapes=[
            Shape("ptv", "ellipsoid", (0.0, 0.0, 0.0), T=78.0, alpha=1.0, beta=1.0,
                  semi=(25.0, 20.0, 22.5)),
            # rectum-like: along z, tangent to the target posteriorly (-y)
            Shape("rectum", "cyl_z", (0.0, -30.0, 0.0), T=26.0, alpha=0.0, beta=0.5,
                  radius=10.0, half_len=30.0),
            # bladder-like: along x, tangent anteriorly (+y) and superiorly (+z)
            Shape("bladder", "cyl_x", (0.0, 26.0, 26.0), T=26.0, alpha=0.0, beta=0.5,
                  radius=20.0, half_len=40.0),
        ],
        gamma=0.1, circular=1, max_leaf_step=2, seed=0,
    )


def _headneck() -> CaseSpec:
    # 180 beams, 60 leaf rows (z) x 40 columns at 5 mm, 192x192x96 at 2.5 mm.
    return CaseSpec(
        name="headneck180",
        grid=(192, 192, 96), h=2.5,
        n_beams=180, n_rows=60, n_cols=40, pitch=5.0,
        sigma_vox=1.5, mu_per_mm=MU_PER_MM, thr=0.66,
        shapes=[
            Shape("ptv1", "ellipsoid", (0.0, 0.0, 0.0), T=70.0, alpha=1.0, beta=1.0,
                  semi=(20.0, 20.0, 20.0)),
            Shape("ptv2", "ellipsoid", (0.0, 0.0, 0.0), T=56.0, alpha=1.0, beta=1.0,
                  semi=(35.0, 35.0, 35.0)),
            Shape("cord", "cyl_z", (0.0, -50.0, 0.0), T=45.0, alpha=0.0, beta=0.5,
                  radius=5.0, half_len=1e9),
            Shape("parotid_l", "ellipsoid", (45.0, -10.0, 10.0), T=26.0, alpha=0.0, beta=0.5,
                  semi=(15.0, 12.0, 20.0)),
            Shape("parotid_r", "ellipsoid", (-45.0, -10.0, 10.0), T=26.0, alpha=0.0, beta=0.5,
                  semi=(15.0, 12.0, 20.0)),
            Shape("brainstem", "cyl_z", (0.0, -30.0, 75.0), T=54.0, alpha=0.0, beta=0.5,
                  radius=12.0, half_len=30.0),
            Shape("mandible", "shell_y", (0.0, 0.0, -30.0), T=70.0, alpha=0.0, beta=0.5,
                  radius=50.0, r_in=45.0, half_len=15.0),
        ],
        gamma=0.1, circular=1, max_leaf_step=2, seed=0,
    )


def tiny_case(n_beams=8, n_rows=4, n_cols=6, grid=(12, 12, 8), h=4.0, pitch=6.0,
              sigma_vox=1.0, thr=0.3, seed=0, gamma=0.1, circular=1, max_leaf_step=2) -> CaseSpec:
    """Small seeded case for the parity tests."""
    nx, ny, nz = grid
    r = 0.25 * min(nx, ny, nz) * h
    return CaseSpec(
        name=f"small{n_beams}x{n_rows}x{n_cols}",
        grid=grid, h=h, n_beams=n_beams, n_rows=n_rows, n_cols=n_cols, pitch=pitch,
        sigma_vox=sigma_vox, mu_per_mm=MU_PER_MM, thr=thr,
        shapes=[
            Shape("target", "ellipsoid", (0.0, 0.0, 0.0), T=60.0, alpha=1.0, beta=1.0,
                  semi=(r, r, r)),
            Shape("oar", "cyl_z", (1.6 * r, 0.0, 0.0), T=20.0, alpha=0.0, beta=0.5,
                  radius=0.6 * r, half_len=1e9),
        ],
        gamma=gamma, circular=circular, max_leaf_step=max_leaf_step, seed=seed,
    )


PRESETS = {"tiny36": _tiny, "prostate180": _prostate, "headneck180": _headneck}


def preset(name: str) -> CaseSpec:
    return PRESETS[name]()
