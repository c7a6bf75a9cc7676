"""Shared test helpers: oracle parameters for a workload and error measures."""
import numpy as np

import oracle


def oracle_cfg(mesh, theta, omega, **kw):
    keys = ("dim", "degree", "r_in", "r_if", "r_out", "height", "n_theta", "n_r_rotor", "n_r_stator", "n_z", "nu",
            "penalty_F", "penalty_rule", "steady", "dt", "n_theta_stator")
    cfg = {k: mesh[k] for k in keys if k in mesh}
    cfg.update(theta_rot=float(theta), omega=float(omega))
    cfg.update(kw)
    return oracle.params(**cfg)


def relmax(a, b):
    """max-norm error of a relative to the max-norm of b."""
    return float(np.abs(np.asarray(a) - np.asarray(b)).max() / np.abs(np.asarray(b)).max())


def small_mesh(dim, k, n_theta=5, n_r_rotor=2, n_r_stator=3, n_z=3, **kw):
    m = dict(dim=dim, degree=k, r_in=0.3, r_if=0.55, r_out=1.0, height=0.8, n_theta=n_theta, n_r_rotor=n_r_rotor,
             n_r_stator=n_r_stator, n_z=n_z if dim == 3 else 1, nu=0.02, steady=1, dt=1.0)
    m.update(kw)
    return m
