"""MI355X-native pair-galaxy cross-correlation (xi_pg, b_pg, Q_eff).

The computation lives in the HIP library ``libpgx.so`` behind the C-ABI of
``include/pgx.h``; this package only marshals arguments.  Importing the
package does not load the library; the first call that needs it does, and
raises if it is missing.
"""
from ._lib import Plan, PgxError, build_digest, load_library


def __getattr__(name):
    # torch-dependent helpers are imported on first use
    if name in ("PairGalaxyXi", "pair_galaxy_xi", "hod_weights", "MultipoleXi", "pair_galaxy_multipoles"):
        from . import autograd
        return getattr(autograd, name)
    if name in ("HodFit", "fit_hod", "projected_2pcf"):
        from . import hodfit
        return getattr(hodfit, "fit" if name == "fit_hod" else name)
    raise AttributeError(name)


__all__ = ["Plan", "PgxError", "build_digest", "load_library", "PairGalaxyXi", "pair_galaxy_xi", "hod_weights",
           "MultipoleXi", "pair_galaxy_multipoles", "HodFit", "fit_hod", "projected_2pcf"]
