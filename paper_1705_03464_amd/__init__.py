"""MI355X-native pair-galaxy cross-correlation (xi_pg, b_pg, Q_eff).

The computation lives in the HIP library ``libpgx.so`` behind the C-ABI of
``include/pgx.h``; this package only marshals arguments.  Importing the
package does not load the library; the first call that needs it does, and
raises if it is missing.
"""
from ._lib import Plan, PgxError, load_library

__all__ = ["Plan", "PgxError", "load_library"]
