"""Plain FP64 CPU oracle for the Hermitian FEAST contour-integration subspace step.

TEST INFRASTRUCTURE ONLY.  Nothing in the product path may import, call, link or
execute anything in this package: only ``tests/``, ``__graft_entry__.smoke()`` and
the ``cpu_baseline`` leg of ``bench.py`` use it.  It shares no code with the HIP
path (no kernels, headers, helpers, tables or constant generators); the two only
meet on seeded inputs produced by ``workloads/``.

Every function follows a passage of the FEAST v4.0 User Guide (arXiv:2002.04807)
and is written to be checked against that text by eye: the contour quadrature
(Section "Search contour", Table tab_contour; the Zolotarev rule fpm(16)=2 in
zolotarev.py), the Hermitian subspace iteration
with Rayleigh-Ritz (Section 1.1 "The FEAST Algorithm", Section 3.2 "FEAST
Hermitian", Tables tab-common1 and tab-rci1, the Hermitian RCI templates), the
residual inverse iteration of v4.0 (Section 1.2, Section 3.1 "Tips"), the
``fpm`` defaults (Table tab_fpm) and the ``info`` codes (Table tab_info).
Readings taken where the guide is silent are listed in each module header.
"""

from .contour import half_contour, rational_filter, gauss_legendre_rule
from .zolotarev import zolotarev_contour, zolotarev_filter, zolotarev_sign
from .splitmix import splitmix64_uniform, initial_subspace
from .ifeast import bicgstab_block, feast_csr, ifeastinit
from . import adjoint
from . import nonhermitian
from . import polynomial
from . import stochastic
from .feast import (
    feastinit,
    expand_uplo,
    feast_dense,
    rayleigh_ritz,
    validate,
)

__all__ = [
    "half_contour",
    "rational_filter",
    "gauss_legendre_rule",
    "zolotarev_contour",
    "zolotarev_filter",
    "zolotarev_sign",
    "splitmix64_uniform",
    "initial_subspace",
    "feastinit",
    "expand_uplo",
    "feast_dense",
    "rayleigh_ritz",
    "validate",
    "bicgstab_block",
    "feast_csr",
    "ifeastinit",
    "adjoint",
    "nonhermitian",
    "polynomial",
    "stochastic",
]
