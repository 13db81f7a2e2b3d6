"""MI355X-native (gfx950) ADER-DG element update for the elastic and
anelastic wave equations with clustered rate-2 local time stepping.

The solver is the C-ABI library libedge_lts.so (include/edge_lts.h) built
from csrc/ (host C++ and HIP kernels); `binding` marshals arguments to it.
"""
from .binding import (Context, EdgError, cluster_host, lib, n_basis, n_face_basis,  # noqa: F401
                      reference_matrices, BC_ABSORB, BC_FREE, BC_INTERIOR, FLAG_CHECK_FINITE, FLAG_GRAPH,
                      FLAG_POISON, FLAG_POISON_EARLY, FLAG_SHUFFLE, STF_HANN, STF_RICKER)
