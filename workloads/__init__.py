"""Seeded synthetic inputs shared by the oracle and the GPU path.

This package only *defines* inputs: the one- and two-body coefficients of a
local impurity Hamiltonian (Sec. 2.1, the local-Hamiltonian equation) and
time-ordered operator strings (the configurations C of Sec. 2.2).  It holds
none of the local-trace arithmetic: no many-body operators in the form the
trace uses, no propagators, no sector blocks, no traces.
"""

from .impurity import Impurity, make_impurity, IMPURITY_NAMES  # noqa: F401
from .configs import make_configs, OperatorString  # noqa: F401
