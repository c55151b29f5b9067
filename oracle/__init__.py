"""FP64 CPU oracle of the EPR iteration -- test infrastructure only (see epr_oracle.py)."""
from . import epr_oracle  # noqa: F401
