"""GRIM-Filter CPU oracle: test infrastructure only (see ``oracle.py``)."""
from .oracle import Oracle, build, load  # noqa: F401
