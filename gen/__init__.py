"""Seeded synthetic inputs shared by the tests, the benchmark and the oracle's
pins.  Holds no stochastic-reconfiguration arithmetic: only random draws and the
networks' log-derivative Jacobians that form the path's input O."""
from . import networks, workloads  # noqa: F401
