"""MI355X-native per-timestep step of the Digital Brain spiking network (arXiv 2211.15963).

The compute path is the HIP library ``libdbsim.so`` (C ABI in ``include/dbsim.h``);
``paper_2211_15963_amd.dbsim`` is its ctypes binding. Network descriptions come from
the seeded generator package ``netgen``.
"""
from .dbsim import Built, Simulator, DbsimError, footprint, lib  # noqa: F401

__all__ = ["Built", "Simulator", "DbsimError", "footprint", "lib"]
