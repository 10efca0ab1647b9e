"""MI355X-native driven-lid-cavity time stepper (vorticity-stream function, SSPRK(5,4)).

The compute path is the HIP library ``libcavity.so`` (sources in ``csrc/``),
reached through the ctypes binding in :mod:`paper_0809_3098_amd.cavity`.
Importing this package loads nothing; import the binding explicitly.
"""

__all__ = ["inputs", "workloads"]
