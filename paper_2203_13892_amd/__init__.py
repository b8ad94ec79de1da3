"""MI355X-native tree-reuse noisy trajectory simulation (TQSim, arXiv 2203.13892).

Importing the package loads nothing; ``paper_2203_13892_amd.tqsim`` binds the
HIP library ``libtqsim.so`` and ``paper_2203_13892_amd.workloads`` generates
seeded circuits.
"""
__all__ = ["tqsim", "workloads"]
