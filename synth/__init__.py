"""Seeded synthetic stereo inputs shared by the oracle tests and the HIP path."""
from .scenes import StereoPair, make_pair, random_labels  # noqa: F401
from .workloads import WORKLOADS, PAPER_PARAMS, workload, make_workload_pair, params_for  # noqa: F401
