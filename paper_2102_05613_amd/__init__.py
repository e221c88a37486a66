"""MI355X many-configuration Markov-chain Monte Carlo (MCMCMC) for the SK spin glass.

A thin ctypes binding over ``libmc3.so`` (C ABI in ``include/mc3.h``): argument
marshalling only, every step of the path runs in the HIP kernels.  PyTorch provides
the device workspace and the stream.  There is no CPU fallback: if the library is not
built, importing :mod:`paper_2102_05613_amd.native` fails loudly.
"""
from .inputs import Workload, couplings_gauss, couplings_pm1, workload, workloads  # noqa: F401

__all__ = ["Workload", "couplings_gauss", "couplings_pm1", "workload", "workloads"]
