"""MI355X (gfx950) local energy and VMC gradient for Pauli-string Hamiltonians.

Hot path: HIP kernels in ``libnqs.so`` behind the C ABI of ``include/nqs.h``;
this package is the thin ctypes binding.  Importing it does not load the
library; the first call does, and raises if it has not been built.
"""
from .api import (Context, Hamiltonian, Plan, EnergyFn, net_desc, param_count, log_psi,
                  local_energy, energy_grad, energy_grad_noalloc, energy_grad_multi, multi_workspace, multi_device_status, connected,
                  reduce_table, device_status, sample, Adam, tune_db_load, tune_db_save)
from ._lib import NQSError, load, LIB_PATH

__all__ = ["Context", "Hamiltonian", "Plan", "EnergyFn", "net_desc", "param_count", "log_psi",
           "local_energy", "energy_grad", "energy_grad_noalloc", "energy_grad_multi", "multi_workspace", "multi_device_status", "connected", "reduce_table",
           "device_status", "sample", "Adam", "tune_db_load", "tune_db_save", "NQSError", "load", "LIB_PATH"]
