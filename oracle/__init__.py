"""Plain, slow, FP64 CPU reference of the local-energy / gradient path.

TEST INFRASTRUCTURE ONLY.  Nothing in the product path may import this
package: only the tests, the smoke check and the benchmark's CPU-baseline leg
use it.  It shares no code with the HIP library and never imports it.

Every function follows a passage of Zhao, Stokes & Veerapaneni,
"Scalable neural quantum states architecture for quantum chemistry"
(arXiv 2208.05637); docstrings cite the section / equation.  Readings of
points the paper leaves open are listed in the module docstrings where they
are taken.

Modules
  pauli : Pauli matrices (Eq. 1), Pauli expansion of H (Eq. hamiltonpauli),
          matrix element rule (Eq. mtx_element), canonical merged term set,
          dense and sector-block Hamiltonians for small n.
  made  : the masked autoregressive amplitude/phase network (Sec. 4,
          Architecture and Constraints, Eq. modifier), FP64 forward and a hand
          reverse pass.
  vmc   : local energy (Eq. local_energy_auto, Alg. 1), the energy estimate
          (Eq. total_energy_sum), the VMC gradient (Eq. grad), and the
          per-(sample, flip-group) validity bits and matrix elements.
  sampler : unique-sample autoregressive sampling (Sec. 4, Sampling).
  adam  : the optimiser step (Sec. 6).

Bit strings are uint64 arrays up to 64 qubits and Python integers (dtype
object) of any width above; every function takes either.
"""
from . import pauli, made, vmc  # noqa: F401
