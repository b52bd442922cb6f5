"""CPU oracle for the thick-restart block Lanczos (TRBL) shell-model eigensolver.

TEST INFRASTRUCTURE ONLY. Plain, slow, FP64 code written from the paper's
definitions; it shares no code with the GPU library. Only ``tests/``,
``__graft_entry__.smoke()`` and the ``cpu_baseline`` leg of ``bench.py`` may
import or run anything in this package.

Modules:
  basis        M-scheme Slater determinants, Table-1 order, product basis (Sec. 2, App. A)
  cg           Clebsch-Gordan coefficients (Racah's closed formula)
  interaction  J-coupled two-body matrix elements -> m-scheme terms (Sec. 2, Hamiltonian)
  hamiltonian  explicit matrix elements <M_i|H|M_j> with Jordan-Wigner signs (App. B)
  trbl         thick-restart block Lanczos, Alg. 4 and the restart equations (Sec. 3.4)
  grad         eigenvalue-sum gradient with respect to two-body matrix elements
"""
