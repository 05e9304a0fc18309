"""MI355X-native quantum-trajectory solver for the QTraj 1.0 method
(arXiv:2107.06147): split-step pseudo-spectral evolution of radial wave
functions under the non-Hermitian singlet/octet Hamiltonian, with the
waiting-time quantum-jump rule, run as hand-written HIP kernels for gfx950
behind the C ABI declared in include/qtraj.h.

`paper_2107_06147_amd.qtraj` is the thin ctypes binding (argument marshalling
only).  `paper_2107_06147_amd.workloads` generates seeded synthetic inputs.
"""
