"""Plain FP64 CPU oracle of the coupled vortex-filament / lattice-Boltzmann step.

TEST INFRASTRUCTURE ONLY.  This package is the slow, obviously correct
reference that the GPU library is checked against.  Only the test suite,
``__graft_entry__.smoke()`` and the ``cpu_baseline`` leg of ``bench.py`` may
import it.  The GPU library (``paper_2108_04435_amd``) never imports,
links or calls anything in here, and nothing in here imports the library.

Source: S. Inui and M. Tsubota, "Coupled dynamics of quantized vortices and
normal fluid in superfluid 4He based on lattice Boltzmann method",
arXiv:2108.04435.  Each function cites the section / equation / table it
follows.  Where the paper is silent the reading taken is named in the
docstring (R-numbers, the same numbering throughout the package).

Modules
-------
d3q19     lattice velocities, weights, opposite directions   (Sec. II.B, Table I)
lbm       equilibrium, Guo/Cheng-Li forcing, four-equation collide, streaming
          with halfway bounce-back and velocity planes          (Sec. II.B)
vfm       filament geometry, Biot-Savart, LIA, Schwarz EoM, mutual-friction
          force, two-point-delta interpolation and spreading,
          mass-balance superflow                      (Sec. II.A, II.B, III.C)
topology  remeshing, reconnection, small-loop removal, compaction
                                                     (Sec. II.A, III.B)
coupled   one coupled time step (RK4 on the filaments, one LBM update)
diagnostics  vortex line length (total and per z slab), normal-fluid
          velocity statistics, vorticity        (Sec. III.A, III.C, IV)

All floating point is IEEE binary64 (numpy float64).  numpy never contracts
a*b+c into a fused multiply-add, so every threshold decision below
(remeshing, reconnection, nearest periodic image) is a deterministic
function of the stored positions.
"""

from . import d3q19, lbm, vfm, topology, coupled, diagnostics  # noqa: F401
