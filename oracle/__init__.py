"""Plain FP64 CPU oracle for monitored free-fermion quantum trajectories.

TEST INFRASTRUCTURE ONLY.  This package is the slow, obviously-correct
reference that the GPU library is checked against.  Only the test suite,
``__graft_entry__.smoke()`` and the ``cpu_baseline`` leg of ``bench.py`` may
import it.  The GPU library never imports, links or calls anything here, and
nothing here imports the GPU library: the two share no code.

Everything follows arXiv:2508.18468 (Fan, Yin, Garcia-Garcia), "Entanglement
dynamics of monitored noninteracting fermions on graphics processing units":

* lattice and hopping matrix            -- Sec. II (model) and Appendix A
* propagator exp(-i H dt)               -- Appendix A (free evolution)
* Neel / checkerboard initial state     -- Appendix A
* projective (PM) measurement           -- Appendix A, Eq. (A1) and Eq. (A2)
* homodyne (QSD) update                 -- Appendix A, Eq. (A4)
* QR re-orthonormalisation              -- Appendix A (after each step)
* entanglement entropy                  -- Sec. II, entropy formula
* mutual information                    -- Sec. IV
* density correlation C(r), G_AB        -- Sec. II Eq. (2), Sec. IV Eq. (5)
* continuous-time projective protocol   -- Appendix A (Poisson waiting times, one site per event)
* RK4 homodyne integrator              -- Appendix A (Eq. (A4) integrated by RK4)

Random numbers: Philox4x64-10 (Salmon et al., SC'11), implemented here from
its published definition, independently of the GPU's implementation.

Parity status of every function is stated in its docstring; the pins live in
``tests/test_oracle_*.py``.
"""

from .lattice import Lattice, hopping_matrix, default_occupied
from .propagator import propagator
from .philox import philox4x64_10, u01, pm_uniforms, qsd_normals
from .trajectory import (initial_state, propagate, born_probabilities,
                         pm_measure, qsd_update, reorthonormalize, step,
                         run_trajectory)
from .observables import (correlation_matrix, region_spectrum, entropy_from_spectrum,
                          entanglement_entropy, mutual_information, density_correlation,
                          particle_covariance)
from .continuous import (event_draws, waiting_time, evolution_operator, evolve, measure_site,
                         state_from_correlation, run_continuous)
from .rk4 import generator as rk4_generator, rk4_propagate, rk4_step, run_rk4

__all__ = [
    "Lattice", "hopping_matrix", "default_occupied", "propagator",
    "philox4x64_10", "u01", "pm_uniforms", "qsd_normals",
    "initial_state", "propagate", "born_probabilities", "pm_measure", "qsd_update",
    "reorthonormalize", "step", "run_trajectory",
    "correlation_matrix", "region_spectrum", "entropy_from_spectrum",
    "entanglement_entropy", "mutual_information", "density_correlation", "particle_covariance",
    "event_draws", "waiting_time", "evolution_operator", "evolve", "measure_site",
    "state_from_correlation", "run_continuous",
    "rk4_generator", "rk4_propagate", "rk4_step", "run_rk4",
]
