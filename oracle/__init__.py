"""CPU oracle for moment propagation with adsorption/desorption.

TEST INFRASTRUCTURE ONLY. A plain, slow FP64 implementation of what the GPU
path computes, written from the paper (arXiv:1303.2470, Secs. II-III) and
pinned by brute force, invariants and the paper's exact results. Only the
test-suite, the smoke check and the CPU-baseline leg of the benchmark may
import it; the product library never does, and shares no code with it.

Modules:
  core          ctypes front end of the C oracle (classification, link
                probabilities, propagation, VACF, BGK flow)
  chain         independent brute force: dense Markov matrix, random walkers,
                exact 1D reduction of a slit
  closed_forms  Eqs. 13-15 of the paper
  mlp           FP64 forward/backward/Adam of the surrogate network
"""
from . import core  # noqa: F401
from .core import (bgk, build, classify, d_of_t, lambda_from, links,  # noqa: F401
                   propagate, set_threads, threads, uptake, vacf)
