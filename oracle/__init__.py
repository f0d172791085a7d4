"""FP64 CPU oracle for the FlashVAN hot path -- TEST INFRASTRUCTURE ONLY.

A plain, slow, obviously correct restatement of what the method computes,
written from the paper ("Scalable Physics-Inspired Transformers for Spin
Glasses"): the autoregressive factorisation (Eq. 1, Eq. 11), the spin energies
(Eq. 6, Eq. 8), the concatenated positional embedding (Eq. 15), the decoder
blocks with masked multi-head attention and no output projection (Eqs. 2-3,
Alg. 1, Alg. 2), the variational free energy (Eqs. 4-5) and its REINFORCE
gradient (Eqs. 16-19), the Muon update with Newton-Schulz orthogonalisation
(Methods, comparison of optimisers), the local Monte Carlo refinement and the
self-distillation weights of Eq. (loss2), the overlap distribution and the
annealing schedule (Eq. overlap_distribution; Methods, variational annealing),
the 2^D spin patching of the lattice models (Methods, model configurations and
training settings), and the ordered Markov boundary that sets the sparse attention window (Methods,
ordered Markov boundary; SI Sec. I A).

Only the test-suite, the smoke check and the benchmark's CPU-baseline leg may
import this package.  It shares no code with the HIP path: the two sides agree
by specification (the documented parameter layout, mask rule and random-number
definition), never by a common helper.

Precision: float64 throughout; the sampling decision u < p uses float64 p.
"""
from . import philox, physics, network, sampler, estimator, markov, exact, muon, refine, overlap, patch  # noqa: F401
