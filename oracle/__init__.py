"""FP64 CPU oracle of the look-ahead decentralized particle filter.

TEST INFRASTRUCTURE ONLY.  Nothing in the product path (the HIP library and
its Python binding) imports, calls or links anything here; only the tests,
the smoke check and the CPU-baseline leg of the benchmark do.

The oracle is a plain, slow, readable restatement of the method of
Ahmed, Bibalan, de Freitas and Fauvel, "Decentralized, Adaptive, Look-Ahead
Particle Filtering" (arXiv:1203.2394):

* ``philox``   -- the counter-based generator both sides implement from its
                  published definition (Salmon et al., SC'11), plus the
                  uniform / normal transforms of the random-number contract.
* ``models``   -- the nested state-space model of Section 2, Eq. (1):
                  samplers of the transitions and the log densities.
* ``resample`` -- systematic resampling ("standard resampling", Section 2).
* ``ladpf``    -- one step of the look-ahead DPF (Section 2.2, Fig. 4).
* ``dpf``      -- one step of the plain DPF (Section 2, Fig. 2).
* ``learned``  -- the learned mixture-density proposal and its training
                  (forward, backward, Adam) and the learned step.
* ``kalman``   -- closed-form Kalman filters used to pin the oracle.

Everything is float64 except where a step reproduces a stated FP32 contract
(the random-number transforms are exact in both precisions).
"""
