"""CPU oracle for the counter-guided search sweep.

TEST INFRASTRUCTURE ONLY.  Nothing in the product (the HIP library and its
Python binding) imports, calls or links anything here; only the tests, the
package's smoke check and the CPU-baseline leg of the benchmark do.

The oracle is a plain, slow, obviously correct restatement of the method of
"Using hardware performance counters to speed up autotuning convergence on
GPUs" (Filipovic et al.):

* ``space``    tuning-space enumeration and constraint pruning (Sect. 1, 3.7)
* ``forest``   decision-tree model evaluation (Sect. 3.4.2)
* ``score``    configuration score and normalisation (Sect. 3.6, score and
               score-normalisation equations)
* ``sampling`` score-weighted random draw with removal (Sect. 3.7, Alg. 1)
* ``expert``   bottleneck analysis and counter-change computation
               (Sect. 3.5, equations for b_DRAM ... b_paral and the FP32
               reaction rule)
* ``search``   one search step composed of the above
* ``mlp``      the multilayer-perceptron surrogate used in place of the tree
               model (an extension; plain float64 forward/backward/Adam)

Floating point is float64 for every quantity the paper defines.  Where a
floating-point value decides an integer (the quantised sampling weight), the
oracle additionally evaluates that chain in float32 with a fixed operation
order (``*_fp32`` functions), because the decision must be taken in the same
precision on both sides.
"""
