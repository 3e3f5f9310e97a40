"""Plain FP64 CPU oracle for the data-annealed SMC sampler (test infrastructure).

This package is the checker, not the product.  Only the test-suite, the smoke
entry point and the benchmark's CPU-baseline leg may import it.  It shares no
code with the HIP path: it is written from the paper's equations in plain NumPy
float64, with no blocking, fusion or reordering beyond what the equations state.

Modules
-------
mlp        per-particle MLP log-likelihood and its hand-written gradient
           (Section 3, stochastic estimate; Section 4, image classification)
smc        initialisation, leapfrog/Langevin move, L-kernel weight update,
           normalisation, ESS, systematic resampling, posterior estimates
           (Section 2, Section 2.1)
schedules  the five naive data-annealing schedules (Section 3.1)
sda        smooth data annealing beta updates and weighted moments (Section 3.1)
learned    learned proposal-scale network, its Gaussian move density and its
           FP64 trainer (an extension: the paper's move uses a fixed step)
cnn        small convolutional model for the CIFAR-shaped workload
philox     Philox-4x32-10 counter-based generator (Salmon et al., SC'11)
blr        exact posterior of Bayesian linear regression (closed-form pin)
"""
