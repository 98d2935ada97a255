"""Plain FP64 CPU oracle for the D2Q9 lattice Boltzmann step with Zou & He and
neural outflow boundaries (Bedrunka et al., "Reduction of Outflow Boundary
Influence on Aerodynamic Performance using Neural Networks").

THIS PACKAGE IS TEST INFRASTRUCTURE.  Only ``tests/``, ``__graft_entry__.smoke``
and the ``cpu_baseline`` leg of ``bench.py`` may import it.  The product path
(``paper_2506_05293_amd``) never imports, calls or links anything here, and
nothing here imports the product path: the two share no code.  Inputs that both
sides consume (masks, seeds, case sizes) are built by the callers and passed in.

Every routine is a slow, direct transcription of a passage of the paper
(cited per function) or of a reading of it where the paper is silent; there is
no blocking, fusion or reordering beyond what the cited definition states.

Modules
  d2q9         lattice constants, equilibrium (Eq. 3), moments (Eq. 4),
               BGK (Eq. 2) and MRT collision (named in Sec. 3.2)
  zouhe        Zou & He velocity inlet / pressure outlet (Eqs. 5-11)
  solver       the time step: collide, momentum-exchange force (Eqs. 14-15),
               pull streaming with bounce-back (Eq. 1, Eq. 12 as half-way),
               boundary columns, neural outflow (Eq. 16)
  mlp          the outflow MLP: forward with BF16 emulation, FP64 backward,
               MSE loss (Eq. 17), Adam
  cbc          characteristic outflow (Sec. 4, Eqs. 18-29) and its tuning
               network (Sec. 4.2)
  cbc_train    closed-loop training of the tuning network (Sec. 4.2): the
               step re-expressed in torch FP64, segment loss over Omega_s,
               gradient by reverse-mode differentiation
  d3q19        the step carried to three dimensions (D3Q19, BGK, Zou & He
               faces with transverse corrections, half-way bounce-back,
               momentum exchange)
  splitmix64   the sequential SplitMix64 generator (Steele, Lea & Flood 2014)
  observables  drag/lift coefficients (Eq. 13) and the Strouhal number

The geometry masks (cylinder, NACA0012 of Eq. A.1) are inputs, built by the
product's input generators and pinned on their own by closed-form tests
(area, thickness, symmetry).

Parity status: every function here is pinned by a ``-m "not gpu"`` test in
``tests/test_oracle_*.py`` except where its docstring says "parity unpinned".
"""
