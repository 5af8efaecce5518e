"""On-the-fly statistical model checking of mass-action reaction networks on
AMD Instinct MI355X (Ballarini, Forlin, Mazza, Prandi, PDMC 2009).

The compute path is the HIP library libsmc.so (include/smc.h);
`paper_0912_2551_amd.binding` marshals arguments to it and
`paper_0912_2551_amd.workloads` builds seeded synthetic inputs.  The library
is loaded on first use, so importing the package never needs a GPU.
"""
