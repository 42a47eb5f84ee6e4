"""The synthetic workloads (lattice shapes of the paper's runs, seeded fields).

Each entry names the lattice ``dims = (T, L1, L2, L3)``, the field recipe
(``eps`` = 0 means unit links), the clover coefficient, the bare mass(es),
the alpha profile kind and alpha0 values, the residue, and the seed.
Time is antiperiodic for the fermions (``bc_t = -1``), space periodic.
"""

CONFIGS = {
    # free field, Wilson (c_sw = 0), checked against the momentum-space closed form
    "free_8c16": dict(dims=(16, 8, 8, 8), eps=0.0, csw=0.0, masses=(0.5,),
                      profile="exp", alpha0s=(0.4,), r=1e-11, seed=0),
    # interacting 16^3 x 32, FP64 GPU solve against the FP64 oracle; the heavy-
    # quark profile of the paper for (anti)periodic time, eq. pbcalpha
    "su3_16c32": dict(dims=(32, 16, 16, 16), eps=0.3, csw=1.6, masses=(0.5,),
                      profile="cosh", alpha0s=(0.0, 0.4), r=1e-11, seed=1632),
    # interacting 24^3 x 48, mixed precision (FP32 inner) against FP64
    "su3_24c48": dict(dims=(48, 24, 24, 24), eps=0.25, csw=1.6, masses=(0.5,),
                      profile="cosh", alpha0s=(0.4,), r=1e-11, seed=2448),
    # interacting 32^3 x 64, light mass, CGNR with FP16 storage
    "su3_32c64": dict(dims=(64, 32, 32, 32), eps=0.2, csw=1.6, masses=(0.01,),
                      profile="exp_sym", alpha0s=(0.0, 0.05, 0.1), r=1e-11, seed=3264),
}


def config(name):
    return dict(CONFIGS[name])
