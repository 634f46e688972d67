import os
import sys

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)


def pytest_configure(config):
    config.addinivalue_line("markers", "gpu: needs an MI355X (runs through the C-ABI library)")
    config.addinivalue_line("markers", "slow: long CPU test")


@pytest.fixture(scope="session")
def oracle_mod():
    import oracle
    oracle.build_oracle(force=False)
    return oracle


def make_oracle(cfg, **kw):
    """An oracle set up with the standard species and tables of a config."""
    from oracle import Oracle
    from paper_2109_00214_amd import workload as W
    args = dict(enable_di=cfg.enable_di)
    args.update(kw)
    tables = args.pop("tables", None)
    o = Oracle(cfg.nr, cfg.nz, cfg.R, cfg.L, cfg.V, cfg.dt, cfg.weight, cfg.seed, **args)
    Z, m = W.species_table()
    o.set_species(Z, m)
    for ch, thr, dsq, sig in (tables or W.cross_section_tables()):
        o.set_cross_section(ch, thr, dsq, sig)
    return o
