"""Seeded synthetic grids, topology candidates and injection variants.

Input data only; shared by the solver tests, the benchmark and the CPU oracle.
"""
from .synth import (Grid, Candidates, Workload, KIND_OUTAGE, KIND_SPLIT, MAX_RANK,
                    MAX_SPLIT_DEGREE, make_grid, candidate_topology, is_connected,
                    non_bridges, random_split, sample_candidate, balanced,
                    perturbed_injections, busbar_injection_topologies, workload_tiny,
                    generator_outages, multi_outage_cases, attach_stubs,
                    workload_medium, workload_uneven, workload_brute)
