"""Seeded synthetic inputs shared by the contraction library's callers and the
CPU oracle: random circuits, the canonical network's wire structure, and a
greedy contraction-order finder with index slicing.  No tensor arithmetic."""
from .circuit import (Circuit, Gate, make_rqc, make_uneven_batch, uneven_circuit, random_bitstrings,
                      bits_to_index, near_square_grid, one_qubit_matrix, fsim_matrix,
                      cycle_patterns, pattern_edges)
from .network import NetworkStructure, network_structure
from .order import (greedy_order, slice_to_fit, order_stats, find_order, validate_order,
                    step_masks, live_peak, Plan, OrderStats, schroedinger_order)
