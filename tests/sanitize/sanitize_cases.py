"""Inputs of the sanitizer test: circuits for the planner, invalid requests
for the validation, and small noisy circuits for the oracle."""
import workloads as W


def circuits():
    w3 = W.workload("c3_20q")
    w2 = W.workload("c2_16q")
    ad = W.noise_model([W.rule(["u3", "h"], W.amplitude_damping_kraus(0.1)),
                        W.rule(["cx", "cz"], W.depolarizing_pauli(0.1, 2))],
                       readout=(0.05, 0.02))
    cond = W.random_small(16, 300, seed=6, n_mid=8, p_cond=0.3)
    dense = W.random_dense(14, 40, seed=3)
    plans = {
        "c3_tile13": (w3["circuit"], w3["noise"], 13, 5),
        "c2_tile12": (w2["circuit"], w2["noise"], 12, 4),
        "cond_tile12": (cond, ad, 12, 4),
        "dense_tile13": (dense, ad, 13, 5),
        "c3_lds_sweeps": (w3["circuit"], w3["noise"], 13, 0),
    }
    good = W.random_small(3, 10, seed=1)
    bad_qubit = {"n_qubits": 3, "n_clbits": 0, "ops": [{"kind": "h", "qubits": [3]}]}
    dup_qubit = {"n_qubits": 3, "n_clbits": 0, "ops": [{"kind": "cx", "qubits": [1, 1]}]}
    bad_prob = W.noise_model([W.rule(["h"], W.pauli_table([0.5, 0.6], ["I", "X"]))])
    bad_kraus = W.noise_model([W.rule(["h"], W.kraus_channel([[[1, 0], [0, 0.5]]]))])
    invalid = {
        "qubit_out_of_range": (bad_qubit, None),
        "repeated_qubit": (dup_qubit, None),
        "probabilities": (good, bad_prob),
        "kraus_completeness": (good, bad_kraus),
        "not_attached": (good, ad),
    }
    small = W.random_small(4, 60, seed=9, n_mid=3, p_cond=0.3)
    oracle_cases = {
        "layered_noisy": (W.random_layered(5, 6, seed=2), w3["noise"], 64, 7),
        "mid_measure_conditional": (small, ad, 64, 3),
        "dense_channels": (W.random_dense(5, 12, seed=4), ad, 32, 1),
    }
    return {"plans": plans, "invalid": invalid, "oracle": oracle_cases}
