"""CPU oracle (test infrastructure only): see lb_oracle for what it computes and why."""
