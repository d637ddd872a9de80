// Serving loop (server.cpp) behind the fem_server_* entry points.
#pragma once

#include <string>

#include "solver.hpp"

namespace femheat {

int server_create(const fem_server_opts& o, fem_server** out, std::string* err);
int server_submit(fem_server* s, const fem_request& q, uint64_t* ticket, std::string* err);
int server_poll(fem_server* s, uint64_t ticket, fem_status* st);
int server_wait(fem_server* s, uint64_t ticket, double timeout_s, fem_status* st);
int server_cancel(fem_server* s, uint64_t ticket);
int server_info(fem_server* s, fem_server_info* info);
void server_destroy(fem_server* s);

}  // namespace femheat
